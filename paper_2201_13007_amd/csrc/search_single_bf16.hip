// The single-worker search kernels (search_single.h) for bfloat16 vector storage.
#include "search_single.h"

namespace sa {

int launch_search_single_bf16(const search_detail::KArgs &A, int64_t nq, hipStream_t s)
{
    return single_detail::launch_dt<SA_BF16>(A, nq, s);
}

}  // namespace sa
