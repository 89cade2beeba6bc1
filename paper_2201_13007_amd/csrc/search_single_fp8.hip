// The single-worker search kernels (search_single.h) for fp8 e4m3 vector storage.
#include "search_single.h"

namespace sa {

int launch_search_single_fp8(const search_detail::KArgs &A, int64_t nq, hipStream_t s)
{
    return single_detail::launch_dt<SA_FP8E4M3>(A, nq, s);
}

}  // namespace sa
