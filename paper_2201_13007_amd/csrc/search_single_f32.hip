// The single-worker search kernels (search_single.h) for float32 vector storage.
#include "search_single.h"

namespace sa {

int launch_search_single_f32(const search_detail::KArgs &A, int64_t nq, hipStream_t s)
{
    return single_detail::launch_dt<SA_F32>(A, nq, s);
}

}  // namespace sa
