// The general search kernels (search_multi.h) for float32 vector storage.
#include "search_multi.h"

namespace sa {

int launch_search_multi_f32(const search_detail::KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s)
{
    return search_detail::launch_dt<SA_F32>(A, nq, M, lds, s);
}

}  // namespace sa
