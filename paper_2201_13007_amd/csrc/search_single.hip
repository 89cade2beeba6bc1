// Search kernels with one worker (M = 1): Algorithm 1 run as Algorithm 3 with T = 1.
// One 64-lane workgroup per query; see search_body.h.
#include "search_body.h"

namespace sa {
namespace search_detail {

template <int LPV, int CPL, int NI>
__global__ void __launch_bounds__(64) search_single(KArgs A)
{
    search_body<LPV, CPL, NI, false>(A);
}

template <int LPV, int CPL, int NI>
hipError_t launch1(const KArgs &A, int64_t nq, uint32_t lds, hipStream_t s)
{
    auto k = search_single<LPV, CPL, NI>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)nq), dim3(64), lds, s, A);
    return hipGetLastError();
}

template <int LPV, int CPL>
hipError_t launch1_ni(const KArgs &A, int64_t nq, uint32_t lds, hipStream_t s)
{
    const int ni = (A.L + 63) / 64;
    if (ni <= 1) return launch1<LPV, CPL, 1>(A, nq, lds, s);
    if (ni <= 2) return launch1<LPV, CPL, 2>(A, nq, lds, s);
    if (ni <= 4) return launch1<LPV, CPL, 4>(A, nq, lds, s);
    if (ni <= 6) return launch1<LPV, CPL, 6>(A, nq, lds, s);
    if (ni <= 8) return launch1<LPV, CPL, 8>(A, nq, lds, s);
    return launch1<LPV, CPL, 16>(A, nq, lds, s);
}

}  // namespace search_detail

int launch_search_single(const search_detail::KArgs &A, int64_t nq, uint32_t lds, hipStream_t s)
{
    using namespace search_detail;
    const int nch = A.d / 4;
    hipError_t e;
    if (nch <= 8) e = launch1_ni<8, 1>(A, nq, lds, s);
    else if (nch <= 16) e = launch1_ni<16, 1>(A, nq, lds, s);
    else if (nch <= 32) e = launch1_ni<32, 1>(A, nq, lds, s);
    else if (nch <= 64) e = launch1_ni<64, 1>(A, nq, lds, s);
    else if (nch <= 128) e = launch1_ni<64, 2>(A, nq, lds, s);
    else e = launch1_ni<64, 4>(A, nq, lds, s);
    if (e != hipSuccess) return hip_fail(e, "search kernel launch");
    return SA_OK;
}

}  // namespace sa
