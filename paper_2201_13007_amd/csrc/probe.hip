// Gather ceiling: the bandwidth that random whole-row gathers of vectors reach on this
// GPU, the access pattern of the search's distance step (rows spread over the whole
// array, lanes of a group reading one row's consecutive 16-byte chunks, loads issued
// unconditionally).  A measurement tool beside the search, not part of it.
#include "search_body.h"

namespace sa {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    // a 32-bit integer hash (xorshift-multiply rounds)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Every wavefront gathers `iters` passes of 64 / LPV random rows, four passes in flight,
// and folds what it read into one float per lane so that no load is dead.
template <int LPV>
__global__ void __launch_bounds__(256) gather_probe_kernel(const float *vec, int64_t n, int d, int64_t ld,
                                                           int64_t iters, uint32_t seed, float *sink)
{
    constexpr int U = 4;
    const int lane = __lane_id(), grp = lane / LPV, g = lane % LPV;
    const uint32_t wave = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int nch = d >> 2;
    float acc[U] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; it += U) {
        float4 x[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t h = mix32(seed ^ mix32(wave * 0x9e3779b9u + (uint32_t)(it + u) * 0x85ebca6bu + grp));
            const int64_t row = (int64_t)(h % (uint32_t)n);
            const float4 *p = reinterpret_cast<const float4 *>(vec + row * ld);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = g + LPV * i;
                x[u][i] = p[c < nch ? c : 0];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (g + LPV * i < nch) acc[u] += x[u][i].x + x[u][i].y + x[u][i].z + x[u][i].w;
    }
    sink[(size_t)wave * 64 + lane] = acc[0] + acc[1] + acc[2] + acc[3];
}

template <int LPV>
hipError_t launch_probe(const float *vec, int64_t n, int d, int64_t ld, int64_t iters, int waves, uint32_t seed,
                        float *sink, hipStream_t s)
{
    hipLaunchKernelGGL(gather_probe_kernel<LPV>, dim3((unsigned)(waves / 4)), dim3(256), 0, s, vec, n, d, ld, iters,
                       seed, sink);
    return hipGetLastError();
}

}  // namespace
}  // namespace sa

using namespace sa;

extern "C" int sa_gather_probe(const float *vec_dev, int64_t n, int32_t d, int64_t ld, int64_t iters, int32_t waves,
                               uint32_t seed, float *sink_dev, void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(vec_dev, n, d, ld, "vectors")) != SA_OK) return rc;
    if (n < 1 || n > 0xFFFFFFFFll) return set_error(SA_EINVAL, "n must be in [1, 2^32)");
    if (d > 1024) return set_error(SA_EUNSUPPORTED, "d=%d exceeds 1024", d);
    if (iters < 4 || iters % 4 != 0) return set_error(SA_EINVAL, "iters must be a positive multiple of 4");
    if (waves < 4 || waves % 4 != 0) return set_error(SA_EINVAL, "waves must be a positive multiple of 4");
    if (!sink_dev) return set_error(SA_EINVAL, "sink is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e;
    switch (search_detail::lanes_per_vector(d)) {
    case 1: e = launch_probe<1>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    case 2: e = launch_probe<2>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    case 4: e = launch_probe<4>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    case 8: e = launch_probe<8>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    case 16: e = launch_probe<16>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    case 32: e = launch_probe<32>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    default: e = launch_probe<64>(vec_dev, n, d, ld, iters, waves, seed, sink_dev, s); break;
    }
    if (e != hipSuccess) return hip_fail(e, "gather probe launch");
    return SA_OK;
}
