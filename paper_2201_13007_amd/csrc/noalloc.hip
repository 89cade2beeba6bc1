// sa_search_noalloc: the search of sa_search with its workspace in a static device array
// of the library, for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid it).  Contract in include/speedann.h.
#include "sa_internal.h"

#include <mutex>

namespace sa {
namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // per device
constexpr int MAX_DEVICES = 64;

// The workspace of every sa_search_noalloc call on a device: each device holds its own
// copy from the library's load to the end of the process.  Host code never takes the
// address of this name (on the host it is a stand-in, not a device address); it uses
// the address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEVICES];   // device address of scratch, per device
bool g_cleared[MAX_DEVICES];    // its zero fill is enqueued

__global__ void zero_fill(uint4 *p, size_t n)
{
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = z;
}

// The current device's scratch address (looked up once per device, with that device
// current); on the first call for a device a zero fill of the whole array is enqueued on
// s, ahead of the search that follows it.
int device_scratch(hipStream_t s, void **out)
{
    int dev = 0;
    SA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(SA_EUNSUPPORTED, "device %d: at most %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255u) != 0) return set_error(SA_EHIP, "scratch array at a bad address %p", p);
        g_scratch[dev] = p;
    }
    if (!g_cleared[dev]) {
        hipLaunchKernelGGL(zero_fill, dim3(1024), dim3(256), 0, s, static_cast<uint4 *>(g_scratch[dev]),
                           SCRATCH_BYTES / sizeof(uint4));
        SA_HIP(hipGetLastError());
        g_cleared[dev] = true;
    }
    *out = g_scratch[dev];
    return SA_OK;
}

}  // namespace
}  // namespace sa

using namespace sa;

extern "C" {

int sa_search_noalloc(const sa_index *index, const float *queries_dev, int64_t nq, int64_t ldq, int32_t k, int32_t L,
                      int32_t M, const sa_search_params *params, int32_t *ids_dev, float *dists_dev,
                      sa_query_stats *stats_dev, void *hip_stream)
{
    sa_search_params p;
    if (params) p = *params;
    else sa_default_params(&p);
    int rc;
    if ((rc = check_search(index, nq, k, L, M, p)) != SA_OK) return rc;
    const size_t need = sa_search_workspace_bytes(index, nq, k, L, M, &p);
    if (need > SCRATCH_BYTES)
        return set_error(SA_ECAPACITY,
                         "sa_search_noalloc: nq=%lld, L=%d, M=%d need %zu bytes of scratch; its size is %zu "
                         "(search fewer queries per call, or use sa_search with a workspace)",
                         (long long)nq, L, M, need, SCRATCH_BYTES);
    if ((rc = check_device()) != SA_OK) return rc;
    void *ws = nullptr;
    if ((rc = device_scratch((hipStream_t)hip_stream, &ws)) != SA_OK) return rc;
    return sa_search(index, queries_dev, nq, ldq, k, L, M, &p, ids_dev, dists_dev, stats_dev, ws, SCRATCH_BYTES,
                     hip_stream);
}

}  // extern "C"
