// Vertex renumbering of an index (the GPU counterpart of the neighbour grouping of
// Sec. 4.4: vertices a search meets together are stored together), the permutation of
// vectors and adjacency rows into the new order, and the mapping of result ids back to
// the original numbering.  Contracts are in include/speedann.h.
//
// The order itself is an offline step: the in-degree histogram is counted on the GPU,
// the sort and the breadth-first walk run on the host over a copy of the adjacency.
#include "sa_internal.h"

#include <algorithm>
#include <numeric>
#include <vector>

namespace sa {
namespace {

__global__ void indegree_kernel(const int32_t *adj, int64_t total, int64_t n, int32_t *deg)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = adj[i];
        if (u >= 0 && u < n) atomicAdd(deg + u, 1);
    }
}

// dst row i = src row perm[i]; rows of w 32-bit words, one block per row
__global__ void permute_rows_kernel(const uint32_t *src, int64_t n, int64_t w, const int32_t *perm, uint32_t *dst)
{
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int32_t p = perm[i];
        uint32_t *t = dst + i * w;
        if (p < 0 || p >= n) {   // not a permutation entry: the row is zeroed
            for (int64_t c = threadIdx.x; c < w; c += blockDim.x) t[c] = 0u;
            continue;
        }
        const uint32_t *s = src + (int64_t)p * w;
        for (int64_t c = threadIdx.x; c < w; c += blockDim.x) t[c] = s[c];
    }
}

__global__ void inverse_kernel(const int32_t *perm, int64_t n, int32_t *inv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (perm[i] >= 0 && perm[i] < n) inv[perm[i]] = (int32_t)i;
}

// adj_out row i = adj row perm[i] with every id u replaced by inv[u] (-1 stays -1)
__global__ void permute_graph_kernel(const int32_t *adj, int64_t n, int32_t R, const int32_t *perm, const int32_t *inv,
                                     int32_t *out)
{
    const int64_t total = n * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / R;
        const int32_t j = (int32_t)(e - i * R);
        const int32_t p = perm[i];
        const int32_t u = (p >= 0 && p < n) ? adj[(int64_t)p * R + j] : -1;
        out[e] = (u >= 0 && u < n) ? inv[u] : -1;
    }
}

// ids of job b's query (order[b], or b) are its first k (qk[q], or k) entries of row q
__global__ void map_ids_kernel(int32_t *ids, int64_t ldo, int64_t njobs, int32_t k, const int32_t *order,
                               const int32_t *qk, const int32_t *id_map, int64_t n)
{
    const int64_t job = blockIdx.x;
    if (job >= njobs) return;
    const int64_t q = order ? order[job] : job;
    const int kq = qk ? qk[q] : k;
    for (int p = threadIdx.x; p < kq; p += blockDim.x) {
        const int32_t v = ids[q * ldo + p];
        if (v >= 0 && v < n) ids[q * ldo + p] = id_map[v];
    }
}

unsigned grid_for(int64_t work, int block)
{
    const int64_t g = (work + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

int launch_map_ids(int32_t *ids, int64_t ldo, int64_t njobs, int32_t k, const int32_t *order, const int32_t *qk,
                   const int32_t *id_map, int64_t n, hipStream_t s)
{
    if (njobs == 0) return SA_OK;
    hipLaunchKernelGGL(map_ids_kernel, dim3((unsigned)njobs), dim3(64), 0, s, ids, ldo, njobs, k, order, qk, id_map, n);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

}  // namespace sa

using namespace sa;

extern "C" {

int sa_graph_order(const int32_t *adj_dev, int64_t n, int32_t R, int32_t entry, int32_t mode, int32_t *perm_dev,
                   void *hip_stream)
{
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [1, 2^31)");
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (!adj_dev || !perm_dev) return set_error(SA_EINVAL, "NULL argument");
    if (mode != SA_ORDER_DEGREE && mode != SA_ORDER_BFS) return set_error(SA_EINVAL, "unknown order mode %d", mode);
    if (mode == SA_ORDER_BFS && (entry < 0 || entry >= n)) return set_error(SA_EINVAL, "entry out of range");
    int rc;
    if ((rc = check_device()) != SA_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<int32_t> perm(n);
    if (mode == SA_ORDER_DEGREE) {
        int32_t *deg = nullptr;
        SA_HIP(hipMallocAsync(reinterpret_cast<void **>(&deg), 4 * (size_t)n, s));
        hipError_t e = hipMemsetAsync(deg, 0, 4 * (size_t)n, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(indegree_kernel, dim3(grid_for(n * R, 256)), dim3(256), 0, s, adj_dev, n * R, n, deg);
            e = hipGetLastError();
        }
        std::vector<int32_t> dh(n);
        if (e == hipSuccess) e = hipMemcpyAsync(dh.data(), deg, 4 * (size_t)n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFreeAsync(deg, s);
        if (e != hipSuccess) return hip_fail(e, "in-degree count");
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return dh[a] > dh[b]; });
    } else {
        std::vector<int32_t> ah((size_t)n * R);
        SA_HIP(hipMemcpyAsync(ah.data(), adj_dev, 4 * (size_t)n * R, hipMemcpyDeviceToHost, s));
        SA_HIP(hipStreamSynchronize(s));
        std::vector<uint8_t> seen(n, 0);
        int64_t tail = 0;
        perm[tail++] = entry;
        seen[entry] = 1;
        for (int64_t head = 0; head < tail; ++head) {
            const int32_t *row = ah.data() + (size_t)perm[head] * R;
            for (int j = 0; j < R; ++j) {
                const int32_t u = row[j];
                if (u >= 0 && u < n && !seen[u]) {
                    seen[u] = 1;
                    perm[tail++] = u;
                }
            }
        }
        for (int64_t v = 0; v < n; ++v)
            if (!seen[v]) perm[tail++] = (int32_t)v;
    }
    SA_HIP(hipMemcpyAsync(perm_dev, perm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s));
    SA_HIP(hipStreamSynchronize(s));
    return SA_OK;
}

int sa_permute_rows(const void *src_dev, int64_t n, int64_t row_bytes, const int32_t *perm_dev, void *dst_dev,
                    void *hip_stream)
{
    if (n < 0 || row_bytes <= 0 || row_bytes % 4 != 0) return set_error(SA_EINVAL, "row_bytes must be a positive multiple of 4");
    if (n > 0 && (!src_dev || !perm_dev || !dst_dev)) return set_error(SA_EINVAL, "NULL argument");
    if (src_dev == dst_dev && n > 0) return set_error(SA_EINVAL, "src and dst must not be the same buffer");
    int rc;
    if ((rc = check_device()) != SA_OK) return rc;
    if (n == 0) return SA_OK;
    hipLaunchKernelGGL(permute_rows_kernel, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(128), 0,
                       (hipStream_t)hip_stream, static_cast<const uint32_t *>(src_dev), n, row_bytes / 4, perm_dev,
                       static_cast<uint32_t *>(dst_dev));
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int sa_permute_graph(const int32_t *adj_dev, int64_t n, int32_t R, const int32_t *perm_dev, int32_t *inv_dev,
                     int32_t *adj_out_dev, void *hip_stream)
{
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [1, 2^31)");
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (!adj_dev || !perm_dev || !inv_dev || !adj_out_dev) return set_error(SA_EINVAL, "NULL argument");
    if (adj_dev == adj_out_dev) return set_error(SA_EINVAL, "adj and adj_out must not be the same buffer");
    int rc;
    if ((rc = check_device()) != SA_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(inverse_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, perm_dev, n, inv_dev);
    SA_HIP(hipGetLastError());
    hipLaunchKernelGGL(permute_graph_kernel, dim3(grid_for(n * R, 256)), dim3(256), 0, s, adj_dev, n, R, perm_dev,
                       inv_dev, adj_out_dev);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int sa_index_set_id_map(sa_index *index, const int32_t *id_map_dev)
{
    if (!index) return set_error(SA_EINVAL, "index is NULL");
    index->id_map = id_map_dev;
    return SA_OK;
}

}  // extern "C"
