// C ABI of libspeedann: argument validation, error strings, and the calls that string
// the kernels together.  Declarations and their contracts are in include/speedann.h.
#include "sa_internal.h"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

namespace sa {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return set_error(SA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int medoid_device(const float *base, int64_t n, int d, int64_t ld, int32_t *out, hipStream_t s);
int prune_device(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *cand, int kc, int R,
                 int mode, int32_t *adj, hipStream_t s);
int repair_device(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj_dev, int R,
                  int32_t entry, int keep_local, int hubs, int hub_keep_local, int64_t *bridges_out,
                  int64_t *ncomp_out, hipStream_t s);
int reverse_edges_device(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj_dev, int R,
                         int64_t *added_out, hipStream_t s);

int check_device()
{
    static int cached = 0;   // 0 unknown, 1 ok, negative error
    if (cached == 1) return SA_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(SA_EUNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev,
                         prop.gcnArchName);
    cached = 1;
    return SA_OK;
}

int check_matrix(const void *p, int64_t rows, int32_t d, int64_t ld, const char *name)
{
    if (rows < 0) return set_error(SA_EINVAL, "%s: negative row count", name);
    if (rows > 0 && p == nullptr) return set_error(SA_EINVAL, "%s is NULL", name);
    if (d < 4 || d % 4 != 0 || d > 4096)
        return set_error(SA_EINVAL, "%s: d=%d must be a multiple of 4 in [4, 4096] (pad with zeros)", name, d);
    if (ld < d || ld % 4 != 0) return set_error(SA_EINVAL, "%s: row stride %lld must be >= d and a multiple of 4", name, (long long)ld);
    if (((uintptr_t)p & 15u) != 0) return set_error(SA_EINVAL, "%s must be 16-byte aligned", name);
    return SA_OK;
}

int check_search(const sa_index *ix, int64_t nq, int32_t k, int32_t L, int32_t M, const sa_search_params &p)
{
    if (!ix) return set_error(SA_EINVAL, "index is NULL");
    if (nq < 0 || nq > 0x7FFFFFFF) return set_error(SA_EINVAL, "nq=%lld out of range", (long long)nq);
    if (k < 1 || L < k || L > 1024) return set_error(SA_EINVAL, "need 1 <= k <= L <= 1024 (k=%d, L=%d)", k, L);
    if (M < 1 || M > 16) return set_error(SA_EINVAL, "M=%d must be in [1, 16]", M);
    if (p.sync < SA_SYNC_BSP || p.sync > SA_SYNC_ADAPTIVE) return set_error(SA_EINVAL, "unknown sync %d", p.sync);
    if (!(p.rho >= 0.0f) || !std::isfinite(p.rho)) return set_error(SA_EINVAL, "rho must be finite and >= 0");
    if (p.max_substeps < 0) return set_error(SA_EINVAL, "max_substeps must be >= 0");
    if (p.rerank < -1) return set_error(SA_EINVAL, "rerank=%d must be -1, 0 or positive", p.rerank);
    if (p.rerank != 0 && !ix->vec32) return set_error(SA_EINVAL, "re-rank needs the index's float32 vectors");
    return SA_OK;
}

}  // namespace sa

using namespace sa;

extern "C" {

const char *sa_last_error(void) { return g_last_error.c_str(); }

void sa_default_params(sa_search_params *out)
{
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->sync = SA_SYNC_ADAPTIVE;
    out->static_I = 0;
    out->rho = 0.8;
    out->staged = 1;
}

int sa_knn_ex(const float *base_dev, int64_t n, int32_t d, int64_t ld, const float *queries_dev, int64_t nq,
              int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids_dev, float *dists_dev,
              int32_t path, int32_t *path_used_out, void *hip_stream)
{
    int rc;
    if (path_used_out) *path_used_out = SA_KNN_AUTO;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if ((rc = check_matrix(queries_dev, nq, d, ldq, "queries")) != SA_OK) return rc;
    if (n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be < 2^31");
    if (k < 1 || k > 256) return set_error(SA_EINVAL, "k=%d must be in [1, 256]", k);
    if (metric != SA_L2 && metric != SA_IP) return set_error(SA_EINVAL, "unknown metric %d", metric);
    if (nq > 0 && (ids_dev == nullptr || dists_dev == nullptr)) return set_error(SA_EINVAL, "output is NULL");
    if (exclude_self && nq > n) return set_error(SA_EINVAL, "exclude_self needs the queries to be base rows");
    if (path != SA_KNN_AUTO && path != SA_KNN_SCAN && path != SA_KNN_MFMA)
        return set_error(SA_EINVAL, "unknown kNN path %d", path);
    if ((rc = check_device()) != SA_OK) return rc;
    return launch_knn(base_dev, n, d, ld, queries_dev, nq, ldq, k, metric, exclude_self, ids_dev, dists_dev, path,
                      path_used_out, (hipStream_t)hip_stream);
}

int64_t sa_knn_last_rescanned(void) { return knn_rescanned; }

int sa_index_analyze(sa_index *index, void *hip_stream)
{
    if (!index) return set_error(SA_EINVAL, "index is NULL");
    index->int_lo = 1;
    index->int_hi = 0;
    if (index->dtype != SA_F32) return SA_OK;
    int rc;
    if ((rc = check_device()) != SA_OK) return rc;
    SA_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    return index_integer_range(static_cast<const float *>(index->codes), index->n, index->d, index->ldc, &index->int_lo,
                               &index->int_hi);
}

int32_t sa_index_integer_range(const sa_index *index, int32_t *lo, int32_t *hi)
{
    if (!index || index->int_lo > index->int_hi) return 0;
    if (lo) *lo = index->int_lo;
    if (hi) *hi = index->int_hi;
    return 1;
}

int sa_knn(const float *base_dev, int64_t n, int32_t d, int64_t ld, const float *queries_dev, int64_t nq, int64_t ldq,
           int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids_dev, float *dists_dev, void *hip_stream)
{
    return sa_knn_ex(base_dev, n, d, ld, queries_dev, nq, ldq, k, metric, exclude_self, ids_dev, dists_dev,
                     SA_KNN_AUTO, nullptr, hip_stream);
}

int sa_medoid(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t *entry_out, void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if (n < 1) return set_error(SA_EINVAL, "n must be >= 1");
    if (!entry_out) return set_error(SA_EINVAL, "entry_out is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    return medoid_device(base_dev, n, d, ld, entry_out, (hipStream_t)hip_stream);
}

int sa_prune(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, const int32_t *cand_dev,
             int32_t kc, int32_t R, int32_t prune, int32_t *adj_dev, void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if (kc < 1 || kc > 64) return set_error(SA_EINVAL, "candidate list width %d must be in [1, 64]", kc);
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (prune != 0 && prune != 1) return set_error(SA_EINVAL, "prune must be 0 or 1");
    if (metric != SA_L2 && metric != SA_IP) return set_error(SA_EINVAL, "unknown metric %d", metric);
    if (n > 0 && (!cand_dev || !adj_dev)) return set_error(SA_EINVAL, "NULL candidate or adjacency array");
    if ((rc = check_device()) != SA_OK) return rc;
    return prune_device(base_dev, n, d, ld, metric, cand_dev, kc, R, prune, adj_dev, (hipStream_t)hip_stream);
}

int sa_repair(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t *adj_dev, int32_t R,
              int32_t entry, int32_t keep_local, int32_t hubs, int32_t hub_keep_local, int64_t *bridges_out,
              int64_t *components_out, void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [1, 2^31)");
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (entry < 0 || entry >= n) return set_error(SA_EINVAL, "entry %d out of range", entry);
    if (keep_local < 0 || keep_local > R) return set_error(SA_EINVAL, "keep_local must be in [0, R]");
    if (hub_keep_local < 0 || hub_keep_local > R) return set_error(SA_EINVAL, "hub_keep_local must be in [0, R]");
    if (hubs < 0) return set_error(SA_EINVAL, "hubs must be >= 0");
    if (!adj_dev) return set_error(SA_EINVAL, "adjacency is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    return repair_device(base_dev, n, d, ld, metric, adj_dev, R, entry, keep_local, hubs, hub_keep_local, bridges_out,
                         components_out, (hipStream_t)hip_stream);
}

int sa_reverse_edges(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t *adj_dev,
                     int32_t R, int64_t *added_out, void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [1, 2^31)");
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (metric != SA_L2 && metric != SA_IP) return set_error(SA_EINVAL, "unknown metric %d", metric);
    if (!adj_dev) return set_error(SA_EINVAL, "adjacency is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    return reverse_edges_device(base_dev, n, d, ld, metric, adj_dev, R, added_out, (hipStream_t)hip_stream);
}

int sa_build_graph(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t knn_k, int32_t R,
                   int32_t prune, int32_t repair, int32_t keep_local, int32_t hubs, int32_t hub_keep_local,
                   int32_t *adj_dev, int32_t *entry_out, int64_t *bridges_out, int64_t *components_out,
                   void *hip_stream)
{
    int rc;
    if ((rc = check_matrix(base_dev, n, d, ld, "base")) != SA_OK) return rc;
    if (n < 2 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [2, 2^31)");
    if (knn_k < 1 || knn_k > 64) return set_error(SA_EINVAL, "knn_k=%d must be in [1, 64]", knn_k);
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (!adj_dev || !entry_out) return set_error(SA_EINVAL, "NULL output");
    if (keep_local < 0 || keep_local > R || hub_keep_local < 0 || hub_keep_local > R || hubs < 0)
        return set_error(SA_EINVAL, "keep_local and hub_keep_local must be in [0, R], hubs >= 0");
    if ((rc = check_device()) != SA_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = medoid_device(base_dev, n, d, ld, entry_out, s)) != SA_OK) return rc;
    int32_t *cand = nullptr;
    float *cd = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&cand), sizeof(int32_t) * n * knn_k) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&cd), sizeof(float) * n * knn_k) != hipSuccess) {
        if (cand) (void)hipFree(cand);
        return set_error(SA_ENOMEM, "build_graph: candidate lists do not fit");
    }
    rc = launch_knn(base_dev, n, d, ld, base_dev, n, ld, knn_k, metric, 1, cand, cd, SA_KNN_AUTO, nullptr, s);
    if (rc == SA_OK) rc = prune_device(base_dev, n, d, ld, metric, cand, knn_k, R, prune, adj_dev, s);
    if (rc == SA_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "build_graph");
    }
    (void)hipFree(cand);
    (void)hipFree(cd);
    if (bridges_out) *bridges_out = 0;
    if (components_out) *components_out = 0;
    if (rc == SA_OK && repair) rc = reverse_edges_device(base_dev, n, d, ld, metric, adj_dev, R, nullptr, s);
    if (rc == SA_OK && repair)
        rc = repair_device(base_dev, n, d, ld, metric, adj_dev, R, *entry_out, keep_local, hubs, hub_keep_local,
                           bridges_out, components_out, s);
    return rc;
}

int sa_index_create_q(const void *codes_dev, int32_t dtype, const float *scale_dev, int64_t ldc,
                      const float *vec32_dev, int64_t ld32, int64_t n, int32_t d, int32_t metric,
                      const int32_t *adj_dev, int32_t R, int32_t entry, sa_index **out)
{
    int rc;
    if (!out) return set_error(SA_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != SA_F32 && dtype != SA_BF16 && dtype != SA_FP8E4M3) return set_error(SA_EINVAL, "unknown dtype %d", dtype);
    if ((rc = check_matrix(codes_dev, n, d, ldc, "vectors")) != SA_OK) return rc;
    if (dtype == SA_FP8E4M3 && !scale_dev) return set_error(SA_EINVAL, "fp8 vectors need their scales");
    if (vec32_dev && (rc = check_matrix(vec32_dev, n, d, ld32, "float32 vectors")) != SA_OK) return rc;
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(SA_EINVAL, "n must be in [1, 2^31)");
    if (R < 1 || R > 64) return set_error(SA_EINVAL, "R=%d must be in [1, 64]", R);
    if (entry < 0 || entry >= n) return set_error(SA_EINVAL, "entry %d out of range [0, %lld)", entry, (long long)n);
    if (metric != SA_L2 && metric != SA_IP) return set_error(SA_EINVAL, "unknown metric %d", metric);
    if (!adj_dev) return set_error(SA_EINVAL, "adjacency is NULL");
    sa_index *ix = new (std::nothrow) sa_index;
    if (!ix) return set_error(SA_ENOMEM, "out of host memory");
    ix->codes = codes_dev; ix->scale = scale_dev; ix->ldc = ldc; ix->dtype = dtype;
    ix->vec32 = vec32_dev; ix->ld32 = vec32_dev ? ld32 : 0;
    ix->n = n; ix->d = d; ix->metric = metric;
    ix->adj = adj_dev; ix->R = R; ix->entry = entry;
    *out = ix;
    return SA_OK;
}

int sa_index_create(const float *vec_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, const int32_t *adj_dev,
                    int32_t R, int32_t entry, sa_index **out)
{
    return sa_index_create_q(vec_dev, SA_F32, nullptr, ld, vec_dev, ld, n, d, metric, adj_dev, R, entry, out);
}

int sa_quantize(const float *x_dev, int64_t n, int32_t d, int64_t ld, int32_t dtype, void *codes_dev, int64_t ldc,
                float *scale_dev, void *hip_stream)
{
    int rc;
    if (dtype != SA_BF16 && dtype != SA_FP8E4M3) return set_error(SA_EINVAL, "dtype %d: quantize to bf16 or fp8", dtype);
    if ((rc = check_matrix(x_dev, n, d, ld, "vectors")) != SA_OK) return rc;
    if ((rc = check_matrix(codes_dev, n, d, ldc, "codes")) != SA_OK) return rc;
    if (n > 0 && !scale_dev) return set_error(SA_EINVAL, "scale is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    return launch_quantize(x_dev, n, d, ld, dtype, codes_dev, ldc, scale_dev, (hipStream_t)hip_stream);
}

void sa_index_destroy(sa_index *index) { delete index; }


size_t sa_search_workspace_bytes(const sa_index *index, int64_t nq, int32_t k, int32_t L, int32_t M,
                                 const sa_search_params *params)
{
    sa_search_params p;
    if (params) p = *params;
    else sa_default_params(&p);
    if (check_search(index, nq, k, L, M, p) != SA_OK) return 0;
    return search_workspace_bytes(nq, L, M, p, index->R);
}

int sa_search(const sa_index *index, const float *queries_dev, int64_t nq, int64_t ldq, int32_t k, int32_t L,
              int32_t M, const sa_search_params *params, int32_t *ids_dev, float *dists_dev,
              sa_query_stats *stats_dev, void *workspace, size_t ws_bytes, void *hip_stream)
{
    sa_search_params p;
    if (params) p = *params;
    else sa_default_params(&p);
    int rc;
    if ((rc = check_search(index, nq, k, L, M, p)) != SA_OK) return rc;
    if ((rc = check_matrix(queries_dev, nq, index->d, ldq, "queries")) != SA_OK) return rc;
    if (nq > 0 && (!ids_dev || !dists_dev)) return set_error(SA_EINVAL, "output is NULL");
    if ((rc = check_device()) != SA_OK) return rc;
    SearchLaunch a;
    a.codes = index->codes; a.scale = index->scale; a.ldc = index->ldc; a.dtype = index->dtype;
    a.vec32 = index->vec32; a.ld32 = index->ld32;
    a.n = index->n; a.d = index->d; a.metric = index->metric;
    a.adj = index->adj; a.R = index->R; a.entry = index->entry; a.id_map = index->id_map;
    a.int_lo = index->int_lo; a.int_hi = index->int_hi;
    a.queries = queries_dev; a.ldq = ldq; a.nq = nq; a.k = k; a.L = L; a.M = M; a.p = p;
    a.ids = ids_dev; a.dists = dists_dev; a.stats = stats_dev; a.workspace = workspace; a.ws_bytes = ws_bytes;
    return launch_search(a, (hipStream_t)hip_stream);
}

}  // extern "C"
