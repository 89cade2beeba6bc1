// Internal declarations shared by the HIP sources of libspeedann (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/speedann.h"

namespace sa {

// ---------------------------------------------------------------- errors (host)

int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define SA_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

// ---------------------------------------------------------------- keys
// A list entry is the 64-bit key (ordered distance bits << 32 | id).  Ordering the
// keys as unsigned integers orders entries by (distance, id): the float-to-unsigned map
// below is monotone over all non-NaN floats, and -0 is folded into +0 first so that
// equal distances compare equal and fall through to the id.

constexpr uint64_t KEY_EMPTY = ~0ull;

__host__ __device__ inline uint32_t float_to_ordered(float f)
{
    if (f == 0.0f) f = 0.0f;
    uint32_t b;
    __builtin_memcpy(&b, &f, 4);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__host__ __device__ inline float ordered_to_float(uint32_t o)
{
    uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

__host__ __device__ inline uint64_t make_key(float dist, int32_t id)
{
    return ((uint64_t)float_to_ordered(dist) << 32) | (uint32_t)id;
}

__host__ __device__ inline int32_t key_id(uint64_t k) { return (int32_t)(uint32_t)(k & 0xFFFFFFFFu); }
__host__ __device__ inline float key_dist(uint64_t k) { return ordered_to_float((uint32_t)(k >> 32)); }

// ---------------------------------------------------------------- launchers

// Exact kNN through the path chosen by `path` (sa_knn_path); *path_used gets the one that
// ran.  Synchronous.
int launch_knn(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq, int64_t ldq,
               int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists, int32_t path,
               int32_t *path_used, hipStream_t stream);
// The double-precision scan (any data); enqueued only.  With qmap, job j is query qmap[j]
// (its row, its excluded self id and its output row).
int launch_knn_scan(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq,
                    int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists,
                    hipStream_t stream, const int32_t *qmap = nullptr);
// Queries that the last launch_knn on this thread handed from the MFMA float path to the
// scan because they could not show their margin.
extern thread_local int64_t knn_rescanned;

struct SearchLaunch {
    const void *codes;     // stored vectors (float32, bf16 or fp8 codes), rows of ldc elements
    const float *scale;    // fp8 scales
    int64_t ldc;
    int32_t dtype;
    const float *vec32;    // float32 vectors for the re-rank (may be null)
    int64_t ld32, n;
    int32_t d, metric;
    const int32_t *adj;
    int32_t R, entry;
    const float *queries;
    int64_t ldq, nq;
    int32_t k, L, M;
    sa_search_params p;
    int32_t *ids;
    float *dists;
    sa_query_stats *stats;
    void *workspace;
    size_t ws_bytes;
    // batches (device arrays, or null): per-query L and k, and the query each workgroup
    // runs; L above is then the largest L and nq the number of workgroups
    const int32_t *qL = nullptr, *qk = nullptr, *order = nullptr;
    int64_t ldo = 0;       // row stride of ids and dists (0: k)
    const int32_t *id_map = nullptr;   // result ids go through it (a renumbered index)
    // float32 vectors that are all integers in [int_lo, int_hi] with every exact partial
    // sum below 2^24 (int_lo > int_hi: not so); see index_integer_range
    int32_t int_lo = 1, int_hi = 0;
    // persistent form (null: one workgroup per job): a resident grid of workgroups takes
    // the nq jobs from this device counter pair (zero before the launch, zero after it);
    // the workspace then needs one region per resident workgroup, at most nq.  Not with a
    // re-rank (its lists stay in the regions of their jobs).
    int32_t *jobctr = nullptr;
};

// Workgroups of kernel k (block threads, lds bytes of dynamic LDS) that the device can
// hold at once, at most njobs: the grid of a persistent launch.  Cached per kernel,
// LDS size and device.
hipError_t resident_grid(const void *k, int block, uint32_t lds, int64_t njobs, int64_t *grid);
// The largest log2 of sets, in [lmin, lmax], for a filter of 4 << l bytes of LDS on top of
// base that leaves kernel k (block threads) as many workgroups per CU as the smallest
// does: the occupancy its registers allow is kept, and LDS they leave idle is used.
// Cached per kernel and device.
hipError_t lds_fill_log2(const void *k, int block, uint32_t base, int lmin, int lmax, int *out);

// Whether every stored float32 coordinate is an integer such that, for d-dimensional
// vectors and queries in the same range, every partial sum of a squared distance or
// inner product is an integer below 2^24: then float32 arithmetic in any order is exact
// and equals the double-precision result.  Sets [*lo, *hi] (lo > hi: not so).
// Synchronous (null stream).
int index_integer_range(const float *x, int64_t n, int32_t d, int64_t ld, int32_t *lo, int32_t *hi);

// ids of each job's first k (or qk[q]) results replaced by id_map[id]; enqueued only
int launch_map_ids(int32_t *ids, int64_t ldo, int64_t njobs, int32_t k, const int32_t *order, const int32_t *qk,
                   const int32_t *id_map, int64_t n, hipStream_t s);

int launch_quantize(const float *x, int64_t n, int32_t d, int64_t ld, int32_t dtype, void *codes, int64_t ldc,
                    float *scale, hipStream_t stream);

size_t search_workspace_bytes(int64_t nq, int32_t L, int32_t M, const sa_search_params &p, int32_t R);
int launch_search(const SearchLaunch &a, hipStream_t stream);
// LDS bytes one workgroup of the general kernel needs, and the visited-table sizes
// (log2; lds 0 = none) a search with these parameters takes
uint32_t search_lds_bytes(int32_t L, int32_t M, int32_t llog2, int32_t d);
void search_table_log2(const sa_search_params &p, int32_t L, int32_t M, int32_t R, int32_t *llog2, int32_t *glog2);

// Register-queue slots per lane the search kernels are compiled for: ceil(L / 64)
// rounded up: for one walker (the single-worker kernel) to 1, 2, ..., 8 or 16, for more
// (the general kernel) to 1, 2, 4, 6, 8 or 16.
inline int queue_slots_bucket(int L, int M)
{
    const int ni = (L + 63) / 64;
    if (M == 1 && ni <= 8) return ni < 1 ? 1 : ni;
    return ni <= 1 ? 1 : ni <= 2 ? 2 : ni <= 4 ? 4 : ni <= 6 ? 6 : ni <= 8 ? 8 : 16;
}

// ---------------------------------------------------------------- C ABI helpers (host)

int check_device();
int check_matrix(const void *p, int64_t rows, int32_t d, int64_t ld, const char *name);
int check_search(const sa_index *ix, int64_t nq, int32_t k, int32_t L, int32_t M, const sa_search_params &p);

}  // namespace sa

struct sa_index {
    const void *codes;    // stored vectors, rows of ldc elements of dtype
    const float *scale;   // fp8 scales
    int64_t ldc;
    int32_t dtype;
    const float *vec32;   // float32 vectors for the re-rank (may be null)
    int64_t ld32;
    int64_t n;
    int32_t d, metric;
    const int32_t *adj;
    int32_t R, entry;
    const int32_t *id_map = nullptr;   // new id -> original id, for renumbered indexes
    int32_t int_lo = 1, int_hi = 0;    // index_integer_range of float32 codes
};
