/*
 * speedann.h — C ABI of the MI355X (gfx950) implementation of the intra-query parallel
 * graph search of Speed-ANN (Peng, Zhang, Li et al., arXiv 2201.13007).
 *
 * Conventions for every entry point
 *   - Pointers named *_dev are device (HBM) pointers; all others are host pointers.
 *   - The caller owns every buffer.  Nothing here frees a caller buffer.  An index
 *     object borrows its device arrays: they must outlive it.
 *   - Calls that take a hip_stream enqueue work on that stream (NULL = the default
 *     stream) and return before it finishes, unless stated otherwise.
 *   - Return value: SA_OK (0) or a negative sa_status.  sa_last_error() returns a
 *     message for the calling thread's most recent failure.
 *   - Squared l2 distance is reported for SA_L2: it ranks like the l2 distance the
 *     paper uses (Sec. 2.1).  SA_IP reports the negated inner product, so that smaller
 *     is closer for both metrics.
 *   - Lists, results and ground truth are ordered by the key (distance, id) ascending:
 *     equal distances go to the smaller id.
 *   - Each distance is accumulated in double precision from the float32 inputs and
 *     rounded once to float32 (round to nearest even).
 */
#ifndef SPEEDANN_H
#define SPEEDANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SA_OK = 0,
    SA_EINVAL = -1,        /* invalid argument */
    SA_ENOMEM = -2,        /* a device allocation failed (graph construction only) */
    SA_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    SA_EUNSUPPORTED = -4,  /* valid but not supported (e.g. no gfx950 device) */
    SA_ECAPACITY = -5      /* workspace too small, or a fixed capacity was exceeded */
} sa_status;

typedef enum { SA_L2 = 0, SA_IP = 1 } sa_metric;

/* Vector storage of an index (not from the paper, which stores float32):
 *   SA_F32      float32
 *   SA_BF16     bfloat16: the upper half of the float32 pattern rounded to nearest even;
 *               no scale (a value is its code)
 *   SA_FP8E4M3  8-bit e4m3, finite variant (bias 7, 3 mantissa bits, subnormals m * 2^-9,
 *               largest 448, no infinities; codes 0x7F and 0xFF are NaN in the format,
 *               sa_quantize never writes them and an index must not hold them) with a
 *               float32 scale per vector: a coordinate stands for scale * value(code),
 *               computed in float32.
 * Distances are computed on these values exactly as on float32 vectors. */
typedef enum { SA_F32 = 0, SA_BF16 = 1, SA_FP8E4M3 = 2 } sa_dtype;

/* Synchronisation schedule of the local searches (Algorithm 3, CheckMetrics):
 *   SA_SYNC_BSP       merge the local queues after every local step (the Top-M scheme
 *                     of Sec. 4.1, bulk synchronous)
 *   SA_SYNC_STATIC    merge after static_I local steps; static_I <= 0 never merges
 *                     before the local queues run out of unchecked candidates
 *                     (the no-synchronisation variant of Sec. 4.3)
 *   SA_SYNC_ADAPTIVE  merge when the mean update position of the active workers is at
 *                     least L * rho (Sec. 4.3, Algorithm 2) */
typedef enum { SA_SYNC_BSP = 0, SA_SYNC_STATIC = 1, SA_SYNC_ADAPTIVE = 2 } sa_sync;

typedef struct {
    int32_t sync;           /* sa_sync; default SA_SYNC_ADAPTIVE */
    int32_t static_I;       /* SA_SYNC_STATIC interval; default 0 */
    double rho;             /* SA_SYNC_ADAPTIVE position ratio; default 0.8 (Sec. 5 uses 0.8/0.9).
                               The test is mean(U) >= L * rho, evaluated in double precision. */
    int32_t staged;         /* 1: expansion width starts at 1 and doubles after every merge
                               (Sec. 4.2, Algorithm 3); 0: width M from the start. default 1 */
    int32_t max_substeps;   /* stop a query after this many local steps (flag in stats);
                               0 = 1<<22 */
    int32_t lds_hash_slots; /* visited-set slots kept in on-chip LDS per query, power of
                               two >= 64; -1 = none (the set starts in the workspace);
                               0 = chosen from M.  A query whose visited set outgrows half
                               of it moves the set to the workspace. */
    int32_t ws_hash_slots;  /* visited-set slots per query in the workspace, power of two;
                               0 = chosen from L and M */
    int32_t rerank;         /* 0 (default): none.  > 0: the first min(rerank, |S|) entries of the
                               final list get exact distances from the index's float32 vectors
                               and the first k of them by key are returned; -1: the whole final
                               list.  Needs float32 vectors in the index (SA_EINVAL otherwise). */
    int32_t ws_hash_init;   /* one walker without an LDS table: the visited-set slots a query
                               starts with, a power of two >= 128 with 3/4 of it above R
                               (ignored for M >= 2); capped at ws_hash_slots; 0 = automatic:
                               ws_hash_slots when the tables of the queries that can be
                               resident at once fit in 128 MB at that size, else the larger
                               of 8192 and 24 L, rounded up.  A query whose set would pass three quarters
                               of its table moves it into one twice as large (flag
                               SA_QFLAG_SPILLED), up to ws_hash_slots.  Smaller tables keep more
                               of the visited sets of the queries in flight in the caches. */
} sa_search_params;

/* Per-query counters written by sa_search when stats_dev is not NULL. */
typedef struct {
    int32_t global_steps;   /* global steps that dispatched work */
    int32_t substeps;       /* lockstep local steps */
    int32_t expansions;     /* candidates marked checked */
    int32_t dist_comps;     /* distances computed (= visited vertices, entry included) */
    int32_t merges;         /* merges of the local queues into the global queue */
    int32_t flags;          /* SA_QFLAG_* */
    uint64_t t_start;       /* device real-time counter (100 MHz) at query start / end */
    uint64_t t_end;
} sa_query_stats;

#define SA_QFLAG_MAX_STEPS 1   /* stopped by max_substeps: result is the global queue then */
#define SA_QFLAG_CAPACITY 2    /* the workspace visited set filled up: result is partial */
#define SA_QFLAG_SPILLED 4     /* the visited set outgrew its first table (the LDS table, or
                                  with one walker the first workspace table) and moved */

typedef struct sa_index sa_index;

const char *sa_last_error(void);

/* Fills *out with the defaults listed in sa_search_params. */
void sa_default_params(sa_search_params *out);

/* ------------------------------------------------------------------ exact search */

/* Exact k nearest neighbours by linear scan (Sec. 2.1, the naive solution of Def. 1):
 * for every query row, the k smallest keys (distance, id) over all n base rows.
 *   base_dev     n rows of d float32, row stride ld floats (ld >= d), 16-byte aligned
 *   queries_dev  nq rows, stride ldq
 *   exclude_self when queries_dev == base_dev: row i skips base id i (graph construction)
 *   ids_dev      nq x k int32, dists_dev nq x k float32 (row-major); padded with
 *                (-1, +inf) when n (minus the excluded row) < k
 * 1 <= k <= 256.  Same as sa_knn_ex with SA_KNN_AUTO.  Synchronous: it returns after the
 * results are written. */
int sa_knn(const float *base_dev, int64_t n, int32_t d, int64_t ld, const float *queries_dev, int64_t nq,
           int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids_dev, float *dists_dev,
           void *hip_stream);

/* Two ways to compute the same exact result:
 *   SA_KNN_SCAN  double-precision accumulation on the vector units, any float data.
 *   SA_KNN_MFMA  bf16 matrix-core products, in one of two forms.
 *                Integer-valued data (every base and query coordinate an integer in
 *                [-255, 255], d <= 256, k <= 128): the coordinates, products and partial
 *                sums are all exact (each sum stays below 2^24 in magnitude), the squared
 *                distance |q|^2 + |x|^2 - 2 q.x is formed in 32-bit integers and rounded
 *                once to float32, and the keys equal the double-precision ones bit for bit.
 *                Other finite float data (d <= 1024, k <= 96): coordinates split into bf16
 *                high and low parts, three products per block give approximate distances
 *                within a proven bound (L2 data are first moved by the base mean, which
 *                leaves distances unchanged), each query keeps its 128 best candidates, and a
 *                second kernel rescores them with the scan's double-precision arithmetic;
 *                where the bound shows that no other point can enter a query's k best,
 *                its row is the scan's bit for bit, and the queries for which it cannot
 *                (many distances tied within the bound) are rescored by the scan alone
 *                (sa_knn_last_rescanned counts them).  Either form copies
 *                base and queries to temporary bf16 arrays (hipMalloc, freed before
 *                returning) and checks the values on the device first.
 *   SA_KNN_AUTO  SA_KNN_MFMA when a form applies and succeeds, else SA_KNN_SCAN. */
typedef enum { SA_KNN_AUTO = 0, SA_KNN_SCAN = 1, SA_KNN_MFMA = 2 } sa_knn_path;

/* sa_knn with an explicit path.  SA_KNN_MFMA on data or shapes it cannot take exactly
 * returns SA_EUNSUPPORTED.  *path_used_out (if not NULL) receives the path that ran
 * (SA_KNN_SCAN or SA_KNN_MFMA; SA_KNN_AUTO when nq == 0).  Synchronous. */
int sa_knn_ex(const float *base_dev, int64_t n, int32_t d, int64_t ld, const float *queries_dev, int64_t nq,
              int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids_dev, float *dists_dev,
              int32_t path, int32_t *path_used_out, void *hip_stream);

/* The number of queries that the last sa_knn / sa_knn_ex call made on the calling thread
 * handed from the float form of SA_KNN_MFMA to the scan because their candidate lists
 * could not show the margin (0 when that form did not run).  Results are exact either
 * way; the count only says how much of the call ran on the slower path. */
int64_t sa_knn_last_rescanned(void);

/* ------------------------------------------------------------------ graph construction
 * The paper searches a graph built offline (NSG, Sec. 2.2) and does not construct one.
 * These calls build the fixed-width graph the search reads: adj_dev is n x R int32,
 * row-major, each row's out-neighbours first, padded with -1. */

/* Entry point: the row nearest to the mean of all rows (double precision), ties to the
 * smaller id.  Synchronous; result in *entry_out. */
int sa_medoid(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t *entry_out, void *hip_stream);

/* Row pruning of candidate lists cand_dev (n x kc int32, each row sorted by key, as
 * sa_knn returns them with exclude_self).  prune 0: keep the first R.  prune 1
 * (relative-neighbourhood rule): scan the candidates in order, keep c unless an already
 * kept s has d(s, c) < d(p, c), stop at R kept.  Enqueued on hip_stream. */
int sa_prune(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, const int32_t *cand_dev,
             int32_t kc, int32_t R, int32_t prune, int32_t *adj_dev, void *hip_stream);

/* Reverse edges, in place (synchronous): with the graph as it stands, every vertex c
 * appends to its row the sources p of its in-edges (p -> c) that the row does not hold
 * yet, in key order (d(c, p), p), while the row has fewer than R entries.  All rows read
 * the graph as it was before any append.  *added_out (if not NULL) gets the count. */
int sa_reverse_edges(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t *adj_dev,
                     int32_t R, int64_t *added_out, void *hip_stream);

/* Connectivity repair of adj_dev in place (synchronous; copies the graph to the host):
 * (1) weakly connected components, each with its medoid as representative;
 * (2) gateway rows: every representative (keeping its first keep_local edges), the entry
 *     and the hubs - the `hubs` - 1 other vertices nearest to the mean of all rows,
 *     representatives excepted (keeping hub_keep_local edges each) - get a new row: the
 *     kept edges, then links to other representatives chosen by the relative-
 *     neighbourhood rule over all of them in key order and filled with the nearest
 *     ones.  On clustered data this is what lets a search that starts at the medoid
 *     leave the medoid's cluster;
 * (3) in increasing id order every vertex not reachable from the entry gets an edge from
 *     the nearest reachable vertex with a free slot.
 * Writes the number of (3) edges and of components to the outputs when not NULL.
 * SA_ECAPACITY if (3) finds no reachable vertex with a free slot. */
int sa_repair(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t *adj_dev,
              int32_t R, int32_t entry, int32_t keep_local, int32_t hubs, int32_t hub_keep_local,
              int64_t *bridges_out, int64_t *components_out, void *hip_stream);

/* Whole pipeline: entry = sa_medoid; candidates = sa_knn(knn_k, exclude_self);
 * adj = sa_prune; if repair, sa_reverse_edges then sa_repair(keep_local, hubs, hub_keep_local).  Synchronous.  Allocates its
 * temporaries with hipMalloc and frees them before returning. */
int sa_build_graph(const float *base_dev, int64_t n, int32_t d, int64_t ld, int32_t metric, int32_t knn_k,
                   int32_t R, int32_t prune, int32_t repair, int32_t keep_local, int32_t hubs,
                   int32_t hub_keep_local, int32_t *adj_dev, int32_t *entry_out, int64_t *bridges_out,
                   int64_t *components_out, void *hip_stream);

/* ------------------------------------------------------------------ the search */

/* Wraps borrowed device arrays: vec_dev (n rows of d float32, stride ld floats,
 * 16-byte aligned, ld % 4 == 0, ld >= d), adj_dev (n x R int32, -1 padded, ids in
 * [0, n), no id twice in a row), entry in [0, n).  1 <= R <= 64, n < 2^31. */
int sa_index_create(const float *vec_dev, int64_t n, int32_t d, int64_t ld, int32_t metric,
                    const int32_t *adj_dev, int32_t R, int32_t entry, sa_index **out);
void sa_index_destroy(sa_index *index);

/* Scans an index's float32 storage once (synchronous: waits for hip_stream, then runs on
 * the null stream).  If every coordinate is an integer in a range [lo, hi] such that
 * (hi - lo)^2 * d and max(|lo|, |hi|)^2 * d are below 2^24, every partial sum of a squared
 * distance or inner product between vectors and queries in that range is an integer
 * below 2^24, exact in float32 in any order of addition.  sa_search with one walker then
 * accumulates the distances of the queries whose coordinates are all integers in [lo, hi]
 * in float32 (fewer registers, more queries in flight) and the others in double, in two
 * launches; every key is the same as without the scan.  Without this call, or for other
 * storage types, the search accumulates in double.  Returns SA_OK whether or not the data
 * qualify (sa_index_integer_range tells). */
int sa_index_analyze(sa_index *index, void *hip_stream);

/* 1 and [*lo, *hi] (either pointer may be NULL) when sa_index_analyze found the index's
 * vectors integer-valued as described there; 0 otherwise. */
int32_t sa_index_integer_range(const sa_index *index, int32_t *lo, int32_t *hi);

/* Reduced-precision copy of n vectors (rows of d float32, stride ld, 16-byte aligned):
 *   dtype      SA_BF16 or SA_FP8E4M3
 *   codes_dev  n rows of ldc codes (2 bytes each for bf16, 1 for fp8), ldc >= d,
 *              ldc % 4 == 0, 16-byte aligned; columns d..ldc-1 get code 0
 *   scale_dev  n floats: amax / 448 per vector for fp8 (1 for a zero vector), 1 for bf16
 * Codes round to nearest even; fp8 saturates at 448.  Enqueued on hip_stream. */
int sa_quantize(const float *x_dev, int64_t n, int32_t d, int64_t ld, int32_t dtype, void *codes_dev, int64_t ldc,
                float *scale_dev, void *hip_stream);

/* sa_index_create for any storage: codes_dev holds n rows of ldc elements of dtype (for
 * SA_F32 the float32 vectors, 16-byte aligned, ldc % 4 == 0), scale_dev the fp8 scales
 * (ignored otherwise), vec32_dev (may be NULL) the float32 vectors with stride ld32, read
 * only by the re-rank.  The index borrows every array. */
int sa_index_create_q(const void *codes_dev, int32_t dtype, const float *scale_dev, int64_t ldc,
                      const float *vec32_dev, int64_t ld32, int64_t n, int32_t d, int32_t metric,
                      const int32_t *adj_dev, int32_t R, int32_t entry, sa_index **out);

/* Bytes of workspace sa_search needs for nq queries (visited sets that outgrow LDS). */
size_t sa_search_workspace_bytes(const sa_index *index, int64_t nq, int32_t k, int32_t L, int32_t M,
                                 const sa_search_params *params);

/* Intra-query parallel search (Algorithm 3; Algorithm 1 when M = 1), one workgroup per
 * query and one wavefront per worker (two workers that merge after every local step,
 * SA_SYNC_BSP, over adjacency rows of at most 32 entries share one wavefront; results and
 * counters are the same either way):
 *   queries_dev  nq x d float32, stride ldq floats (16-byte aligned rows); d <= 1024
 *   k, L         results per query and queue capacity, 1 <= k <= L <= 1024
 *   M            workers (the paper's T, the maximum expansion width), 1 <= M <= 16
 *   params       NULL for defaults
 *   ids_dev      nq x k int32, dists_dev nq x k float32; padded with (-1, +inf) when
 *                fewer than k vertices were reached
 *   stats_dev    NULL or nq sa_query_stats
 *   workspace    sa_search_workspace_bytes(...) bytes of device memory, 256-byte aligned,
 *                zero-filled before its first use.  Every call leaves it zero-filled again
 *                when it completes, so one buffer serves any number of calls; calls that
 *                share a workspace must not overlap.
 * Allocates nothing.  Enqueued on hip_stream: kernel launches only (two of the search
 * kernel when sa_index_analyze found integer data, then a re-rank and an id-map kernel
 * when asked for), so the call can be captured in a HIP graph. */
int sa_search(const sa_index *index, const float *queries_dev, int64_t nq, int64_t ldq, int32_t k, int32_t L,
              int32_t M, const sa_search_params *params, int32_t *ids_dev, float *dists_dev,
              sa_query_stats *stats_dev, void *workspace, size_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sa_search with the same arguments
 * except the workspace, which is a static 64 MiB device array of the library instead
 * (every device the library runs on holds its own copy until the process ends).  Calls
 * whose workspace would exceed it (sa_search_workspace_bytes > 64 MiB; e.g. L = 192,
 * M = 2 takes 64 KB per query) are rejected with SA_ECAPACITY.  All calls on one device
 * share that array, as sa_search calls that share a workspace do: calls that overlap
 * on one device (other streams, other host threads) race and must not be made.  The
 * first call on a device also enqueues, ahead of its search, a kernel that zero-fills the
 * array (every search leaves it zero again).  Allocates nothing and calls no allocating
 * routine; enqueued on hip_stream like sa_search. */
int sa_search_noalloc(const sa_index *index, const float *queries_dev, int64_t nq, int64_t ldq, int32_t k,
                      int32_t L, int32_t M, const sa_search_params *params, int32_t *ids_dev, float *dists_dev,
                      sa_query_stats *stats_dev, void *hip_stream);

/* ------------------------------------------------------------------ renumbering
 *
 * The GPU counterpart of the neighbour grouping of Sec. 4.4: renumber the vertices so
 * that vertices a search meets together sit together in memory.  An index built over
 * the permuted vectors and graph, with sa_index_set_id_map(perm), returns ids in the
 * original numbering; its searches are the searches of the renumbered graph (equal
 * distances are ordered by the new ids). */
typedef enum {
    SA_ORDER_DEGREE = 0,   /* in-degree descending, ties by id */
    SA_ORDER_BFS = 1       /* breadth-first from entry, neighbours in row order; unreachable vertices last, by id */
} sa_order;

/* perm_dev (n int32, device) gets the order: perm[i] = original id of new vertex i.
 * adj_dev: n x R int32 (-1 padded).  Offline step: counts on the device, orders on the
 * host; synchronous; allocates temporaries. */
int sa_graph_order(const int32_t *adj_dev, int64_t n, int32_t R, int32_t entry, int32_t mode, int32_t *perm_dev,
                   void *hip_stream);

/* dst row i = src row perm[i], rows of row_bytes (a multiple of 4) for vectors or codes;
 * a perm entry outside [0, n) gives a zero row.  src and dst must differ.  Enqueued. */
int sa_permute_rows(const void *src_dev, int64_t n, int64_t row_bytes, const int32_t *perm_dev, void *dst_dev,
                    void *hip_stream);

/* adj_out row i = adj row perm[i] with ids renumbered through inv (written to inv_dev,
 * n int32: inv[perm[i]] = i); the entry of the new graph is inv[entry].  adj and adj_out
 * must differ.  Enqueued. */
int sa_permute_graph(const int32_t *adj_dev, int64_t n, int32_t R, const int32_t *perm_dev, int32_t *inv_dev,
                     int32_t *adj_out_dev, void *hip_stream);

/* Result ids of every later search on index go through id_map_dev (n int32, device,
 * borrowed; NULL to stop): a small kernel after the search maps them on the same
 * stream. */
int sa_index_set_id_map(sa_index *index, const int32_t *id_map_dev);

/* ------------------------------------------------------------------ measurement
 *
 * Gather ceiling (a measurement tool, not part of the search): `waves` wavefronts each
 * read iters x 64 / g whole rows of vec_dev (n rows of d float32, stride ld) chosen by
 * a 32-bit hash of (seed, wavefront, pass, group), g lanes per row as the search's
 * distance step uses them, and write one float per lane to sink_dev (waves x 64
 * floats).  Rows read = waves * iters * 64 / g, g = the search's lanes per vector for
 * d (for d = 128: 8).  iters and waves are positive multiples of 4; n < 2^32.
 * Enqueued on hip_stream; time it with events. */
int sa_gather_probe(const float *vec_dev, int64_t n, int32_t d, int64_t ld, int64_t iters, int32_t waves,
                    uint32_t seed, float *sink_dev, void *hip_stream);

/* ------------------------------------------------------------------ batches
 *
 * A batch is a fixed set of nq queries, each with its own L, k and M, searched together:
 * the inter-query parallelism of Sec. 1 on top of the intra-query parallelism of
 * Algorithm 3.  The result of every query is exactly
 * the one sa_search gives for it alone with its own (L, k, M) and the batch's shared
 * params, whatever the batch holds and however it is tuned.
 *
 * The plan groups the queries into classes of equal M and equal register-queue size
 * (ceil(L / 64), rounded up to 1-8 or 16 when M = 1 and to 1, 2, 4, 6, 8 or 16 when
 * M >= 2), one kernel launch each, longest L
 * first within a class; classes go to up to eight internal streams (each wants a
 * hardware queue of its own: GPU_MAX_HW_QUEUES, default 4).  sa_batch_run only
 * enqueues kernel launches and event records and waits, so it can be captured in a HIP
 * graph from hip_stream (the classes become parallel branches) and replayed.  The
 * workspace holds the uploaded per-query arrays, two job counters per class (zero
 * between runs) and one visited-set region per query (as sa_search sizes them for the
 * class's largest L, for the largest of the LDS-table settings the tuner may choose; a
 * persistent class uses one per resident workgroup); the search regions are zero
 * between runs.  A re-rank (params->rerank != 0) runs after each class's search, as in
 * sa_search, and needs the index's float32 vectors. */
typedef struct sa_batch sa_batch;

/* L, k, M: host arrays of nq entries, copied (1 <= k <= L <= 1024, 1 <= M <= 16).
 * params: NULL for defaults; shared by every query. */
int sa_batch_create(const sa_index *index, int64_t nq, const int32_t *L, const int32_t *k, const int32_t *M,
                    const sa_search_params *params, sa_batch **out);
void sa_batch_destroy(sa_batch *batch);
size_t sa_batch_workspace_bytes(const sa_batch *batch);

/* Writes the batch's per-query arrays into workspace (sa_batch_workspace_bytes bytes,
 * 256-byte aligned, zero-filled before its first use) and waits for the copy.  Once per
 * workspace, before the first run or tune on it; not for capture. */
int sa_batch_upload(const sa_batch *batch, void *workspace, size_t ws_bytes, void *hip_stream);

/* Searches the batch: queries_dev nq x d float32 (stride ldq), ids_dev / dists_dev rows
 * of stride ldo >= the largest k, of which row q gets its first k[q] entries (the rest
 * is not written), stats_dev NULL or nq sa_query_stats.  Allocates nothing; enqueued on
 * hip_stream (forking onto the batch's streams and joining back); runs that share a
 * workspace must not overlap. */
int sa_batch_run(const sa_batch *batch, const float *queries_dev, int64_t ldq, int32_t *ids_dev, float *dists_dev,
                 int64_t ldo, sa_query_stats *stats_dev, void *workspace, size_t ws_bytes, void *hip_stream);

/* Autotuner (best of reps after one warm run each).  First every class alone, in each
 * of its forms: one workgroup per query, or persistent (as many workgroups as the device
 * holds at once, taking the class's queries from a device counter in the plan's order;
 * not with a re-rank), each with each LDS visited-table setting sa_batch_class_options
 * lists.  Then the whole batch on 1, 2, 4 and 8 streams for three plans: every class one
 * workgroup per query, every class persistent, each class in its fastest form; the
 * fastest plan and stream count are kept (sa_batch_describe reports every time).  Results
 * do not depend on the choice.  Synchronous; overwrites ids_dev and dists_dev. */
int sa_batch_tune(sa_batch *batch, const float *queries_dev, int64_t ldq, int32_t *ids_dev, float *dists_dev,
                  int64_t ldo, void *workspace, size_t ws_bytes, int32_t reps, void *hip_stream);

/* Sets the configuration by hand: streams 1, 2, 4 or 8; lds_hash_slots for the classes with
 * two or more walkers (as in sa_search_params; it must give each such class the table one
 * of its options gives). */
int sa_batch_set_config(sa_batch *batch, int32_t streams, int32_t lds_hash_slots);

/* Number of classes of the plan (in the order sa_batch_describe lists them). */
int32_t sa_batch_classes(const sa_batch *batch);

/* The settings class cls may run with: *count lds_hash_slots values (the first cap of them
 * into lds_values), and whether the persistent form is allowed (no re-rank).  The
 * workspace holds room for each of them. */
int sa_batch_class_options(const sa_batch *batch, int32_t cls, int32_t *lds_values, int32_t cap, int32_t *count,
                           int32_t *persistent_ok);

/* Sets class cls by hand: an lds_hash_slots value that gives the table one of its options
 * gives, and the persistent form (1) or one workgroup per query (0). */
int sa_batch_set_class(sa_batch *batch, int32_t cls, int32_t lds_hash_slots, int32_t persistent);

/* JSON description of the plan (classes, their sizes, configuration, last tuning) into
 * buf (NUL-terminated, truncated to len); returns the length it needs including the NUL,
 * or a negative status. */
int64_t sa_batch_describe(const sa_batch *batch, char *buf, size_t len);

/* ------------------------------------------------------------------ serving
 *
 * A request loop over a resident index: requests (one query each, with its own k, L and
 * M) are submitted from any host thread and served by a worker thread of the library
 * with continuous batching.  Requests wait in one of up to four lanes by L (<= 128,
 * <= 256, <= 512, above; fewer lanes if slots < 4), each with its own slots (slot s
 * serves lane s mod lanes; every slot has a stream of its own).  Whenever a slot is free, the worker admits its
 * lane's waiting requests in arrival order into it, up to max_batch and while their
 * visited-set regions (sized as sa_search sizes them for the request's register-queue
 * size) fit the slot's share of workspace_bytes, and launches them: one copy in, then
 * per class of equal M and queue size, shortest first, a launch, the copy of its
 * results and an event, after which its requests are complete.  Requests that arrive
 * while micro-batches run are admitted into the next free slot, so their work overlaps
 * on the device, and a short search never waits for a long one's slot.  A request's result is the
 * one sa_search gives for it alone, whatever it was batched with.  Give the process at
 * least slots + 1 hardware queues (HIP reads GPU_MAX_HW_QUEUES, default 4, at start-up):
 * streams beyond the queue count share queues and run their kernels one after another,
 * which put 20 ms on a 5 ms request at 16 slots over 4 queues.  The worker owns all
 * its device and pinned host memory, allocated at creation; the index must outlive
 * the server. */
typedef struct sa_server sa_server;

typedef struct {
    int32_t slots;            /* micro-batches in flight at once, 1..16 (default 8) */
    int32_t max_batch;        /* requests per micro-batch, 1..65536 (default 1024) */
    int32_t max_pending;      /* waiting requests held before submit reports SA_ECAPACITY (default 65536) */
    int32_t k_max;            /* largest k a request may ask (default 100) */
    size_t workspace_bytes;   /* device workspace for visited sets, split over the slots (default 1 GiB) */
} sa_server_config;

void sa_server_default_config(sa_server_config *cfg);

/* params: NULL for defaults, shared by every request (a re-rank needs the index's
 * float32 vectors). */
int sa_server_create(const sa_index *index, const sa_search_params *params, const sa_server_config *cfg,
                     sa_server **out);

/* Stops admitting, waits for the micro-batches in flight, frees everything.  Results
 * not yet polled are dropped. */
void sa_server_destroy(sa_server *server);

/* Queues one request: query_host d float32 (copied before return), 1 <= k <= min(L,
 * k_max), L <= 1024, 1 <= M <= 16; tag is returned with its result.  Thread-safe.
 * SA_ECAPACITY when max_pending requests are already waiting. */
int sa_server_submit(sa_server *server, const float *query_host, int32_t k, int32_t L, int32_t M, uint64_t tag);

/* Takes up to max finished requests, waiting up to wait_us microseconds for the first:
 * tags[i], ids (row i of stride ldo >= k_max: its first k entries), dists likewise,
 * t_submit_ns / t_done_ns (steady-clock nanoseconds; either array may be NULL).
 * Returns the count, or a negative status.  Thread-safe. */
int32_t sa_server_poll(sa_server *server, int32_t max, uint64_t *tags, int32_t *ids, float *dists, int64_t ldo,
                       int64_t *t_submit_ns, int64_t *t_done_ns, int32_t wait_us);

/* Load replay: submits request i (queries_host row i, stride ldq; k[i], L[i], M[i]) at
 * arrival_ns[i] nanoseconds after the call starts (non-decreasing), collects every
 * result into row i of ids / dists (stride ldo) and latency_ns[i] = completion time -
 * scheduled arrival, and returns the wall time from the first arrival to the last
 * completion in *wall_ns.  Blocks until all n are done; requests submitted by others
 * meanwhile are served too but not collected here. */
int sa_server_replay(sa_server *server, const float *queries_host, int64_t n, int64_t ldq, const int32_t *k,
                     const int32_t *L, const int32_t *M, const int64_t *arrival_ns, int32_t *ids, float *dists,
                     int64_t ldo, int64_t *latency_ns, int64_t *wall_ns);

/* Counters since creation: requests completed, micro-batches launched, kernel launches,
 * largest micro-batch, and the sum of micro-batch sizes. */
int sa_server_stats(const sa_server *server, int64_t *completed, int64_t *batches, int64_t *launches,
                    int64_t *max_batch_seen, int64_t *sum_batch);

#ifdef __cplusplus
}
#endif

#endif /* SPEEDANN_H */
