/*
 * CPU oracle for the Speed-ANN hot path (arXiv 2201.13007).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  The GPU library never links,
 * calls or includes anything from here, and this file includes nothing from it.
 *
 * Plain, slow, obviously correct C.  Every list is an array that is re-sorted after
 * each insertion; every set is a byte map.  Floating point: each distance is
 * accumulated in double precision in index order and rounded once to float
 * (round to nearest even); lists are ordered by the key (distance, id) ascending.
 *
 * Contents and the passages they follow:
 *   or_distance       squared l2 (the ranking of the l2 distance, Sec. 2.1) or the
 *                     negated inner product
 *   or_knn            linear scan (the naive exact solution, Sec. 2.1, Def. 1)
 *   or_bfis           best-first search, Algorithm 1
 *   or_topm           Top-M parallel neighbour expansion, Sec. 4.1 (top M unchecked
 *                     candidates per step), optionally staged (Sec. 4.2: M doubles
 *                     every step from 1)
 *   or_speedann       Algorithm 3 with CheckMetrics (Algorithm 2), emulated in
 *                     lockstep: workers take one local step each per sub-step, in
 *                     worker order, against one exact shared visited set
 *   graph helpers     medoid, row pruning, connectivity repair (graph construction is
 *                     outside the paper, which takes an NSG graph as given, Sec. 2.2)
 *   reduced precision vector storage in bf16 or fp8 e4m3 with a per-vector scale, and
 *                     the exact re-rank of a final candidate list (outside the paper,
 *                     which stores float32): or_quantize, or_dequantize, or_rerank
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - the starting point is marked visited when it is added (Algorithm 1 adds it
 *     without marking it);
 *   - the update position of a worker that inserted nothing that survived the
 *     truncation, or that was idle, is L; positions are 0-based after truncation;
 *   - "divide all unchecked vertices from S into LS": every local queue starts as a
 *     full copy of S; the j-th unchecked entry of S (in key order) belongs to worker
 *     j mod m; the other workers see it as FOREIGN (it occupies a slot but they never
 *     expand it);
 *   - merge: the union of S and every local queue, one entry per id, CHECKED if any
 *     copy is CHECKED, truncated to L;
 *   - the check runs after every sub-step; "M <- 2M" is capped at T.
 *
 * parity pins: see tests/test_oracle*.py (exact kNN at L >= reachable set, M=1
 * reduces to Algorithm 1, synchronising every step reduces to Top-M, adaptive with
 * ratio 0 reduces to Top-M and with ratio above 1 to no synchronisation, hand-derived
 * traces under tests/golden/).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_L2 0
#define OR_IP 1

#define OR_SYNC_BSP 0
#define OR_SYNC_STATIC 1
#define OR_SYNC_ADAPTIVE 2

typedef struct {
    int64_t global_steps;   /* iterations of the outer loop that dispatched work */
    int64_t substeps;       /* lockstep local steps (one per worker per sub-step) */
    int64_t expansions;     /* vertices marked checked */
    int64_t dist_comps;     /* distances computed = size of the visited set */
    int64_t merges;         /* merges of the local queues into S */
} or_stats;

/* ---------------------------------------------------------------- distance */

float or_distance(const float *a, const float *b, int d, int metric)
{
    double acc = 0.0;
    if (metric == OR_L2) {
        for (int i = 0; i < d; ++i) {
            double t = (double)a[i] - (double)b[i];
            acc += t * t;
        }
        return (float)acc;
    }
    for (int i = 0; i < d; ++i) acc += (double)a[i] * (double)b[i];
    return (float)(-acc);
}

/* ---------------------------------------------------------------- entries */

typedef struct {
    float dist;
    int32_t id;
    int32_t state;      /* search lists: see ST_* */
} entry;

enum { ST_UNCHECKED = 0, ST_CHECKED = 1, ST_FOREIGN = 2 };

static int key_less(float da, int32_t ia, float db, int32_t ib)
{
    if (da < db) return 1;
    if (da > db) return 0;
    return ia < ib;
}

static int entry_cmp(const void *pa, const void *pb)
{
    const entry *a = (const entry *)pa, *b = (const entry *)pb;
    if (key_less(a->dist, a->id, b->dist, b->id)) return -1;
    if (key_less(b->dist, b->id, a->dist, a->id)) return 1;
    return 0;
}

static void sort_entries(entry *e, int64_t n) { qsort(e, (size_t)n, sizeof(entry), entry_cmp); }

static const float *row(const float *base, int64_t i, int64_t ld) { return base + i * ld; }

/* ---------------------------------------------------------------- exact kNN */

/* For each query, the k smallest keys (distance, id) over all n base vectors.
 * With exclude_self, query i (a base vector itself) skips base id i.
 * Short results are padded with (-1, +inf). */
static void knn_impl(const float *base, int64_t n, int d, int64_t ld, const float *queries, int64_t nq,
                     int64_t ldq, int k, int metric, int exclude_self, const int32_t *self_ids, int32_t *ids,
                     float *dists);

void or_knn(const float *base, int64_t n, int d, int64_t ld, const float *queries, int64_t nq,
            int64_t ldq, int k, int metric, int exclude_self, int32_t *ids, float *dists)
{
    knn_impl(base, n, d, ld, queries, nq, ldq, k, metric, exclude_self, NULL, ids, dists);
}

/* As or_knn, but query qi skips base id self_ids[qi] (queries that are base rows). */
void or_knn_self(const float *base, int64_t n, int d, int64_t ld, const float *queries, int64_t nq,
                 int64_t ldq, int k, int metric, const int32_t *self_ids, int32_t *ids, float *dists)
{
    knn_impl(base, n, d, ld, queries, nq, ldq, k, metric, 1, self_ids, ids, dists);
}

static void knn_impl(const float *base, int64_t n, int d, int64_t ld, const float *queries, int64_t nq,
                     int64_t ldq, int k, int metric, int exclude_self, const int32_t *self_ids, int32_t *ids,
                     float *dists)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; ++qi) {
        entry *top = (entry *)malloc(sizeof(entry) * (size_t)(k + 1));
        int cnt = 0;
        const float *q = row(queries, qi, ldq);
        for (int64_t i = 0; i < n; ++i) {
            if (exclude_self && i == (self_ids ? (int64_t)self_ids[qi] : qi)) continue;
            float dd = or_distance(q, row(base, i, ld), d, metric);
            if (cnt == k && !key_less(dd, (int32_t)i, top[k - 1].dist, top[k - 1].id)) continue;
            /* insertion into the sorted top list */
            int pos = cnt < k ? cnt : k - 1;
            while (pos > 0 && key_less(dd, (int32_t)i, top[pos - 1].dist, top[pos - 1].id)) {
                top[pos] = top[pos - 1];
                --pos;
            }
            top[pos].dist = dd;
            top[pos].id = (int32_t)i;
            if (cnt < k) ++cnt;
        }
        for (int j = 0; j < k; ++j) {
            ids[qi * k + j] = j < cnt ? top[j].id : -1;
            dists[qi * k + j] = j < cnt ? top[j].dist : INFINITY;
        }
        free(top);
    }
}

/* ---------------------------------------------------------------- search: shared helpers */

typedef struct {
    const float *base;
    int64_t n, ld;
    int d, metric;
    const int32_t *adj;
    int R;
    const float *q;
} problem;

static float pdist(const problem *p, int32_t v) { return or_distance(p->q, row(p->base, v, p->ld), p->d, p->metric); }

static void emit(const entry *S, int64_t len, int k, int32_t *ids, float *dists)
{
    for (int j = 0; j < k; ++j) {
        ids[j] = j < len ? S[j].id : -1;
        dists[j] = j < len ? S[j].dist : INFINITY;
    }
}

/* ---------------------------------------------------------------- Algorithm 1 */

int or_bfis(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
            int32_t entry_id, const float *q, int k, int L, int32_t *ids, float *dists, or_stats *st)
{
    problem P = {base, n, ld, d, metric, adj, R, q};
    or_stats s = {0, 0, 0, 0, 0};
    uint8_t *visited = (uint8_t *)calloc((size_t)n, 1);
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)(L + R));
    if (!visited || !S) { free(visited); free(S); return -2; }
    int64_t len = 0;

    /* compute dist(P, Q) and add P into S */
    S[len].dist = pdist(&P, entry_id); S[len].id = entry_id; S[len].state = ST_UNCHECKED; ++len;
    visited[entry_id] = 1; s.dist_comps = 1;

    for (;;) {
        /* i <- index of the first unchecked vertex in S */
        int64_t i = -1;
        for (int64_t j = 0; j < len; ++j) if (S[j].state == ST_UNCHECKED) { i = j; break; }
        if (i < 0) break;
        S[i].state = ST_CHECKED;
        s.expansions++; s.global_steps++; s.substeps++;
        int32_t v = S[i].id;
        for (int r = 0; r < R; ++r) {
            int32_t u = adj[(int64_t)v * R + r];
            if (u < 0) continue;
            if (visited[u]) continue;
            visited[u] = 1;
            s.dist_comps++;
            S[len].dist = pdist(&P, u); S[len].id = u; S[len].state = ST_UNCHECKED; ++len;
        }
        sort_entries(S, len);
        if (len > L) len = L;
    }
    emit(S, len, k, ids, dists);
    if (st) *st = s;
    free(visited); free(S);
    return 0;
}

/* ---------------------------------------------------------------- Top-M (Sec. 4.1) */

/* Each step expands the first m unchecked candidates of S (all of them when fewer),
 * inserts the union of their unvisited neighbours and truncates S to L.  The
 * neighbours are visited in (expanded candidate order, adjacency slot) order.
 * staged: m = 1 at the first step and doubles every step up to M (Sec. 4.2, t = 1). */
int or_topm(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
            int32_t entry_id, const float *q, int k, int L, int M, int staged, int32_t *ids, float *dists,
            or_stats *st)
{
    problem P = {base, n, ld, d, metric, adj, R, q};
    or_stats s = {0, 0, 0, 0, 0};
    uint8_t *visited = (uint8_t *)calloc((size_t)n, 1);
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)(L + (int64_t)M * R));
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    if (!visited || !S || !act) { free(visited); free(S); free(act); return -2; }
    int64_t len = 0;
    int m = staged ? 1 : M;

    S[len].dist = pdist(&P, entry_id); S[len].id = entry_id; S[len].state = ST_UNCHECKED; ++len;
    visited[entry_id] = 1; s.dist_comps = 1;

    for (;;) {
        int na = 0;
        for (int64_t j = 0; j < len && na < m; ++j)
            if (S[j].state == ST_UNCHECKED) { S[j].state = ST_CHECKED; act[na++] = S[j].id; }
        if (na == 0) break;
        s.expansions += na; s.global_steps++; s.substeps++; s.merges++;
        for (int a = 0; a < na; ++a) {
            int32_t v = act[a];
            for (int r = 0; r < R; ++r) {
                int32_t u = adj[(int64_t)v * R + r];
                if (u < 0 || visited[u]) continue;
                visited[u] = 1;
                s.dist_comps++;
                S[len].dist = pdist(&P, u); S[len].id = u; S[len].state = ST_UNCHECKED; ++len;
            }
        }
        sort_entries(S, len);
        if (len > L) len = L;
        if (staged && m < M) m = (2 * m < M) ? 2 * m : M;
    }
    emit(S, len, k, ids, dists);
    if (st) *st = s;
    free(visited); free(S); free(act);
    return 0;
}

/* ---------------------------------------------------------------- Algorithm 3 */

/* CheckMetrics (Algorithm 2): true iff the mean of the update positions of the m
 * active workers is at least L * ratio. */
static int check_metrics(const int32_t *U, int m, int L, double ratio)
{
    int64_t sum = 0;
    for (int t = 0; t < m; ++t) sum += U[t];
    double mean = (double)sum / (double)m;
    return mean >= (double)L * ratio;
}

/* T workers (the maximum expansion width); sync selects CheckMetrics:
 *   OR_SYNC_BSP       merge after every sub-step
 *   OR_SYNC_STATIC    merge after static_I sub-steps (static_I <= 0: only when every
 *                     local queue is exhausted, i.e. no synchronisation)
 *   OR_SYNC_ADAPTIVE  Algorithm 2 with position ratio rho
 * staged: the expansion width starts at 1 and doubles after every merge (Algorithm 3);
 * otherwise it is T from the start. */
int or_speedann(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
                int32_t entry_id, const float *q, int k, int L, int T, int sync, int static_I, double rho,
                int staged, int max_substeps, int32_t *ids, float *dists, or_stats *st)
{
    problem P = {base, n, ld, d, metric, adj, R, q};
    or_stats s = {0, 0, 0, 0, 0};
    uint8_t *visited = (uint8_t *)calloc((size_t)n, 1);
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)L);
    entry *LS = (entry *)malloc(sizeof(entry) * (size_t)T * (size_t)(L + R));
    int64_t *LSlen = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    entry *all = (entry *)malloc(sizeof(entry) * (size_t)(T + 1) * (size_t)L);
    if (!visited || !S || !LS || !LSlen || !U || !all) {
        free(visited); free(S); free(LS); free(LSlen); free(U); free(all);
        return -2;
    }
    int rc = 0;
    int64_t len = 0;
    int m = staged ? 1 : T;

    /* compute dist(P, Q); add P into S */
    S[len].dist = pdist(&P, entry_id); S[len].id = entry_id; S[len].state = ST_UNCHECKED; ++len;
    visited[entry_id] = 1; s.dist_comps = 1;

    for (;;) {
        /* divide all unchecked vertices from S into LS: the j-th unchecked entry goes to
         * worker j mod m; each local queue is a copy of S */
        int64_t nunchecked = 0;
        for (int t = 0; t < m; ++t) LSlen[t] = len;
        for (int64_t j = 0; j < len; ++j) {
            int owner = -1;
            if (S[j].state == ST_UNCHECKED) owner = (int)(nunchecked++ % m);
            for (int t = 0; t < m; ++t) {
                entry e = S[j];
                if (e.state == ST_UNCHECKED && owner != t) e.state = ST_FOREIGN;
                LS[(int64_t)t * (L + R) + j] = e;
            }
        }
        /* all local queues empty of unchecked work: done */
        if (nunchecked == 0) break;
        s.global_steps++;

        /* local best-first searches in lockstep until CheckMetrics asks for a merge or
         * no worker has unchecked vertices left */
        int sub_in_step = 0;
        for (;;) {
            int any = 0;
            for (int t = 0; t < m; ++t) {
                entry *Q = LS + (int64_t)t * (L + R);
                for (int64_t j = 0; j < LSlen[t]; ++j) if (Q[j].state == ST_UNCHECKED) { any = 1; break; }
            }
            if (!any) break;
            /* step limit (not part of the paper): merge, then stop */
            if (max_substeps > 0 && s.substeps >= max_substeps) { rc = 1; break; }
            s.substeps++; sub_in_step++;
            for (int t = 0; t < m; ++t) {
                entry *Q = LS + (int64_t)t * (L + R);
                int64_t i = -1;
                for (int64_t j = 0; j < LSlen[t]; ++j) if (Q[j].state == ST_UNCHECKED) { i = j; break; }
                U[t] = L;
                if (i < 0) continue;                     /* idle worker */
                Q[i].state = ST_CHECKED;
                s.expansions++;
                int32_t v = Q[i].id;
                int64_t before = LSlen[t];
                for (int r = 0; r < R; ++r) {
                    int32_t u = adj[(int64_t)v * R + r];
                    if (u < 0 || visited[u]) continue;
                    visited[u] = 1;
                    s.dist_comps++;
                    Q[LSlen[t]].dist = pdist(&P, u); Q[LSlen[t]].id = u; Q[LSlen[t]].state = ST_UNCHECKED;
                    LSlen[t]++;
                }
                if (LSlen[t] > before) {
                    /* the update position is the best position of a newly inserted
                     * candidate after the queue is sorted and truncated */
                    entry *newest = (entry *)malloc(sizeof(entry) * (size_t)(LSlen[t] - before));
                    memcpy(newest, Q + before, sizeof(entry) * (size_t)(LSlen[t] - before));
                    int64_t nnew = LSlen[t] - before;
                    sort_entries(Q, LSlen[t]);
                    if (LSlen[t] > L) LSlen[t] = L;
                    for (int64_t j = 0; j < LSlen[t]; ++j) {
                        int isnew = 0;
                        for (int64_t x = 0; x < nnew; ++x) if (newest[x].id == Q[j].id) { isnew = 1; break; }
                        if (isnew) { U[t] = (int32_t)j; break; }
                    }
                    free(newest);
                }
            }
            int merge_now;
            if (sync == OR_SYNC_BSP) merge_now = 1;
            else if (sync == OR_SYNC_STATIC) merge_now = static_I > 0 && sub_in_step >= static_I;
            else merge_now = check_metrics(U, m, L, rho);
            if (merge_now) break;
        }

        /* merge LS into S: one entry per id, CHECKED if any copy is CHECKED */
        int64_t na = 0;
        for (int64_t j = 0; j < len; ++j) all[na++] = S[j];
        for (int t = 0; t < m; ++t)
            for (int64_t j = 0; j < LSlen[t]; ++j) all[na++] = LS[(int64_t)t * (L + R) + j];
        sort_entries(all, na);
        len = 0;
        for (int64_t j = 0; j < na; ++j) {
            int checked = all[j].state == ST_CHECKED;
            if (len > 0 && S[len - 1].id == all[j].id) {
                if (checked) S[len - 1].state = ST_CHECKED;
                continue;
            }
            if (len == L) continue;      /* keep scanning only for duplicates of kept ids */
            S[len].dist = all[j].dist; S[len].id = all[j].id;
            S[len].state = checked ? ST_CHECKED : ST_UNCHECKED;
            ++len;
        }
        s.merges++;
        if (rc == 1) break;
        if (staged && m < T) m = (2 * m < T) ? 2 * m : T;
    }
    emit(S, len, k, ids, dists);
    if (st) *st = s;
    free(visited); free(S); free(LS); free(LSlen); free(U); free(all);
    return rc;
}

/* ---------------------------------------------------------------- batch drivers */

/* algo: 0 = Algorithm 1, 1 = Top-M, 2 = Algorithm 3.  One query per OpenMP iteration;
 * queries are independent, so the thread count changes nothing but the time. */
int or_search_batch(int algo, const float *base, int64_t n, int d, int64_t ld, int metric,
                    const int32_t *adj, int R, int32_t entry_id, const float *queries, int64_t nq,
                    int64_t ldq, int k, int L, int M, int sync, int static_I, double rho, int staged,
                    int max_substeps, int32_t *ids, float *dists, or_stats *stats)
{
    int rc_all = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all)
    for (int64_t qi = 0; qi < nq; ++qi) {
        or_stats s;
        int rc;
        const float *q = row(queries, qi, ldq);
        if (algo == 0)
            rc = or_bfis(base, n, d, ld, metric, adj, R, entry_id, q, k, L, ids + qi * k, dists + qi * k, &s);
        else if (algo == 1)
            rc = or_topm(base, n, d, ld, metric, adj, R, entry_id, q, k, L, M, staged, ids + qi * k,
                         dists + qi * k, &s);
        else
            rc = or_speedann(base, n, d, ld, metric, adj, R, entry_id, q, k, L, M, sync, static_I, rho,
                             staged, max_substeps, ids + qi * k, dists + qi * k, &s);
        if (stats) stats[qi] = s;
        rc_all |= rc != 0 ? (rc < 0 ? 2 : 1) : 0;
    }
    return rc_all;
}

/* ---------------------------------------------------------------- graph construction */

/* mean of the rows listed in members (all rows when members is NULL), summed in index
 * order in double precision; then the member whose squared distance to that mean
 * (double precision, index order) is smallest, ties to the smaller id */
static int64_t medoid_of(const float *base, int64_t ld, int d, const int32_t *members, int64_t cnt)
{
    double *mean = (double *)calloc((size_t)d, sizeof(double));
    for (int64_t a = 0; a < cnt; ++a) {
        const float *x = row(base, members ? members[a] : a, ld);
        for (int i = 0; i < d; ++i) mean[i] += (double)x[i];
    }
    for (int i = 0; i < d; ++i) mean[i] /= (double)cnt;
    int64_t best = -1;
    double bestd = INFINITY;
    for (int64_t a = 0; a < cnt; ++a) {
        int64_t v = members ? members[a] : a;
        const float *x = row(base, v, ld);
        double acc = 0.0;
        for (int i = 0; i < d; ++i) { double t = (double)x[i] - mean[i]; acc += t * t; }
        if (acc < bestd || (acc == bestd && v < best)) { bestd = acc; best = v; }
    }
    free(mean);
    return best;
}

int64_t or_medoid(const float *base, int64_t n, int d, int64_t ld) { return medoid_of(base, ld, d, NULL, n); }

/* Row pruning.  cand: n x kc candidate ids of each vertex, sorted by key (distance to
 * the vertex, id).  prune 0: keep the first R.  prune 1 (relative-neighbourhood rule):
 * scan the candidates in order and keep c unless some already kept s has
 * d(s, c) < d(p, c), stopping at R kept.  adj: n x R, padded with -1. */
void or_prune(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *cand, int kc,
              int R, int prune, int32_t *adj)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; ++p) {
        int32_t *out = adj + p * R;
        int kept = 0;
        for (int j = 0; j < kc && kept < R; ++j) {
            int32_t c = cand[p * kc + j];
            if (c < 0) continue;
            int keep = 1;
            if (prune == 1) {
                float dpc = or_distance(row(base, p, ld), row(base, c, ld), d, metric);
                for (int a = 0; a < kept; ++a) {
                    float dsc = or_distance(row(base, out[a], ld), row(base, c, ld), d, metric);
                    if (dsc < dpc) { keep = 0; break; }
                }
            }
            if (keep) out[kept++] = c;
        }
        for (int j = kept; j < R; ++j) out[j] = -1;
    }
}

static int row_degree(const int32_t *adj, int R, int64_t v)
{
    int deg = 0;
    for (int r = 0; r < R; ++r) if (adj[v * R + r] >= 0) deg++;
    return deg;
}

/* breadth-first marking from src over the directed graph; returns newly marked count */
static int64_t mark_from(const int32_t *adj, int R, int64_t n, int32_t src, uint8_t *mark, int32_t *queue)
{
    if (mark[src]) return 0;
    int64_t head = 0, tail = 0, cnt = 0;
    mark[src] = 1; queue[tail++] = src; cnt++;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int r = 0; r < R; ++r) {
            int32_t u = adj[(int64_t)v * R + r];
            if (u < 0 || u >= n || mark[u]) continue;
            mark[u] = 1; queue[tail++] = u; cnt++;
        }
    }
    return cnt;
}

static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

/* Reverse edges: with the pruned graph as it stands, every vertex c appends to its row
 * the sources p of its in-edges (p -> c) that its row does not hold yet, in key order
 * (d(c, p), p), while the row has fewer than R entries.  All rows read the graph as it
 * was before any append.  Returns the number of edges added. */
int64_t or_reverse_edges(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj, int R)
{
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)R);
    memcpy(snap, adj, sizeof(int32_t) * (size_t)n * (size_t)R);
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t p = 0; p < n; ++p)
        for (int r = 0; r < R; ++r) if (snap[p * R + r] >= 0) start[snap[p * R + r] + 1]++;
    for (int64_t c = 0; c < n; ++c) start[c + 1] += start[c];
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(start[n] > 0 ? start[n] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t c = 0; c < n; ++c) fill[c] = start[c];
    for (int64_t p = 0; p < n; ++p)
        for (int r = 0; r < R; ++r) {
            int32_t c = snap[p * R + r];
            if (c >= 0) src[fill[c]++] = (int32_t)p;
        }
    int64_t added = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : added)
    for (int64_t c = 0; c < n; ++c) {
        int64_t cnt = start[c + 1] - start[c];
        if (cnt == 0) continue;
        int deg = 0;
        for (int r = 0; r < R; ++r) if (snap[c * R + r] >= 0) deg++;
        if (deg >= R) continue;
        entry *e = (entry *)malloc(sizeof(entry) * (size_t)cnt);
        for (int64_t a = 0; a < cnt; ++a) {
            int32_t p = src[start[c] + a];
            e[a].dist = or_distance(row(base, c, ld), row(base, p, ld), d, metric);
            e[a].id = p;
            e[a].state = 0;
        }
        sort_entries(e, cnt);
        for (int64_t a = 0; a < cnt && deg < R; ++a) {
            int dup = 0;
            for (int r = 0; r < deg; ++r) if (adj[c * R + r] == e[a].id) { dup = 1; break; }
            if (dup) continue;
            adj[c * R + deg] = e[a].id;
            deg++;
            added++;
        }
        free(e);
    }
    free(snap); free(start); free(src); free(fill);
    return added;
}

/* Connectivity repair, in three parts, all deterministic:
 *  (1) components: the weakly connected components of the pruned graph, numbered by
 *      their smallest member id; each gets a representative, its medoid;
 *  (2) gateway rows: every representative (keeping keep_local of its edges), the entry
 *      and the hubs - the `hubs` vertices nearest to the mean of all rows (double
 *      precision, key (distance, id)), representatives excepted (keeping hub_keep_local
 *      edges each) - get a new row: its first kept edges that are not links, then
 *      links to other representatives.  The links are chosen with the
 *      relative-neighbourhood rule over all other representatives in key order
 *      (distance to the source, id), up to R - kept of them, and the remaining slots
 *      are filled with the nearest representatives not yet linked.  Every row is
 *      computed from the graph as it was before this part;
 *  (3) reachability: in increasing id order, every vertex u not reachable from the entry
 *      gets an edge from the reachable vertex nearest to it (key (distance, id)) among
 *      those with a free slot; then everything reachable from u is marked.
 * Returns the number of edges added in (3), or -1 if (3) found no vertex with a free
 * slot.  ncomp_out receives the component count. */
int64_t or_repair(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj, int R,
                  int32_t entry_id, int keep_local, int hubs, int hub_keep_local, int64_t *ncomp_out)
{
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) par[i] = i;
    for (int64_t v = 0; v < n; ++v)
        for (int r = 0; r < R; ++r) {
            int32_t u = adj[v * R + r];
            if (u < 0) continue;
            int64_t a = uf_find(par, v), b = uf_find(par, u);
            if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
        }
    /* components in order of smallest member */
    int64_t *comp_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *root_comp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) root_comp[i] = -1;
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t rt = uf_find(par, i);
        if (root_comp[rt] < 0) root_comp[rt] = nc++;
        comp_of[i] = root_comp[rt];
    }
    if (ncomp_out) *ncomp_out = nc;
    int64_t *start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) start[comp_of[i] + 1]++;
    for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    for (int64_t c = 0; c < nc; ++c) fill[c] = start[c];
    for (int64_t i = 0; i < n; ++i) members[fill[comp_of[i]]++] = (int32_t)i;
    int32_t *rep = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
    for (int64_t c = 0; c < nc; ++c)
        rep[c] = (int32_t)medoid_of(base, ld, d, members + start[c], start[c + 1] - start[c]);

    /* (2) gateway rows: sources are the representatives, then the entry and the other
     * hubs (vertices nearest to the mean, representatives excepted) */
    uint8_t *is_rep = (uint8_t *)calloc((size_t)n, 1);
    for (int64_t c = 0; c < nc; ++c) is_rep[rep[c]] = 1;
    int64_t nhub = 0;
    int32_t *hub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(hubs > 0 ? hubs + 1 : 1));
    if (nc > 1) {
        if (!is_rep[entry_id]) hub[nhub++] = entry_id;
        if (hubs > 1) {
            double *mean = (double *)calloc((size_t)d, sizeof(double));
            for (int64_t v = 0; v < n; ++v)
                for (int i = 0; i < d; ++i) mean[i] += (double)row(base, v, ld)[i];
            for (int i = 0; i < d; ++i) mean[i] /= (double)n;
            /* the hubs smallest keys (distance to the mean, id) by repeated insertion */
            double *hd = (double *)malloc(sizeof(double) * (size_t)hubs);
            int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)hubs);
            int cnt = 0;
            for (int64_t v = 0; v < n; ++v) {
                if (is_rep[v] || v == entry_id) continue;
                double acc = 0.0;
                for (int i = 0; i < d; ++i) { double t = (double)row(base, v, ld)[i] - mean[i]; acc += t * t; }
                int limit = hubs - 1;
                if (cnt == limit && !(acc < hd[limit - 1] || (acc == hd[limit - 1] && v < hi[limit - 1]))) continue;
                int pos = cnt < limit ? cnt : limit - 1;
                while (pos > 0 && (acc < hd[pos - 1] || (acc == hd[pos - 1] && v < hi[pos - 1]))) {
                    hd[pos] = hd[pos - 1]; hi[pos] = hi[pos - 1]; --pos;
                }
                hd[pos] = acc; hi[pos] = (int32_t)v;
                if (cnt < limit) ++cnt;
            }
            for (int j = 0; j < cnt; ++j) hub[nhub++] = hi[j];
            free(mean); free(hd); free(hi);
        }
    }
    int64_t nsrc = nc > 1 ? nc + nhub : 0;
    int32_t *links = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsrc > 0 ? nsrc : 1) * (size_t)R);
    int *kept_local = (int *)malloc(sizeof(int) * (size_t)(nsrc > 0 ? nsrc : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < nsrc; ++a) {
        int32_t v = a < nc ? rep[a] : hub[a - nc];
        int kl = a < nc ? keep_local : hub_keep_local;
        int cap = R - kl;
        kept_local[a] = kl;
        int32_t *out = links + a * R;
        for (int x = 0; x < R; ++x) out[x] = -1;
        if (cap <= 0) continue;
        /* candidates: every other representative, sorted by key */
        entry *cand = (entry *)malloc(sizeof(entry) * (size_t)nc);
        int64_t ncand = 0;
        for (int64_t c = 0; c < nc; ++c) {
            if (rep[c] == v) continue;
            cand[ncand].dist = or_distance(row(base, v, ld), row(base, rep[c], ld), d, metric);
            cand[ncand].id = rep[c]; cand[ncand].state = 0;
            ++ncand;
        }
        sort_entries(cand, ncand);
        int kept = 0;
        for (int64_t j = 0; j < ncand && kept < cap; ++j) {
            int keep = 1;
            for (int x = 0; x < kept; ++x) {
                float dsc = or_distance(row(base, out[x], ld), row(base, cand[j].id, ld), d, metric);
                if (dsc < cand[j].dist) { keep = 0; break; }
            }
            if (keep) { out[kept++] = cand[j].id; cand[j].state = 1; }
        }
        for (int64_t j = 0; j < ncand && kept < cap; ++j)
            if (cand[j].state == 0) out[kept++] = cand[j].id;
        free(cand);
    }
    /* rewrite the rows: first kept edges not among the links, then the links */
    for (int64_t a = 0; a < nsrc; ++a) {
        int32_t v = a < nc ? rep[a] : hub[a - nc];
        int32_t *rw = adj + (int64_t)v * R;
        int32_t newrow[256];
        int cnt = 0;
        const int32_t *lk = links + a * R;
        for (int r = 0; r < R && cnt < kept_local[a]; ++r) {
            int32_t u = rw[r];
            if (u < 0) continue;
            int dup = 0;
            for (int x = 0; x < R; ++x) if (lk[x] == u) dup = 1;
            if (!dup) newrow[cnt++] = u;
        }
        for (int x = 0; x < R; ++x) if (lk[x] >= 0) newrow[cnt++] = lk[x];
        for (int r = 0; r < R; ++r) rw[r] = r < cnt ? newrow[r] : -1;
    }
    free(links); free(kept_local); free(hub); free(is_rep);

    /* (3) reachability */
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t added = 0;
    mark_from(adj, R, n, entry_id, mark, queue);
    for (int64_t u = 0; u < n; ++u) {
        if (mark[u]) continue;
        int64_t best = -1;
        float bestd = INFINITY;
        for (int64_t w = 0; w < n; ++w) {
            if (!mark[w] || row_degree(adj, R, w) >= R) continue;
            float dd = or_distance(row(base, w, ld), row(base, u, ld), d, metric);
            if (best < 0 || key_less(dd, (int32_t)w, bestd, (int32_t)best)) { bestd = dd; best = w; }
        }
        if (best < 0) { added = -1; break; }
        adj[best * R + row_degree(adj, R, best)] = (int32_t)u;
        added++;
        mark_from(adj, R, n, (int32_t)u, mark, queue);
    }
    free(mark); free(queue);
    free(par); free(comp_of); free(root_comp); free(start); free(members); free(fill); free(rep);
    return added;
}

/* number of vertices reachable from src */
int64_t or_reachable(const int32_t *adj, int R, int64_t n, int32_t src, uint8_t *mark_out)
{
    uint8_t *mark = mark_out ? mark_out : (uint8_t *)calloc((size_t)n, 1);
    if (mark_out) memset(mark_out, 0, (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t c = mark_from(adj, R, n, src, mark, queue);
    free(queue);
    if (!mark_out) free(mark);
    return c;
}

/* ---------------------------------------------------------------- reduced precision
 *
 * Storage formats, from their definitions (not part of the paper):
 *   OR_BF16  the upper half of the float32 pattern, rounded to nearest even; no scale
 *            (bf16 keeps float32's exponent range, so a scale would change nothing).
 *   OR_FP8   e4m3 with finite values only: sign, 4 exponent bits (bias 7), 3 mantissa
 *            bits; exponent field 0 holds subnormals m * 2^-9, the pattern S.1111.111 is
 *            not a number, so the largest value is 1.75 * 2^8 = 448.  Each vector gets the
 *            scale amax / 448 (1 for a zero vector); a coordinate is divided by it in
 *            float, rounded to nearest even and saturated at 448.
 * A stored coordinate stands for scale * value(code), computed in float (one rounding). */

#define OR_F32 0
#define OR_BF16 1
#define OR_FP8 2

static uint16_t bf16_encode(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);   /* nearest, ties to the even upper half */
    return (uint16_t)(b >> 16);
}

static float bf16_decode(uint16_t c)
{
    uint32_t b = (uint32_t)c << 16;
    float x;
    memcpy(&x, &b, 4);
    return x;
}

static uint8_t fp8_encode(float x)
{
    const uint8_t sign = signbit(x) ? 0x80 : 0x00;
    double a = fabs((double)x);
    if (!(a < 448.0)) return (uint8_t)(sign | 0x7E);   /* saturate (NaN included) */
    int e2;
    (void)frexp(a, &e2);   /* a = f * 2^e2, f in [0.5, 1) */
    int E = e2 - 1;        /* a in [2^E, 2^(E+1)) */
    if (a == 0.0 || E < -6) {
        double m = nearbyint(a / ldexp(1.0, -9));   /* subnormal units, ties to even */
        return (uint8_t)(sign | (uint8_t)m);         /* m == 8 is the smallest normal */
    }
    double m = nearbyint((a / ldexp(1.0, E) - 1.0) * 8.0);
    if (m == 8.0) { m = 0.0; E += 1; }
    if (E > 8 || (E == 8 && m > 6.0)) return (uint8_t)(sign | 0x7E);
    return (uint8_t)(sign | (uint8_t)((E + 7) << 3) | (uint8_t)m);
}

static float fp8_decode(uint8_t c)
{
    const int e = (c >> 3) & 0xF, m = c & 7;
    double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    if (e == 15 && m == 7) v = NAN;
    return (float)((c & 0x80) ? -v : v);
}

/* codes: n rows of d codes (2 bytes for bf16, 1 for fp8), dense; scale: n floats */
void or_quantize(const float *x, int64_t n, int d, int64_t ld, int dtype, void *codes, float *scale)
{
    for (int64_t i = 0; i < n; ++i) {
        const float *r = x + i * ld;
        if (dtype == OR_BF16) {
            uint16_t *c = (uint16_t *)codes + i * d;
            for (int j = 0; j < d; ++j) c[j] = bf16_encode(r[j]);
            scale[i] = 1.0f;
        } else {
            uint8_t *c = (uint8_t *)codes + i * d;
            float amax = 0.0f;
            for (int j = 0; j < d; ++j) amax = fmaxf(amax, fabsf(r[j]));
            const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
            for (int j = 0; j < d; ++j) c[j] = fp8_encode(r[j] / s);
            scale[i] = s;
        }
    }
}

/* the float32 values the codes stand for: out[i][j] = scale[i] * value(code) */
void or_dequantize(const void *codes, const float *scale, int64_t n, int d, int dtype, float *out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j) {
            const float v = dtype == OR_BF16 ? bf16_decode(((const uint16_t *)codes)[i * d + j])
                                             : fp8_decode(((const uint8_t *)codes)[i * d + j]);
            out[i * d + j] = dtype == OR_BF16 ? v : scale[i] * v;
        }
}

/* Exact re-rank: each query's candidate list cand[q][0..L) (-1 padded) gets its distances
 * recomputed on base (float32) and the first k by key are written out, (-1, +inf) padded. */
void or_rerank(const float *base, int d, int64_t ld, int metric, const float *queries, int64_t nq, int64_t ldq,
               const int32_t *cand, int L, int k, int32_t *ids, float *dists)
{
    entry *e = (entry *)malloc(sizeof(entry) * (size_t)(L > 0 ? L : 1));
    for (int64_t q = 0; q < nq; ++q) {
        int64_t cnt = 0;
        for (int j = 0; j < L; ++j) {
            const int32_t id = cand[q * L + j];
            if (id < 0) continue;
            e[cnt].dist = or_distance(queries + q * ldq, base + (int64_t)id * ld, d, metric);
            e[cnt].id = id;
            e[cnt].state = 0;
            cnt++;
        }
        qsort(e, (size_t)cnt, sizeof(entry), entry_cmp);
        emit(e, cnt, k, ids + q * k, dists + q * k);
    }
    free(e);
}
