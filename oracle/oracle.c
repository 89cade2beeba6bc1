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
 *   - the starting point counts as visited as soon as it is on the list (Algorithm 1
 *     puts it there without marking it);
 *   - a worker's update position is its best new entry's 0-based place after the cut to
 *     L, and L when nothing it added stayed or when it had nothing to expand;
 *   - how a global step splits the work: each worker's local list starts as a copy of S;
 *     the unchecked entries of S, in key order, are dealt to the workers in turn (the j-th
 *     to worker j mod m), and in a worker's copy the entries dealt to others are FOREIGN
 *     (they keep their places, that worker never expands them);
 *   - merging: one entry per vertex from S and every local list, checked if any copy
 *     is, the L best kept;
 *   - the schedule is consulted after every round of local steps; the number of active
 *     workers doubles up to T, never past it.
 *
 * Pins: tests/test_oracle.py (exact kNN when L covers the reachable set, one worker is
 * Algorithm 1, merging after every local step is Top-M, CheckMetrics with ratio 0 merges
 * every step and above 1 never, static schedules and the step limit on hand-derived
 * traces under tests/golden/, exact kNN against a brute force in numpy).
 *
 * Trace: or_search_batch_traced also records, per query, the expansions, the entries they
 * added and the smallest relative gap between neighbouring keys that any decision of the
 * search depended on; tests use it to tell a disagreement caused by rounding (keys within
 * the tolerance) from a wrong step.
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
    int64_t flags;          /* 1: stopped by the step limit (Algorithm 3 only) */
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

/* ---------------------------------------------------------------- search: common parts */

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

/* Optional record of one query's search, for explaining a disagreement with another
 * implementation of it.  Every decision a search takes is an order between keys, so the
 * smallest relative gap between two keys of distinct vertices that stand next to each
 * other in a sorted list, within the first L + 1 places (the ones that decide what is
 * kept, expanded and reported), bounds how far a distance may move before some decision
 * can change.  The expansions and the entries each of them added are listed too. */
typedef struct {
    double min_gap;        /* |a - b| / max(|a|, |b|) of that pair; +inf if there was none */
    int64_t gap_step;      /* local step after which the pair was seen (0: none yet) */
    float gap_dist[2];     /* the pair's keys */
    int32_t gap_id[2];
    int64_t n_exp;         /* expansions, and entries they added: every one counts, */
    int64_t n_keys;        /* even past the capacity of the lists below */
} or_trace;

typedef struct {
    or_trace *t;           /* NULL: nothing is recorded */
    int32_t *exp;          /* 4 ints per expansion: local step, worker, vertex, entries added */
    float *key_dist;       /* the entries added, in order */
    int32_t *key_id;
    int64_t cap_exp, cap_keys;
} tracer;

/* What a search keeps besides its lists: the visited map (one byte per vertex: its distance
 * has been computed), the counters and the trace. */
typedef struct {
    problem P;
    uint8_t *visited;
    or_stats st;
    tracer tr;
} search_ctx;

static int ctx_open(search_ctx *c, const problem *P, const tracer *tr)
{
    c->P = *P;
    memset(&c->st, 0, sizeof(c->st));
    if (tr) c->tr = *tr;
    else memset(&c->tr, 0, sizeof(c->tr));
    if (c->tr.t) {
        memset(c->tr.t, 0, sizeof(*c->tr.t));
        c->tr.t->min_gap = INFINITY;
        c->tr.t->gap_id[0] = c->tr.t->gap_id[1] = -1;
    }
    c->visited = (uint8_t *)calloc((size_t)P->n, 1);
    return c->visited ? 0 : -2;
}

/* The list starts with the entry point alone, unchecked; the entry point counts as
 * visited from the start (a reading: the paper adds it without marking it). */
static int64_t put_start(search_ctx *c, entry *list, int32_t v)
{
    list[0].dist = pdist(&c->P, v);
    list[0].id = v;
    list[0].state = ST_UNCHECKED;
    c->visited[v] = 1;
    c->st.dist_comps = 1;
    return 1;
}

/* Expanding v: each neighbour of v that is not visited yet, in the order of its row,
 * becomes visited, gets its distance and is appended to the list as unchecked.  Returns
 * how many were appended. */
static int64_t expand(search_ctx *c, int32_t v, entry *list, int64_t *len, int64_t step, int worker)
{
    const int64_t before = *len;
    const int R = c->P.R;
    c->st.expansions++;
    for (int r = 0; r < R; ++r) {
        const int32_t u = c->P.adj[(int64_t)v * R + r];
        if (u < 0 || c->visited[u]) continue;
        c->visited[u] = 1;
        c->st.dist_comps++;
        list[*len].dist = pdist(&c->P, u);
        list[*len].id = u;
        list[*len].state = ST_UNCHECKED;
        ++*len;
    }
    const int64_t added = *len - before;
    or_trace *t = c->tr.t;
    if (t) {
        if (t->n_exp < c->tr.cap_exp) {
            int32_t *e = c->tr.exp + 4 * t->n_exp;
            e[0] = (int32_t)step; e[1] = worker; e[2] = v; e[3] = (int32_t)added;
        }
        t->n_exp++;
        for (int64_t a = 0; a < added; ++a, t->n_keys++)
            if (t->n_keys < c->tr.cap_keys) {
                c->tr.key_dist[t->n_keys] = list[before + a].dist;
                c->tr.key_id[t->n_keys] = list[before + a].id;
            }
    }
    return added;
}

static void note_gaps(search_ctx *c, const entry *list, int64_t len, int L, int64_t step)
{
    or_trace *t = c->tr.t;
    if (!t) return;
    for (int64_t j = 0; j + 1 < len && j < L; ++j) {
        if (list[j].id == list[j + 1].id) continue;
        const double a = list[j].dist, b = list[j + 1].dist;
        const double scale = fmax(fabs(a), fabs(b));
        const double gap = scale > 0.0 ? fabs(b - a) / scale : 0.0;
        if (gap < t->min_gap) {
            t->min_gap = gap;
            t->gap_step = step;
            t->gap_dist[0] = list[j].dist; t->gap_id[0] = list[j].id;
            t->gap_dist[1] = list[j + 1].dist; t->gap_id[1] = list[j + 1].id;
        }
    }
}

/* Orders list[0..len) by key and keeps its first L entries; returns the new length. */
static int64_t order_and_cut(search_ctx *c, entry *list, int64_t len, int L, int64_t step)
{
    sort_entries(list, len);
    note_gaps(c, list, len, L, step);
    return len > L ? L : len;
}

static int64_t first_unchecked(const entry *list, int64_t len)
{
    for (int64_t j = 0; j < len; ++j)
        if (list[j].state == ST_UNCHECKED) return j;
    return -1;
}

/* ---------------------------------------------------------------- Algorithm 1 */

/* Best-first search: the list keeps the L best vertices seen so far; each step expands the
 * best one not expanded yet, until none is left. */
static int bfis_run(const problem *P, const tracer *tr, int32_t entry_id, int k, int L, int32_t *ids, float *dists,
                    or_stats *st)
{
    search_ctx c;
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)(L + P->R));
    if (ctx_open(&c, P, tr) != 0 || !S) { free(c.visited); free(S); return -2; }
    int64_t len = put_start(&c, S, entry_id);
    for (;;) {
        const int64_t i = first_unchecked(S, len);
        if (i < 0) break;
        S[i].state = ST_CHECKED;
        c.st.global_steps++;
        c.st.substeps++;
        expand(&c, S[i].id, S, &len, c.st.substeps, 0);
        len = order_and_cut(&c, S, len, L, c.st.substeps);
    }
    emit(S, len, k, ids, dists);
    if (st) *st = c.st;
    free(c.visited); free(S);
    return 0;
}

int or_bfis(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
            int32_t entry_id, const float *q, int k, int L, int32_t *ids, float *dists, or_stats *st)
{
    const problem P = {base, n, ld, d, metric, adj, R, q};
    return bfis_run(&P, NULL, entry_id, k, L, ids, dists, st);
}

/* ---------------------------------------------------------------- Top-M (Sec. 4.1) */

/* Each step expands the m best unchecked candidates together (all of them when there are
 * fewer), adds the union of their new neighbours and keeps the L best.  The neighbours are
 * taken in the order (candidate in list order, position in its row).  staged: m is 1 at
 * the first step and doubles after every step up to M (Sec. 4.2 with t = 1). */
static int topm_run(const problem *P, const tracer *tr, int32_t entry_id, int k, int L, int M, int staged,
                    int32_t *ids, float *dists, or_stats *st)
{
    search_ctx c;
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)(L + (int64_t)M * P->R));
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    if (ctx_open(&c, P, tr) != 0 || !S || !act) { free(c.visited); free(S); free(act); return -2; }
    int64_t len = put_start(&c, S, entry_id);
    int m = staged ? 1 : M;
    for (;;) {
        int na = 0;
        for (int64_t j = 0; j < len && na < m; ++j)
            if (S[j].state == ST_UNCHECKED) { S[j].state = ST_CHECKED; act[na++] = S[j].id; }
        if (na == 0) break;
        c.st.global_steps++;
        c.st.substeps++;
        c.st.merges++;
        for (int a = 0; a < na; ++a) expand(&c, act[a], S, &len, c.st.substeps, a);
        len = order_and_cut(&c, S, len, L, c.st.substeps);
        if (staged && m < M) m = (2 * m < M) ? 2 * m : M;
    }
    emit(S, len, k, ids, dists);
    if (st) *st = c.st;
    free(c.visited); free(S); free(act);
    return 0;
}

int or_topm(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
            int32_t entry_id, const float *q, int k, int L, int M, int staged, int32_t *ids, float *dists,
            or_stats *st)
{
    const problem P = {base, n, ld, d, metric, adj, R, q};
    return topm_run(&P, NULL, entry_id, k, L, M, staged, ids, dists, st);
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

/* Whether the workers merge after the local step just taken, the local_steps-th of this
 * global step: after every one (bsp), after static_I of them (static; static_I <= 0:
 * never, so only when no worker has work left), or when CheckMetrics says so (adaptive). */
static int merge_due(int sync, int static_I, double rho, const int32_t *U, int m, int L, int local_steps)
{
    if (sync == OR_SYNC_BSP) return 1;
    if (sync == OR_SYNC_STATIC) return static_I > 0 && local_steps >= static_I;
    return check_metrics(U, m, L, rho);
}

/* The start of a global step (a reading of how Algorithm 3 splits the work): the unchecked
 * entries of S, in key order, are dealt to the m workers in turn, the j-th to worker
 * j mod m.  Each worker's local list is a copy of S in which the entries dealt to the
 * others are FOREIGN: they keep their places but that worker never expands them.  Returns
 * the number of unchecked entries dealt. */
static int64_t deal(const entry *S, int64_t len, int m, entry *LS, int64_t stride, int64_t *LSlen)
{
    int64_t dealt = 0;
    for (int t = 0; t < m; ++t) LSlen[t] = len;
    for (int64_t j = 0; j < len; ++j) {
        const int owner = S[j].state == ST_UNCHECKED ? (int)(dealt++ % m) : -1;
        for (int t = 0; t < m; ++t) {
            entry e = S[j];
            if (e.state == ST_UNCHECKED && owner != t) e.state = ST_FOREIGN;
            LS[(int64_t)t * stride + j] = e;
        }
    }
    return dealt;
}

/* One local step of one worker: it expands the first entry of its own list that it may
 * expand, adds what it found and keeps the L best.  Returns its update position (Sec. 4.3:
 * the 0-based place of the best entry this step added, after the cut), or L when it had
 * nothing to expand or nothing it added stayed (readings). */
static int32_t local_step(search_ctx *c, entry *list, int64_t *len, int L, int worker)
{
    const int64_t i = first_unchecked(list, *len);
    if (i < 0) return L;
    list[i].state = ST_CHECKED;
    const int64_t before = *len;
    const int64_t added = expand(c, list[i].id, list, len, c->st.substeps, worker);
    if (added == 0) return L;
    entry *fresh = (entry *)malloc(sizeof(entry) * (size_t)added);
    memcpy(fresh, list + before, sizeof(entry) * (size_t)added);
    *len = order_and_cut(c, list, *len, L, c->st.substeps);
    int32_t U = L;
    for (int64_t j = 0; j < *len && U == L; ++j)
        for (int64_t x = 0; x < added; ++x)
            if (fresh[x].id == list[j].id) { U = (int32_t)j; break; }
    free(fresh);
    return U;
}

/* The merge (Algorithm 3): S and the m local lists become one list with one entry per
 * vertex, checked if any copy is (FOREIGN counts as unchecked), in key order, cut to L.
 * all: room for every entry of S and of the lists.  Returns the new length of S. */
static int64_t merge_into(search_ctx *c, entry *S, int64_t len, const entry *LS, int64_t stride,
                          const int64_t *LSlen, int m, entry *all, int L)
{
    int64_t na = 0;
    for (int64_t j = 0; j < len; ++j) all[na++] = S[j];
    for (int t = 0; t < m; ++t)
        for (int64_t j = 0; j < LSlen[t]; ++j) all[na++] = LS[(int64_t)t * stride + j];
    sort_entries(all, na);
    /* copies of one vertex carry one key, so they sit together */
    int64_t nd = 0;
    for (int64_t j = 0; j < na; ++j) {
        const int checked = all[j].state == ST_CHECKED;
        if (nd > 0 && all[nd - 1].id == all[j].id) {
            if (checked) all[nd - 1].state = ST_CHECKED;
            continue;
        }
        all[nd] = all[j];
        all[nd].state = checked ? ST_CHECKED : ST_UNCHECKED;
        ++nd;
    }
    note_gaps(c, all, nd, L, c->st.substeps);
    const int64_t keep = nd > L ? L : nd;
    memcpy(S, all, sizeof(entry) * (size_t)keep);
    return keep;
}

/* Speed-ANN with T workers, run in lockstep: within a global step every worker with work
 * takes one local step per round, in worker order, against one shared visited set, so that
 * a vertex two workers reach in the same round goes to the lower worker (and, within a
 * worker, the earlier row position).  After each round the schedule decides whether the
 * workers merge; they also merge when none has work left.  staged: the number of active
 * workers starts at 1 and doubles after each merge, up to T (Algorithm 3); otherwise it is
 * T throughout.  max_substeps > 0 (not in the paper): when that many local steps have been
 * taken in all, the global step in progress merges and the search ends (stats flag 1,
 * return value 1). */
static int speedann_run(const problem *P, const tracer *tr, int32_t entry_id, int k, int L, int T, int sync,
                        int static_I, double rho, int staged, int max_substeps, int32_t *ids, float *dists,
                        or_stats *st)
{
    search_ctx c;
    const int64_t stride = L + P->R;
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)L);
    entry *LS = (entry *)malloc(sizeof(entry) * (size_t)T * (size_t)stride);
    int64_t *LSlen = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    entry *all = (entry *)malloc(sizeof(entry) * (size_t)(T + 1) * (size_t)L);
    if (ctx_open(&c, P, tr) != 0 || !S || !LS || !LSlen || !U || !all) {
        free(c.visited); free(S); free(LS); free(LSlen); free(U); free(all);
        return -2;
    }
    int64_t len = put_start(&c, S, entry_id);
    int m = staged ? 1 : T;
    int ended = 0;
    while (!ended) {
        if (deal(S, len, m, LS, stride, LSlen) == 0) break;
        c.st.global_steps++;
        int local_steps = 0;
        for (;;) {
            int busy = 0;
            for (int t = 0; t < m && !busy; ++t) busy = first_unchecked(LS + (int64_t)t * stride, LSlen[t]) >= 0;
            if (!busy) break;
            if (max_substeps > 0 && c.st.substeps >= max_substeps) {
                ended = 1;
                c.st.flags |= 1;
                break;
            }
            c.st.substeps++;
            local_steps++;
            for (int t = 0; t < m; ++t) U[t] = local_step(&c, LS + (int64_t)t * stride, &LSlen[t], L, t);
            if (merge_due(sync, static_I, rho, U, m, L, local_steps)) break;
        }
        len = merge_into(&c, S, len, LS, stride, LSlen, m, all, L);
        c.st.merges++;
        if (staged && m < T) m = (2 * m < T) ? 2 * m : T;
    }
    emit(S, len, k, ids, dists);
    if (st) *st = c.st;
    free(c.visited); free(S); free(LS); free(LSlen); free(U); free(all);
    return ended;
}

int or_speedann(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
                int32_t entry_id, const float *q, int k, int L, int T, int sync, int static_I, double rho,
                int staged, int max_substeps, int32_t *ids, float *dists, or_stats *st)
{
    const problem P = {base, n, ld, d, metric, adj, R, q};
    return speedann_run(&P, NULL, entry_id, k, L, T, sync, static_I, rho, staged, max_substeps, ids, dists, st);
}

/* ---------------------------------------------------------------- batch drivers */

/* algo: 0 = Algorithm 1, 1 = Top-M, 2 = Algorithm 3.  One query per OpenMP iteration (a
 * single query runs on the calling thread alone); queries are independent, so the thread
 * count changes nothing but the time.  traces
 * (NULL: none) gets one or_trace per query, with cap_exp expansions (4 ints each) and
 * cap_keys added entries per query in texp, tkd and tki. */
int or_search_batch_traced(int algo, const float *base, int64_t n, int d, int64_t ld, int metric,
                           const int32_t *adj, int R, int32_t entry_id, const float *queries, int64_t nq,
                           int64_t ldq, int k, int L, int M, int sync, int static_I, double rho, int staged,
                           int max_substeps, int32_t *ids, float *dists, or_stats *stats, or_trace *traces,
                           int32_t *texp, float *tkd, int32_t *tki, int64_t cap_exp, int64_t cap_keys)
{
    int rc_all = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all) if (nq > 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
        or_stats s;
        int rc;
        const problem P = {base, n, ld, d, metric, adj, R, row(queries, qi, ldq)};
        tracer tr = {0};
        if (traces) {
            tr.t = traces + qi;
            tr.exp = texp + qi * 4 * cap_exp;
            tr.key_dist = tkd + qi * cap_keys;
            tr.key_id = tki + qi * cap_keys;
            tr.cap_exp = cap_exp;
            tr.cap_keys = cap_keys;
        }
        if (algo == 0)
            rc = bfis_run(&P, &tr, entry_id, k, L, ids + qi * k, dists + qi * k, &s);
        else if (algo == 1)
            rc = topm_run(&P, &tr, entry_id, k, L, M, staged, ids + qi * k, dists + qi * k, &s);
        else
            rc = speedann_run(&P, &tr, entry_id, k, L, M, sync, static_I, rho, staged, max_substeps, ids + qi * k,
                              dists + qi * k, &s);
        if (stats) stats[qi] = s;
        rc_all |= rc != 0 ? (rc < 0 ? 2 : 1) : 0;
    }
    return rc_all;
}

int or_search_batch(int algo, const float *base, int64_t n, int d, int64_t ld, int metric,
                    const int32_t *adj, int R, int32_t entry_id, const float *queries, int64_t nq,
                    int64_t ldq, int k, int L, int M, int sync, int static_I, double rho, int staged,
                    int max_substeps, int32_t *ids, float *dists, or_stats *stats)
{
    return or_search_batch_traced(algo, base, n, d, ld, metric, adj, R, entry_id, queries, nq, ldq, k, L, M, sync,
                                  static_I, rho, staged, max_substeps, ids, dists, stats, NULL, NULL, NULL, NULL, 0,
                                  0);
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
