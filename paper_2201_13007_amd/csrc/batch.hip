// Batches of queries with uneven (L, k, M): the plan, its device arrays, the launches
// (capturable in a HIP graph) and the autotuner.  Contracts are in include/speedann.h.
//
// Queries are grouped into classes by walker count M (the general kernel runs M
// wavefronts per workgroup) and by the register-queue size the kernels are compiled for
// (ceil(L / 64) slots per lane, rounded up to 1-8 or 16 for one walker and to 1, 2, 4,
// 6, 8 or 16 for more).  A class is one
// launch with one workgroup per query; it takes its queries longest L first, so the
// hardware dispatcher, which hands out workgroups in index order as slots free up, runs
// the long searches first and the short ones fill the tail.  Classes are spread over up
// to eight streams, longest class first onto the least loaded stream; a run forks them
// from the caller's stream and joins them back with events, so a graph captured from
// that stream holds every class as a parallel branch.
//
// A class runs in one of two forms: one workgroup per query (the hardware dispatcher is
// the work queue), or persistent: as many workgroups as the device holds at once, each
// taking the class's queries from a device counter in the same longest-first order and
// reusing its own visited-set region (a loop around the search costs registers, so
// neither form wins everywhere).  The autotuner times the choices that leave every
// result unchanged: per class the form and the LDS visited table (none, the default, or
// 4096 / 16384 slots where they fit; a table also moves two walkers that merge every step
// out of their shared wavefront into one wavefront each), each class alone; then the
// number of streams (1, 2, 4, 8) for three plans: every class one workgroup per query,
// every class persistent, and each class in its own fastest form; the fastest plan and
// stream count are kept.
#include "sa_internal.h"

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

namespace sa {
namespace {

constexpr int MAX_STREAMS = 8;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ni_bucket(int L, int M) { return queue_slots_bucket(L, M); }

struct BatchClass {
    int32_t M, ni, Lmax, kmax;
    int64_t n, first;        // its queries are order[first .. first + n)
    double cost;             // sum of L over its queries: the scheduling weight
    int32_t glog2;           // workspace table size (log2), fixed by Lmax and M
    int32_t lds;             // lds_hash_slots given to the search: 0 default, -1 none
    int32_t persistent;      // 1: a resident grid takes the queries from a device counter
    size_t region_bytes, ws_off;
    int stream;
};

}  // namespace
}  // namespace sa

using namespace sa;

struct sa_batch {
    const sa_index *ix;
    int64_t nq;
    sa_search_params p;
    std::vector<int32_t> L, k, M, order;
    std::vector<BatchClass> cls;
    int32_t kmax;
    int nstreams;
    hipStream_t streams[MAX_STREAMS];
    hipEvent_t fork, join[MAX_STREAMS];
    size_t off_L, off_k, off_order, off_ctr, ws_bytes;   // off_ctr: two int32 job counters per class
    std::string tuning;      // JSON of the last tuning run
};

namespace {

// The LDS visited-table settings the tuner tries for a class (lds_hash_slots values; the
// caller's own when it set one): the default and none, and tables of 4096 and 16384 slots
// where they fit; none for one walker, whose single-worker kernel keeps its table in the
// workspace.  Settings that give the same table are tried once.
std::vector<int32_t> lds_candidates(const sa_index *ix, const sa_search_params &p, int32_t Lmax, int32_t M)
{
    if (p.lds_hash_slots != 0) return {p.lds_hash_slots};
    if (M == 1) return {0};
    std::vector<int32_t> out, seen;
    for (int32_t v : {0, -1, 4096, 16384}) {
        sa_search_params q = p;
        q.lds_hash_slots = v;
        int32_t llog2, glog2;
        search_table_log2(q, Lmax, M, ix->R, &llog2, &glog2);
        if (llog2 > 0 && ((int64_t(1) << llog2) / 2 < (int64_t)M * ix->R + 1 ||
                          search_lds_bytes(Lmax, M, llog2, ix->d) > 160u * 1024u))
            continue;
        if (std::find(seen.begin(), seen.end(), llog2) != seen.end()) continue;
        seen.push_back(llog2);
        out.push_back(v);
    }
    return out;
}

// whether lds_hash_slots = v gives one of the tables lds_candidates lists
bool lds_allowed(const sa_index *ix, const sa_search_params &p, int32_t Lmax, int32_t M, int32_t v)
{
    auto table = [&](int32_t x) {
        sa_search_params q = p;
        q.lds_hash_slots = x;
        int32_t llog2, glog2;
        search_table_log2(q, Lmax, M, ix->R, &llog2, &glog2);
        return llog2;
    };
    const int32_t t = table(v);
    for (int32_t c : lds_candidates(ix, p, Lmax, M))
        if (table(c) == t) return true;
    return false;
}

// longest class first onto the least loaded of n streams
void assign_streams(sa_batch *b, int n)
{
    std::vector<size_t> idx(b->cls.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return b->cls[a].cost > b->cls[c].cost; });
    std::vector<double> load(n, 0.0);
    for (size_t i : idx) {
        int s = 0;
        for (int t = 1; t < n; ++t)
            if (load[t] < load[s]) s = t;
        b->cls[i].stream = s;
        load[s] += b->cls[i].cost;
    }
    b->nstreams = n;
}

int launch_class(const sa_batch *b, size_t ci, const float *queries, int64_t ldq, int32_t *ids, float *dists,
                 int64_t ldo, sa_query_stats *stats, unsigned char *ws, hipStream_t s)
{
    const BatchClass &c = b->cls[ci];
    const sa_index *ix = b->ix;
    SearchLaunch a;
    a.codes = ix->codes; a.scale = ix->scale; a.ldc = ix->ldc; a.dtype = ix->dtype;
    a.vec32 = ix->vec32; a.ld32 = ix->ld32;
    a.n = ix->n; a.d = ix->d; a.metric = ix->metric;
    a.adj = ix->adj; a.R = ix->R; a.entry = ix->entry; a.id_map = ix->id_map;
    a.int_lo = ix->int_lo; a.int_hi = ix->int_hi;
    a.queries = queries; a.ldq = ldq; a.nq = c.n; a.k = c.kmax; a.L = c.Lmax; a.M = c.M;
    a.p = b->p;
    a.p.lds_hash_slots = c.lds;
    a.ids = ids; a.dists = dists; a.stats = stats;
    a.workspace = ws + c.ws_off; a.ws_bytes = c.region_bytes * (size_t)c.n;
    a.qL = reinterpret_cast<const int32_t *>(ws + b->off_L);
    a.qk = reinterpret_cast<const int32_t *>(ws + b->off_k);
    a.order = reinterpret_cast<const int32_t *>(ws + b->off_order) + c.first;
    a.ldo = ldo;
    a.jobctr = c.persistent ? reinterpret_cast<int32_t *>(ws + b->off_ctr) + 2 * ci : nullptr;
    return launch_search(a, s);
}

int run_batch(const sa_batch *b, const float *queries, int64_t ldq, int32_t *ids, float *dists, int64_t ldo,
              sa_query_stats *stats, void *workspace, hipStream_t s)
{
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    if (b->nstreams <= 1) {
        for (size_t i = 0; i < b->cls.size(); ++i) {
            const int rc = launch_class(b, i, queries, ldq, ids, dists, ldo, stats, ws, s);
            if (rc != SA_OK) return rc;
        }
        return SA_OK;
    }
    SA_HIP(hipEventRecord(b->fork, s));
    for (int t = 0; t < b->nstreams; ++t) SA_HIP(hipStreamWaitEvent(b->streams[t], b->fork, 0));
    // longest class first on each stream
    std::vector<size_t> idx(b->cls.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return b->cls[a].cost > b->cls[c].cost; });
    for (size_t i : idx) {
        const int rc = launch_class(b, i, queries, ldq, ids, dists, ldo, stats, ws, b->streams[b->cls[i].stream]);
        if (rc != SA_OK) return rc;
    }
    for (int t = 0; t < b->nstreams; ++t) {
        SA_HIP(hipEventRecord(b->join[t], b->streams[t]));
        SA_HIP(hipStreamWaitEvent(s, b->join[t], 0));
    }
    return SA_OK;
}

int check_run(const sa_batch *b, const float *queries, int64_t ldq, int32_t *ids, float *dists, int64_t ldo,
              void *workspace, size_t ws_bytes)
{
    int rc;
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if ((rc = check_matrix(queries, b->nq, b->ix->d, ldq, "queries")) != SA_OK) return rc;
    if (b->nq > 0 && (!ids || !dists)) return set_error(SA_EINVAL, "output is NULL");
    if (ldo < b->kmax) return set_error(SA_EINVAL, "ldo=%lld is below the largest k (%d)", (long long)ldo, b->kmax);
    if (ws_bytes < b->ws_bytes)
        return set_error(SA_ECAPACITY, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes,
                         b->ws_bytes);
    if (b->ws_bytes > 0 && (!workspace || ((uintptr_t)workspace & 255u) != 0))
        return set_error(SA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    return check_device();
}

}  // namespace

extern "C" {

int sa_batch_create(const sa_index *index, int64_t nq, const int32_t *L, const int32_t *k, const int32_t *M,
                    const sa_search_params *params, sa_batch **out)
{
    if (!out) return set_error(SA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!index) return set_error(SA_EINVAL, "index is NULL");
    if (nq < 0 || nq > 0x7FFFFFFF) return set_error(SA_EINVAL, "nq=%lld out of range", (long long)nq);
    if (nq > 0 && (!L || !k || !M)) return set_error(SA_EINVAL, "L, k and M must be given for every query");
    sa_search_params p;
    if (params) p = *params;
    else sa_default_params(&p);
    int rc;
    for (int64_t q = 0; q < nq; ++q)
        if ((rc = check_search(index, 1, k[q], L[q], M[q], p)) != SA_OK)
            return set_error(rc, "query %lld: %s", (long long)q, sa_last_error());

    sa_batch *b = new sa_batch();
    b->ix = index;
    b->nq = nq;
    b->p = p;
    b->L.assign(L, L + nq);
    b->k.assign(k, k + nq);
    b->M.assign(M, M + nq);
    b->kmax = 1;
    for (int64_t q = 0; q < nq; ++q) b->kmax = std::max(b->kmax, k[q]);

    // classes by (M, register-queue size); within a class, longest L first
    std::vector<int32_t> idx(nq);
    for (int64_t q = 0; q < nq; ++q) idx[q] = (int32_t)q;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t c) {
        if (M[a] != M[c]) return M[a] < M[c];
        const int na = ni_bucket(L[a], M[a]), nc = ni_bucket(L[c], M[c]);
        if (na != nc) return na < nc;
        return L[a] > L[c];
    });
    b->order = idx;
    size_t off = 0;
    b->off_L = off; off = align256(off + 4 * (size_t)nq);
    b->off_k = off; off = align256(off + 4 * (size_t)nq);
    b->off_order = off; off = align256(off + 4 * (size_t)nq);
    int64_t ncls = 0;
    for (int64_t i = 0; i < nq; ++i)
        ncls += i == 0 || M[idx[i]] != M[idx[i - 1]] || ni_bucket(L[idx[i]], M[idx[i]]) != ni_bucket(L[idx[i - 1]], M[idx[i - 1]]);
    b->off_ctr = off; off = align256(off + 8 * (size_t)ncls);
    for (int64_t i = 0; i < nq;) {
        const int32_t q0 = idx[i];
        BatchClass c{};
        c.M = M[q0];
        c.ni = ni_bucket(L[q0], M[q0]);
        c.first = i;
        c.Lmax = 0;
        c.kmax = 0;
        c.cost = 0;
        int64_t j = i;
        while (j < nq && M[idx[j]] == c.M && ni_bucket(L[idx[j]], c.M) == c.ni) {
            c.Lmax = std::max(c.Lmax, L[idx[j]]);
            c.kmax = std::max(c.kmax, k[idx[j]]);
            c.cost += L[idx[j]];
            ++j;
        }
        c.n = j - i;
        c.lds = p.lds_hash_slots;
        c.persistent = 0;
        // every query of the class gets the table its largest L takes; the region fits the
        // largest of the tables the tuner may choose
        int32_t llog2, glog2;
        search_table_log2(p, c.Lmax, c.M, index->R, &llog2, &glog2);
        c.glog2 = glog2;
        c.region_bytes = 0;
        for (int32_t v : lds_candidates(index, p, c.Lmax, c.M)) {
            sa_search_params q = p;
            q.lds_hash_slots = v;
            c.region_bytes = std::max(c.region_bytes, search_workspace_bytes(1, c.Lmax, c.M, q, index->R));
        }
        c.ws_off = off;
        off = align256(off + c.region_bytes * (size_t)c.n);
        b->cls.push_back(c);
        i = j;
    }
    b->ws_bytes = nq > 0 ? off : 0;

    hipError_t e = hipSuccess;
    for (int t = 0; t < MAX_STREAMS && e == hipSuccess; ++t) {
        e = hipStreamCreateWithFlags(&b->streams[t], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[t], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        sa_batch_destroy(b);
        return hip_fail(e, "batch streams");
    }
    assign_streams(b, 1);
    *out = b;
    return SA_OK;
}

size_t sa_batch_workspace_bytes(const sa_batch *b) { return b ? b->ws_bytes : 0; }

int sa_batch_upload(const sa_batch *b, void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if (ws_bytes < b->ws_bytes)
        return set_error(SA_ECAPACITY, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes,
                         b->ws_bytes);
    if (b->nq == 0) return SA_OK;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0)
        return set_error(SA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    int rc;
    if ((rc = check_device()) != SA_OK) return rc;
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t n4 = 4 * (size_t)b->nq;
    SA_HIP(hipMemcpyAsync(ws + b->off_L, b->L.data(), n4, hipMemcpyHostToDevice, s));
    SA_HIP(hipMemcpyAsync(ws + b->off_k, b->k.data(), n4, hipMemcpyHostToDevice, s));
    SA_HIP(hipMemcpyAsync(ws + b->off_order, b->order.data(), n4, hipMemcpyHostToDevice, s));
    SA_HIP(hipStreamSynchronize(s));
    return SA_OK;
}

int sa_batch_run(const sa_batch *b, const float *queries_dev, int64_t ldq, int32_t *ids_dev, float *dists_dev,
                 int64_t ldo, sa_query_stats *stats_dev, void *workspace, size_t ws_bytes, void *hip_stream)
{
    int rc;
    if ((rc = check_run(b, queries_dev, ldq, ids_dev, dists_dev, ldo, workspace, ws_bytes)) != SA_OK) return rc;
    return run_batch(b, queries_dev, ldq, ids_dev, dists_dev, ldo, stats_dev, workspace, (hipStream_t)hip_stream);
}

int sa_batch_tune(sa_batch *b, const float *queries_dev, int64_t ldq, int32_t *ids_dev, float *dists_dev,
                  int64_t ldo, void *workspace, size_t ws_bytes, int32_t reps, void *hip_stream)
{
    int rc;
    if ((rc = check_run(b, queries_dev, ldq, ids_dev, dists_dev, ldo, workspace, ws_bytes)) != SA_OK) return rc;
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipEvent_t e0, e1;
    SA_HIP(hipEventCreate(&e0));
    SA_HIP(hipEventCreate(&e1));
    // best of reps after one warm run, in ms
    auto timed = [&](auto enqueue, float *best) -> int {
        int r = enqueue();
        *best = 1e30f;
        for (int i = 0; i < reps && r == SA_OK; ++i) {
            hipError_t he = hipEventRecord(e0, s);
            if (he == hipSuccess) r = enqueue();
            if (he == hipSuccess && r == SA_OK) he = hipEventRecord(e1, s);
            if (he == hipSuccess && r == SA_OK) he = hipEventSynchronize(e1);
            float t = 0.f;
            if (he == hipSuccess && r == SA_OK) he = hipEventElapsedTime(&t, e0, e1);
            if (he != hipSuccess && r == SA_OK) r = hip_fail(he, "batch tuning timer");
            *best = std::min(*best, t);
        }
        return r;
    };
    const bool may_persist = b->p.rerank == 0;
    // 1. each class alone, every (table, form) candidate
    struct Pick { int32_t lds; float ms; };
    std::vector<Pick> grid_best(b->cls.size(), {0, 1e30f}), loop_best(b->cls.size(), {0, 1e30f});
    std::string js = "{\"classes\":[";
    for (size_t i = 0; i < b->cls.size() && rc == SA_OK; ++i) {
        BatchClass &c = b->cls[i];
        js += i ? ",[" : "[";
        bool first = true;
        for (int32_t lds : lds_candidates(b->ix, b->p, c.Lmax, c.M)) {
            for (int32_t pers = 0; pers <= (may_persist ? 1 : 0) && rc == SA_OK; ++pers) {
                c.lds = lds;
                c.persistent = pers;
                float ms;
                rc = timed([&] { return launch_class(b, i, queries_dev, ldq, ids_dev, dists_dev, ldo, nullptr, ws, s); },
                           &ms);
                if (rc != SA_OK) break;
                Pick &pk = pers ? loop_best[i] : grid_best[i];
                if (ms < pk.ms) pk = {lds, ms};
                char buf[128];
                snprintf(buf, sizeof buf, "%s{\"lds_hash_slots\":%d,\"persistent\":%d,\"ms\":%.4f}", first ? "" : ",",
                         lds, pers, ms);
                js += buf;
                first = false;
            }
        }
        js += "]";
    }
    js += "],\"plans\":[";
    // 2. whole batch: three plans, each over 1, 2, 4 and 8 streams
    const char *names[3] = {"per_query", "persistent", "mixed"};
    float best = -1.f;
    int best_plan = 0, best_streams = 1;
    bool first = true;
    for (int plan = 0; plan < 3 && rc == SA_OK; ++plan) {
        if (plan > 0 && !may_persist) break;
        for (size_t i = 0; i < b->cls.size(); ++i) {
            BatchClass &c = b->cls[i];
            const bool loop = plan == 1 || (plan == 2 && loop_best[i].ms < grid_best[i].ms);
            c.persistent = loop ? 1 : 0;
            c.lds = loop ? loop_best[i].lds : grid_best[i].lds;
        }
        for (int ns : {1, 2, 4, 8}) {
            if (ns > 1 && (int)b->cls.size() < 2) continue;
            assign_streams(b, ns);
            float ms;
            rc = timed([&] { return run_batch(b, queries_dev, ldq, ids_dev, dists_dev, ldo, nullptr, workspace, s); },
                       &ms);
            if (rc != SA_OK) break;
            char buf[128];
            snprintf(buf, sizeof buf, "%s{\"plan\":\"%s\",\"streams\":%d,\"ms\":%.4f}", first ? "" : ",", names[plan],
                     ns, ms);
            js += buf;
            first = false;
            if (best < 0.f || ms < best) {
                best = ms;
                best_plan = plan;
                best_streams = ns;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (size_t i = 0; i < b->cls.size(); ++i) {
        BatchClass &c = b->cls[i];
        const bool loop = best_plan == 1 || (best_plan == 2 && loop_best[i].ms < grid_best[i].ms);
        c.persistent = loop ? 1 : 0;
        c.lds = loop ? loop_best[i].lds : grid_best[i].lds;
    }
    assign_streams(b, best_streams);
    if (rc != SA_OK) return rc;
    char buf[160];
    snprintf(buf, sizeof buf, "],\"chosen\":{\"plan\":\"%s\",\"streams\":%d,\"ms\":%.4f}}", names[best_plan],
             best_streams, best);
    js += buf;
    b->tuning = js;
    return SA_OK;
}

int sa_batch_set_config(sa_batch *b, int32_t streams, int32_t lds_hash_slots)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if (streams != 1 && streams != 2 && streams != 4 && streams != 8)
        return set_error(SA_EINVAL, "streams must be 1, 2, 4 or 8");
    for (const BatchClass &c : b->cls)
        if (c.M >= 2 && !lds_allowed(b->ix, b->p, c.Lmax, c.M, lds_hash_slots))
            return set_error(SA_EINVAL, "lds_hash_slots=%d is not a setting the plan has room for", lds_hash_slots);
    for (BatchClass &c : b->cls)
        if (c.M >= 2) c.lds = lds_hash_slots;
    assign_streams(b, streams);
    return SA_OK;
}

int32_t sa_batch_classes(const sa_batch *b) { return b ? (int32_t)b->cls.size() : 0; }

int sa_batch_class_options(const sa_batch *b, int32_t cls, int32_t *lds_values, int32_t cap, int32_t *count,
                           int32_t *persistent_ok)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if (cls < 0 || cls >= (int32_t)b->cls.size()) return set_error(SA_EINVAL, "class %d out of range", cls);
    const BatchClass &c = b->cls[cls];
    const std::vector<int32_t> ok = lds_candidates(b->ix, b->p, c.Lmax, c.M);
    if (count) *count = (int32_t)ok.size();
    for (int32_t i = 0; i < (int32_t)ok.size() && i < cap && lds_values; ++i) lds_values[i] = ok[i];
    if (persistent_ok) *persistent_ok = b->p.rerank == 0;
    return SA_OK;
}

int sa_batch_set_class(sa_batch *b, int32_t cls, int32_t lds_hash_slots, int32_t persistent)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if (cls < 0 || cls >= (int32_t)b->cls.size()) return set_error(SA_EINVAL, "class %d out of range", cls);
    BatchClass &c = b->cls[cls];
    if (!lds_allowed(b->ix, b->p, c.Lmax, c.M, lds_hash_slots))
        return set_error(SA_EINVAL, "lds_hash_slots=%d is not a setting class %d has room for", lds_hash_slots, cls);
    if (persistent && b->p.rerank != 0) return set_error(SA_EUNSUPPORTED, "the persistent form takes no re-rank");
    c.lds = lds_hash_slots;
    c.persistent = persistent ? 1 : 0;
    return SA_OK;
}

int64_t sa_batch_describe(const sa_batch *b, char *buf, size_t len)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    std::string js = "{\"queries\":" + std::to_string(b->nq) + ",\"kmax\":" + std::to_string(b->kmax) +
                     ",\"workspace_bytes\":" + std::to_string(b->ws_bytes) + ",\"streams\":" +
                     std::to_string(b->nstreams) + ",\"classes\":[";
    for (size_t i = 0; i < b->cls.size(); ++i) {
        const BatchClass &c = b->cls[i];
        char tmp[400];
        snprintf(tmp, sizeof tmp,
                 "%s{\"M\":%d,\"slots_per_lane\":%d,\"queries\":%lld,\"L_max\":%d,\"k_max\":%d,\"sum_L\":%.0f,"
                 "\"ws_hash_slots\":%d,\"lds_hash_slots\":%d,\"persistent\":%d,\"stream\":%d,\"workspace_bytes\":%zu}",
                 i ? "," : "", c.M, c.ni, (long long)c.n, c.Lmax, c.kmax, c.cost, 1 << c.glog2, c.lds, c.persistent,
                 c.stream, c.region_bytes * (size_t)c.n);
        js += tmp;
    }
    js += "],\"tuning\":" + (b->tuning.empty() ? std::string("null") : b->tuning) + "}";
    if (buf && len > 0) {
        const size_t m = std::min(len - 1, js.size());
        std::copy(js.begin(), js.begin() + m, buf);
        buf[m] = '\0';
    }
    return (int64_t)js.size() + 1;
}

void sa_batch_destroy(sa_batch *b)
{
    if (!b) return;
    for (int t = 0; t < MAX_STREAMS; ++t) {
        if (b->join[t]) (void)hipEventDestroy(b->join[t]);
        if (b->streams[t]) (void)hipStreamDestroy(b->streams[t]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

}  // extern "C"
