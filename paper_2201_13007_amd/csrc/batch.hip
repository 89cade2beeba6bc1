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
// that stream holds every class as a parallel branch.  The autotuner times the choices
// that leave every result unchanged: the number of streams (1, 2, 4, 8) and, for classes
// with two or more walkers, whether the visited set starts in an LDS table.
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
    size_t off_L, off_k, off_order, ws_bytes;
    std::string tuning;      // JSON of the last tuning run
};

namespace {

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

int launch_class(const sa_batch *b, const BatchClass &c, const float *queries, int64_t ldq, int32_t *ids,
                 float *dists, int64_t ldo, sa_query_stats *stats, unsigned char *ws, hipStream_t s)
{
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
    a.p.ws_hash_slots = 1 << c.glog2;
    a.ids = ids; a.dists = dists; a.stats = stats;
    a.workspace = ws + c.ws_off; a.ws_bytes = c.region_bytes * (size_t)c.n;
    a.qL = reinterpret_cast<const int32_t *>(ws + b->off_L);
    a.qk = reinterpret_cast<const int32_t *>(ws + b->off_k);
    a.order = reinterpret_cast<const int32_t *>(ws + b->off_order) + c.first;
    a.ldo = ldo;
    return launch_search(a, s);
}

int run_batch(const sa_batch *b, const float *queries, int64_t ldq, int32_t *ids, float *dists, int64_t ldo,
              sa_query_stats *stats, void *workspace, hipStream_t s)
{
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    if (b->nstreams <= 1) {
        for (const BatchClass &c : b->cls) {
            const int rc = launch_class(b, c, queries, ldq, ids, dists, ldo, stats, ws, s);
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
        const BatchClass &c = b->cls[i];
        const int rc = launch_class(b, c, queries, ldq, ids, dists, ldo, stats, ws, b->streams[c.stream]);
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
        // every query of the class gets the table its largest L takes
        int32_t llog2, glog2;
        search_table_log2(p, c.Lmax, c.M, index->R, &llog2, &glog2);
        c.glog2 = glog2;
        c.region_bytes = search_workspace_bytes(1, c.Lmax, c.M, p, index->R);
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
    bool multi = false;
    for (const BatchClass &c : b->cls) multi |= c.M >= 2;
    const int32_t user_lds = b->p.lds_hash_slots;
    std::vector<int32_t> lds_modes{user_lds};
    if (multi && user_lds == 0) lds_modes.push_back(-1);   // default tables, or none in LDS
    hipEvent_t e0, e1;
    SA_HIP(hipEventCreate(&e0));
    SA_HIP(hipEventCreate(&e1));
    float best = -1.f;
    int best_streams = 1;
    int32_t best_lds = user_lds;
    std::string js = "{\"candidates\":[";
    bool first = true;
    for (int32_t lds : lds_modes) {
        for (int ns : {1, 2, 4, 8}) {
            if (ns > 1 && (int)b->cls.size() < 2) continue;
            for (BatchClass &c : b->cls)
                if (c.M >= 2) c.lds = lds;
            assign_streams(b, ns);
            rc = run_batch(b, queries_dev, ldq, ids_dev, dists_dev, ldo, nullptr, workspace, s);   // warm
            float ms = 1e30f;
            for (int r = 0; r < reps && rc == SA_OK; ++r) {
                hipError_t he = hipEventRecord(e0, s);
                if (he == hipSuccess) rc = run_batch(b, queries_dev, ldq, ids_dev, dists_dev, ldo, nullptr, workspace, s);
                if (he == hipSuccess && rc == SA_OK) he = hipEventRecord(e1, s);
                if (he == hipSuccess && rc == SA_OK) he = hipEventSynchronize(e1);
                float t = 0.f;
                if (he == hipSuccess && rc == SA_OK) he = hipEventElapsedTime(&t, e0, e1);
                if (he != hipSuccess && rc == SA_OK) rc = hip_fail(he, "batch tuning timer");
                ms = std::min(ms, t);
            }
            if (rc != SA_OK) break;
            char buf[160];
            snprintf(buf, sizeof buf, "%s{\"streams\":%d,\"lds_hash_slots\":%d,\"ms\":%.4f}", first ? "" : ",", ns,
                     lds, ms);
            js += buf;
            first = false;
            if (best < 0.f || ms < best) {
                best = ms;
                best_streams = ns;
                best_lds = lds;
            }
        }
        if (rc != SA_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (BatchClass &c : b->cls)
        if (c.M >= 2) c.lds = best_lds;
    assign_streams(b, best_streams);
    if (rc != SA_OK) return rc;
    char buf[160];
    snprintf(buf, sizeof buf, "],\"chosen\":{\"streams\":%d,\"lds_hash_slots\":%d,\"ms\":%.4f}}", best_streams, best_lds,
             best);
    js += buf;
    b->tuning = js;
    return SA_OK;
}

int sa_batch_set_config(sa_batch *b, int32_t streams, int32_t lds_hash_slots)
{
    if (!b) return set_error(SA_EINVAL, "batch is NULL");
    if (streams != 1 && streams != 2 && streams != 4 && streams != 8)
        return set_error(SA_EINVAL, "streams must be 1, 2, 4 or 8");
    for (BatchClass &c : b->cls)
        if (c.M >= 2) c.lds = lds_hash_slots;
    assign_streams(b, streams);
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
        char tmp[320];
        snprintf(tmp, sizeof tmp,
                 "%s{\"M\":%d,\"slots_per_lane\":%d,\"queries\":%lld,\"L_max\":%d,\"k_max\":%d,\"sum_L\":%.0f,"
                 "\"ws_hash_slots\":%d,\"lds_hash_slots\":%d,\"stream\":%d,\"workspace_bytes\":%zu}",
                 i ? "," : "", c.M, c.ni, (long long)c.n, c.Lmax, c.kmax, c.cost, 1 << c.glog2, c.lds, c.stream,
                 c.region_bytes * (size_t)c.n);
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
