// The serving loop (sa_server_*): a worker thread that admits requests into
// micro-batch slots as they free up (continuous batching), and a load-replay helper.
// Contracts are in include/speedann.h.
//
// Requests go to one of up to four lanes by L (<= 128, <= 256, <= 512, above), each with
// its own waiting queue and slots (slot s serves lane s mod lanes), so that a short
// search never waits behind a long one for a slot.  A slot owns a stream, pinned
// staging buffers in and out, device buffers for the queries, the
// per-request (L, k) and the result rows, its share of the workspace, and one event
// per class.  Admission takes a lane's requests in arrival order (a request whose
// visited-set region does not fit the slot's workspace waits for the next slot) and
// stages them sorted by class, so that each class is a contiguous run of rows: classes
// are launched shortest L first, each followed by the copy of its own result rows and
// its own event, and the worker completes a class's requests as soon as its event has
// passed.
#include "sa_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace sa {
namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

constexpr int MAX_LANES = 4;

int lane_index(int L) { return L <= 128 ? 0 : L <= 256 ? 1 : L <= 512 ? 2 : 3; }

struct Request {
    uint64_t tag;
    int32_t k, L, M;
    int64_t t_submit;
    int32_t row;             // row of the query store holding its vector
    size_t region;           // workspace bytes reserved for it
};

struct Done {
    uint64_t tag;
    int32_t k;
    int64_t t_submit, t_done;
    std::vector<int32_t> ids;
    std::vector<float> dists;
};

struct Slot {
    int lane = 0;
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> done;          // one per class, created as needed
    std::vector<std::pair<int, int>> cls;  // row range of each class, in launch order
    size_t next = 0;                       // first class not yet completed
    unsigned char *h_in = nullptr, *h_out = nullptr;
    unsigned char *d_in = nullptr, *d_out = nullptr, *d_ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<Request> reqs;             // staged in class order
    bool busy = false;
};

// class order: walker count, register-queue size, then longest L first
bool class_less(const Request &a, const Request &c)
{
    if (a.M != c.M) return a.M < c.M;
    const int na = queue_slots_bucket(a.L, a.M), nc = queue_slots_bucket(c.L, c.M);
    if (na != nc) return na < nc;
    if (a.L != c.L) return a.L > c.L;
    return a.t_submit < c.t_submit;
}
bool same_class(const Request &a, const Request &c)
{
    return a.M == c.M && queue_slots_bucket(a.L, a.M) == queue_slots_bucket(c.L, c.M);
}

}  // namespace
}  // namespace sa

using namespace sa;

struct sa_server {
    const sa_index *ix;
    sa_search_params p;
    sa_server_config cfg;
    int device;
    int32_t d;
    std::vector<Slot> slots;

    int nlanes;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> waiting[MAX_LANES];
    int64_t nwaiting = 0;
    std::vector<float> store;     // max_pending rows of d floats holding waiting queries
    std::vector<int32_t> free_rows;
    std::deque<Done> finished;
    bool stop = false;
    int error = SA_OK;

    std::atomic<int64_t> completed{0}, batches{0}, launches{0}, max_seen{0}, sum_batch{0};
    std::thread worker;
};

namespace {

size_t in_bytes(const sa_server *S) { return align16(4 * (size_t)S->cfg.max_batch * S->d) + 3 * align16(4 * (size_t)S->cfg.max_batch); }
size_t out_bytes(const sa_server *S) { return 8 * (size_t)S->cfg.max_batch * S->cfg.k_max; }

// bytes of workspace a request reserves: the region of its class's largest possible L
size_t request_region(const sa_server *S, int32_t L, int32_t M)
{
    const int Lb = std::min(1024, 64 * queue_slots_bucket(L, M));
    return search_workspace_bytes(1, Lb, M, S->p, S->ix->R);
}

// Launches the requests of a filled slot (staged in class order): one copy in, then per
// class, shortest first, its launch, the copy of its result rows and its event.
int launch_slot(sa_server *S, Slot &sl)
{
    const int b = (int)sl.reqs.size();
    const int d = S->d;
    const size_t o_L = align16(4 * (size_t)b * d), o_k = o_L + align16(4 * (size_t)b), n_in = o_k + 4 * (size_t)b;
    int32_t *hL = reinterpret_cast<int32_t *>(sl.h_in + o_L);
    int32_t *hk = reinterpret_cast<int32_t *>(sl.h_in + o_k);
    for (int i = 0; i < b; ++i) {
        hL[i] = sl.reqs[i].L;
        hk[i] = sl.reqs[i].k;
    }
    sl.cls.clear();
    for (int i = 0; i < b;) {
        int j = i + 1;
        while (j < b && same_class(sl.reqs[j], sl.reqs[i])) ++j;
        sl.cls.emplace_back(i, j);
        i = j;
    }
    // shortest class first: its requests complete before the long ones start
    std::stable_sort(sl.cls.begin(), sl.cls.end(), [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
        return sl.reqs[x.first].L < sl.reqs[y.first].L;
    });
    while (sl.done.size() < sl.cls.size()) {
        hipEvent_t e;
        SA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        sl.done.push_back(e);
    }
    SA_HIP(hipMemcpyAsync(sl.d_in, sl.h_in, n_in, hipMemcpyHostToDevice, sl.stream));
    const int kmax = S->cfg.k_max;
    int32_t *d_ids = reinterpret_cast<int32_t *>(sl.d_out);
    float *d_dists = reinterpret_cast<float *>(sl.d_out + 4 * (size_t)S->cfg.max_batch * kmax);
    int32_t *h_ids = reinterpret_cast<int32_t *>(sl.h_out);
    float *h_dists = reinterpret_cast<float *>(sl.h_out + 4 * (size_t)S->cfg.max_batch * kmax);
    const sa_index *ix = S->ix;
    size_t ws_off = 0;
    for (size_t c = 0; c < sl.cls.size(); ++c) {
        const int i = sl.cls[c].first, j = sl.cls[c].second;
        const Request &r0 = sl.reqs[i];   // the longest L of its class
        int kc = 1;
        for (int t = i; t < j; ++t) kc = std::max(kc, sl.reqs[t].k);
        SearchLaunch a;
        a.codes = ix->codes; a.scale = ix->scale; a.ldc = ix->ldc; a.dtype = ix->dtype;
        a.vec32 = ix->vec32; a.ld32 = ix->ld32;
        a.n = ix->n; a.d = ix->d; a.metric = ix->metric;
        a.adj = ix->adj; a.R = ix->R; a.entry = ix->entry; a.id_map = ix->id_map;
        a.int_lo = ix->int_lo; a.int_hi = ix->int_hi;
        // the class's rows: query q of the launch is staged row i + q
        a.queries = reinterpret_cast<const float *>(sl.d_in) + (size_t)i * d; a.ldq = d;
        a.nq = j - i; a.k = kc; a.L = r0.L; a.M = r0.M; a.p = S->p;
        a.ids = d_ids + (size_t)i * kmax; a.dists = d_dists + (size_t)i * kmax; a.stats = nullptr;
        const size_t region = search_workspace_bytes(1, r0.L, r0.M, S->p, ix->R);
        a.workspace = sl.d_ws + ws_off; a.ws_bytes = region * (size_t)(j - i);
        ws_off += (a.ws_bytes + 255) & ~size_t(255);
        a.qL = reinterpret_cast<const int32_t *>(sl.d_in + o_L) + i;
        a.qk = reinterpret_cast<const int32_t *>(sl.d_in + o_k) + i;
        a.order = nullptr;
        a.ldo = kmax;
        const int rc = launch_search(a, sl.stream);
        if (rc != SA_OK) return rc;
        const size_t rows = 4 * (size_t)(j - i) * kmax;
        SA_HIP(hipMemcpyAsync(h_ids + (size_t)i * kmax, a.ids, rows, hipMemcpyDeviceToHost, sl.stream));
        SA_HIP(hipMemcpyAsync(h_dists + (size_t)i * kmax, a.dists, rows, hipMemcpyDeviceToHost, sl.stream));
        SA_HIP(hipEventRecord(sl.done[c], sl.stream));
        S->launches.fetch_add(1, std::memory_order_relaxed);
    }
    sl.next = 0;
    sl.busy = true;
    S->batches.fetch_add(1, std::memory_order_relaxed);
    S->sum_batch.fetch_add(b, std::memory_order_relaxed);
    int64_t m = S->max_seen.load();
    while (b > m && !S->max_seen.compare_exchange_weak(m, b)) {
    }
    return SA_OK;
}

// Completes the requests of class c of a slot.
void retire_class(sa_server *S, Slot &sl, size_t c)
{
    const int64_t t = now_ns();
    const int kmax = S->cfg.k_max;
    const int32_t *ids = reinterpret_cast<const int32_t *>(sl.h_out);
    const float *dists = reinterpret_cast<const float *>(sl.h_out + 4 * (size_t)S->cfg.max_batch * kmax);
    const int i0 = sl.cls[c].first, i1 = sl.cls[c].second;
    std::vector<Done> out(i1 - i0);
    for (int i = i0; i < i1; ++i) {
        const Request &r = sl.reqs[i];
        Done &o = out[i - i0];
        o.tag = r.tag;
        o.k = r.k;
        o.t_submit = r.t_submit;
        o.t_done = t;
        o.ids.assign(ids + (size_t)i * kmax, ids + (size_t)i * kmax + r.k);
        o.dists.assign(dists + (size_t)i * kmax, dists + (size_t)i * kmax + r.k);
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        for (Done &o : out) S->finished.push_back(std::move(o));
    }
    S->completed.fetch_add(i1 - i0, std::memory_order_relaxed);
    S->cv_done.notify_all();
}

void worker_main(sa_server *S)
{
    if (hipSetDevice(S->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(S->mu);
        S->error = SA_EHIP;
        S->stop = true;
        S->cv_done.notify_all();
        return;
    }
    for (;;) {
        bool progressed = false, any_busy = false;
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            // classes complete in launch order on the slot's stream
            while (sl.next < sl.cls.size()) {
                const hipError_t q = hipEventQuery(sl.done[sl.next]);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    std::lock_guard<std::mutex> g(S->mu);
                    S->error = hip_fail(q, "serving micro-batch");
                    S->stop = true;
                    break;
                }
                retire_class(S, sl, sl.next++);
                progressed = true;
            }
            if (sl.next >= sl.cls.size() || S->error != SA_OK) {
                sl.reqs.clear();
                sl.busy = false;
            } else {
                any_busy = true;
            }
        }
        // fill free slots from the front of the waiting queue
        for (Slot &sl : S->slots) {
            if (sl.busy) continue;
            {
                std::lock_guard<std::mutex> g(S->mu);
                if (S->error != SA_OK) break;
                std::deque<Request> &wq = S->waiting[sl.lane];
                if (wq.empty()) continue;
                size_t used = 0;
                float *hq = reinterpret_cast<float *>(sl.h_in);
                while (!wq.empty() && (int)sl.reqs.size() < S->cfg.max_batch) {
                    const Request &r = wq.front();
                    if (used + r.region > sl.ws_bytes && !sl.reqs.empty()) break;
                    used += r.region;
                    sl.reqs.push_back(r);
                    wq.pop_front();
                    --S->nwaiting;
                }
                // stage in class order, then give the store rows back
                std::sort(sl.reqs.begin(), sl.reqs.end(), class_less);
                for (size_t i = 0; i < sl.reqs.size(); ++i) {
                    std::memcpy(hq + i * S->d, S->store.data() + (size_t)sl.reqs[i].row * S->d, 4 * (size_t)S->d);
                    S->free_rows.push_back(sl.reqs[i].row);
                }
            }
            S->cv_work.notify_all();   // room in the waiting queue
            const int rc = launch_slot(S, sl);
            if (rc != SA_OK) {
                std::lock_guard<std::mutex> g(S->mu);
                S->error = rc;
                S->stop = true;
                sl.reqs.clear();
                break;
            }
            progressed = true;
            any_busy = true;
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->stop && !any_busy && (S->nwaiting == 0 || S->error != SA_OK)) break;
        if (progressed) continue;
        if (any_busy) {
            // micro-batches on the device: poll their events again shortly
            lk.unlock();
            std::this_thread::yield();
        } else {
            S->cv_work.wait_for(lk, std::chrono::microseconds(500),
                                [&] { return S->stop || S->nwaiting > 0; });
        }
    }
    S->cv_done.notify_all();
}

void free_server(sa_server *S)
{
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        for (hipEvent_t e : sl.done) (void)hipEventDestroy(e);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.d_out) (void)hipFree(sl.d_out);
        if (sl.d_ws) (void)hipFree(sl.d_ws);
    }
    delete S;
}

}  // namespace

extern "C" {

void sa_server_default_config(sa_server_config *cfg)
{
    if (!cfg) return;
    cfg->slots = 8;
    cfg->max_batch = 1024;
    cfg->max_pending = 65536;
    cfg->k_max = 100;
    cfg->workspace_bytes = size_t(1) << 30;
}

int sa_server_create(const sa_index *index, const sa_search_params *params, const sa_server_config *cfg,
                     sa_server **out)
{
    if (!out) return set_error(SA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!index) return set_error(SA_EINVAL, "index is NULL");
    sa_server_config c;
    if (cfg) c = *cfg;
    else sa_server_default_config(&c);
    if (c.slots < 1 || c.slots > 16) return set_error(SA_EINVAL, "slots=%d must be in [1, 16]", c.slots);
    if (c.max_batch < 1 || c.max_batch > 65536) return set_error(SA_EINVAL, "max_batch must be in [1, 65536]");
    if (c.max_pending < 1) return set_error(SA_EINVAL, "max_pending must be >= 1");
    if (c.k_max < 1 || c.k_max > 1024) return set_error(SA_EINVAL, "k_max must be in [1, 1024]");
    sa_search_params p;
    if (params) p = *params;
    else sa_default_params(&p);
    int rc;
    if ((rc = check_search(index, 1, 1, 1024, 16, p)) != SA_OK) return rc;
    if ((rc = check_device()) != SA_OK) return rc;
    int device = 0;
    SA_HIP(hipGetDevice(&device));
    sa_server *S = new sa_server();
    S->ix = index;
    S->p = p;
    S->cfg = c;
    S->d = index->d;
    S->device = device;
    // the largest single request must fit a slot
    const size_t per_slot = c.workspace_bytes / (size_t)c.slots;
    if (per_slot < request_region(S, 1024, 16)) {
        const size_t need = request_region(S, 1024, 16) * (size_t)c.slots;
        delete S;
        return set_error(SA_EINVAL, "workspace_bytes must be at least %zu (one L=1024, M=16 request per slot)", need);
    }
    S->store.resize((size_t)c.max_pending * S->d);
    S->free_rows.resize(c.max_pending);
    for (int32_t i = 0; i < c.max_pending; ++i) S->free_rows[i] = c.max_pending - 1 - i;
    S->nlanes = std::min(MAX_LANES, c.slots);
    S->slots.resize(c.slots);
    hipError_t e = hipSuccess;
    for (size_t si = 0; si < S->slots.size(); ++si) {
        Slot &sl = S->slots[si];
        sl.lane = (int)(si % S->nlanes);
        sl.ws_bytes = per_slot & ~size_t(255);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_in), in_bytes(S), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_out), out_bytes(S), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.d_in), in_bytes(S));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.d_out), out_bytes(S));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.d_ws), sl.ws_bytes);
        if (e == hipSuccess) e = hipMemsetAsync(sl.d_ws, 0, sl.ws_bytes, sl.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
        sl.reqs.reserve(c.max_batch);
    }
    if (e != hipSuccess) {
        free_server(S);
        return hip_fail(e, "server buffers");
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return SA_OK;
}

void sa_server_destroy(sa_server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        for (int l = 0; l < MAX_LANES; ++l) S->waiting[l].clear();
        S->nwaiting = 0;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    free_server(S);
}

int sa_server_submit(sa_server *S, const float *query_host, int32_t k, int32_t L, int32_t M, uint64_t tag)
{
    if (!S) return set_error(SA_EINVAL, "server is NULL");
    if (!query_host) return set_error(SA_EINVAL, "query is NULL");
    if (k < 1 || k > S->cfg.k_max || L < k || L > 1024 || M < 1 || M > 16)
        return set_error(SA_EINVAL, "need 1 <= k <= min(L, k_max=%d), L <= 1024, 1 <= M <= 16 (k=%d, L=%d, M=%d)",
                         S->cfg.k_max, k, L, M);
    Request r;
    r.tag = tag;
    r.k = k;
    r.L = L;
    r.M = M;
    r.region = request_region(S, L, M);
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->error != SA_OK) return set_error(S->error, "the server stopped after an error");
        if (S->stop) return set_error(SA_EINVAL, "the server is stopping");
        if (S->free_rows.empty())
            return set_error(SA_ECAPACITY, "%d requests are already waiting", S->cfg.max_pending);
        r.row = S->free_rows.back();
        S->free_rows.pop_back();
        std::memcpy(S->store.data() + (size_t)r.row * S->d, query_host, 4 * (size_t)S->d);
        r.t_submit = now_ns();
        S->waiting[std::min(lane_index(L), S->nlanes - 1)].push_back(r);
        ++S->nwaiting;
    }
    S->cv_work.notify_one();
    return SA_OK;
}

int32_t sa_server_poll(sa_server *S, int32_t max, uint64_t *tags, int32_t *ids, float *dists, int64_t ldo,
                       int64_t *t_submit_ns, int64_t *t_done_ns, int32_t wait_us)
{
    if (!S) return set_error(SA_EINVAL, "server is NULL");
    if (max < 0 || (max > 0 && (!tags || !ids || !dists))) return set_error(SA_EINVAL, "NULL output");
    if (ldo < S->cfg.k_max) return set_error(SA_EINVAL, "ldo must be >= k_max (%d)", S->cfg.k_max);
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->finished.empty() && wait_us > 0)
        S->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                            [&] { return !S->finished.empty() || S->error != SA_OK; });
    if (S->finished.empty() && S->error != SA_OK) return set_error(S->error, "the server stopped after an error");
    int32_t n = 0;
    while (n < max && !S->finished.empty()) {
        Done &o = S->finished.front();
        tags[n] = o.tag;
        std::copy(o.ids.begin(), o.ids.end(), ids + n * ldo);
        std::copy(o.dists.begin(), o.dists.end(), dists + n * ldo);
        if (t_submit_ns) t_submit_ns[n] = o.t_submit;
        if (t_done_ns) t_done_ns[n] = o.t_done;
        S->finished.pop_front();
        ++n;
    }
    return n;
}

int sa_server_replay(sa_server *S, const float *queries_host, int64_t n, int64_t ldq, const int32_t *k,
                     const int32_t *L, const int32_t *M, const int64_t *arrival_ns, int32_t *ids, float *dists,
                     int64_t ldo, int64_t *latency_ns, int64_t *wall_ns)
{
    if (!S) return set_error(SA_EINVAL, "server is NULL");
    if (n < 0) return set_error(SA_EINVAL, "n < 0");
    if (n > 0 && (!queries_host || !k || !L || !M || !arrival_ns || !ids || !dists || !latency_ns))
        return set_error(SA_EINVAL, "NULL argument");
    if (ldq < S->d) return set_error(SA_EINVAL, "ldq < d");
    if (ldo < S->cfg.k_max) return set_error(SA_EINVAL, "ldo must be >= k_max (%d)", S->cfg.k_max);
    for (int64_t i = 0; i < n; ++i)
        if (k[i] < 1 || k[i] > S->cfg.k_max || L[i] < k[i] || L[i] > 1024 || M[i] < 1 || M[i] > 16 ||
            (i > 0 && arrival_ns[i] < arrival_ns[i - 1]))
            return set_error(SA_EINVAL, "request %lld: bad k, L, M or arrival time", (long long)i);
    const int64_t t0 = now_ns();
    std::atomic<int> err{SA_OK};
    int64_t last_done = t0;
    // collector: results of this replay, by tag = request index
    std::thread collector([&] {
        const int chunk = 256;
        std::vector<uint64_t> tg(chunk);
        std::vector<int32_t> id((size_t)chunk * ldo);
        std::vector<float> ds((size_t)chunk * ldo);
        std::vector<int64_t> td(chunk);
        int64_t got = 0;
        while (got < n && err == SA_OK) {
            const int32_t m = sa_server_poll(S, chunk, tg.data(), id.data(), ds.data(), ldo, nullptr, td.data(), 1000);
            if (m < 0) {
                err = m;
                return;
            }
            for (int32_t j = 0; j < m; ++j) {
                const int64_t i = (int64_t)tg[j];
                if (i < 0 || i >= n) continue;
                std::copy(id.begin() + (size_t)j * ldo, id.begin() + (size_t)j * ldo + k[i], ids + i * ldo);
                std::copy(ds.begin() + (size_t)j * ldo, ds.begin() + (size_t)j * ldo + k[i], dists + i * ldo);
                latency_ns[i] = td[j] - (t0 + arrival_ns[i]);
                last_done = std::max(last_done, td[j]);
                ++got;
            }
        }
    });
    for (int64_t i = 0; i < n && err == SA_OK; ++i) {
        const int64_t due = t0 + arrival_ns[i];
        while (now_ns() < due) {
        }
        int rc;
        while ((rc = sa_server_submit(S, queries_host + i * ldq, k[i], L[i], M[i], (uint64_t)i)) == SA_ECAPACITY)
            std::this_thread::yield();
        if (rc != SA_OK) {
            err = rc;
            break;
        }
    }
    collector.join();
    if (err != SA_OK) return err;
    if (wall_ns) wall_ns[0] = n > 0 ? last_done - (t0 + arrival_ns[0]) : 0;
    return SA_OK;
}

int sa_server_stats(const sa_server *S, int64_t *completed, int64_t *batches, int64_t *launches,
                    int64_t *max_batch_seen, int64_t *sum_batch)
{
    if (!S) return set_error(SA_EINVAL, "server is NULL");
    if (completed) *completed = S->completed.load();
    if (batches) *batches = S->batches.load();
    if (launches) *launches = S->launches.load();
    if (max_batch_seen) *max_batch_seen = S->max_seen.load();
    if (sum_batch) *sum_batch = S->sum_batch.load();
    return SA_OK;
}

}  // extern "C"
