// Host side of the search: parameter resolution, LDS layout, workspace sizing and the
// launch of the single-worker kernel (search_single.h) or of the general kernel
// (search_multi.h, whose body is in search_body.h), one instantiation per storage type.
#include "search_body.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

namespace sa {
namespace {

using search_detail::Ctrl;
using search_detail::KArgs;

struct Layout {
    uint32_t o_skey, o_srank, o_schk, o_pub, o_newkey, o_claim, o_ctrl, o_hash, o_q, total;
};

uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

// S, the rank array and the published new keys of a merge exist only with M >= 2; the
// query takes 16 floats per lane of a vector group
Layout make_layout(int L, int M, int llog2, int lpv)
{
    Layout Y;
    const uint32_t LL = M >= 2 ? (uint32_t)L : 0u;
    uint32_t o = 0;
    Y.o_skey = o; o += 2u * 8u * LL;
    Y.o_srank = o; o += 4u * LL;
    Y.o_schk = o; o = align_up(o + 2u * LL, 16);
    Y.o_pub = o; o += M >= 2 ? 8u * search_detail::PUBCAP : 0u;
    o = align_up(o, 16);
    Y.o_newkey = o; o += 8u * 64u * M;
    Y.o_claim = o; o += 4u * 64u * M;
    Y.o_ctrl = o; o += align_up(sizeof(Ctrl), 16);
    Y.o_hash = o; o += llog2 > 0 ? (8u << llog2) : 0u;
    Y.o_q = o; o += 64u * (uint32_t)lpv;
    Y.total = o;
    return Y;
}

int ilog2_exact(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// One worker with no LDS table runs the single-worker kernel, whose workspace table holds
// 32-bit entries (id + 1) and needs no claim order; so do two workers that merge after
// every local step over rows of at most 32 entries (both rows fill one wavefront, and with
// every-step merges one queue holds what the two local queues would).  Every other case
// runs the general kernel with 64-bit entries that carry the claim tag.
bool compact_table(int M, int llog2, int sync, int R)
{
    return llog2 == 0 && (M == 1 || (M == 2 && sync == SA_SYNC_BSP && R <= 32));
}

void resolve_params(const sa_search_params &in, int L, int M, int R, int &llog2, int &glog2, int &max_sub)
{
    max_sub = in.max_substeps > 0 ? in.max_substeps : (1 << 22);
    if (in.lds_hash_slots > 0) llog2 = ilog2_exact(in.lds_hash_slots);
    else if (in.lds_hash_slots < 0) llog2 = 0;
    else if (M <= 2) llog2 = 0;     // one or two workers: favour occupancy over LDS latency
    else if (M < 8) llog2 = 12;
    else {
        // eight or more workers are for latency: a table of about 16 L slots keeps the
        // visited set (some 8 L vertices) in LDS, if the layout leaves room for it
        llog2 = 12;
        for (int lg = ilog2_exact(std::min<int64_t>(16ll * L, 1 << 14)); lg > 12; --lg)
            if (make_layout(L, M, lg, 64).total <= 160u * 1024u) {
                llog2 = lg;
                break;
            }
    }
    if (in.ws_hash_slots > 0) glog2 = ilog2_exact(in.ws_hash_slots);
    else {
        // the visited set holds at most 1 + E * R vertices after E expansions, and E stays
        // close to L.  The single-worker region (4-byte entries; a search may start in a
        // prefix of it, see glog2_init below) takes 32 L slots: its
        // three-quarter limit sits near 24 L, several times the 8 L or so a search visits
        // at these R; the general table keeps 64 L.  8 M R more cover the M R vertices one
        // local step may add on top.
        const bool compact = compact_table(M, llog2, in.sync, R);
        int64_t want = (compact ? 32ll : 64ll) * L + 8ll * M * R;
        // at least 8192 slots (16384 for eight or more workers, which explore more before they
        // merge): at small L a rare query visits several times the usual 8-15 L vertices, and
        // one that fills its region stops with a partial result
        want = std::max<int64_t>(want, !compact && M >= 8 ? 16384 : 8192);
        // a re-rank takes the last 1025 entries of the slot list, beyond the three
        // quarters the search may fill: at least 8192 slots
        if (in.rerank != 0 && want < 8192) want = 8192;
        glog2 = ilog2_exact(want);
    }
}

size_t bytes_per_slot(int M, int llog2, int sync, int R) { return compact_table(M, llog2, sync, R) ? 8 : 16; }

}  // namespace

uint32_t search_lds_bytes(int32_t L, int32_t M, int32_t llog2, int32_t d)
{
    return make_layout(L, M, llog2, search_detail::lanes_per_vector(d)).total;
}

void search_table_log2(const sa_search_params &p, int32_t L, int32_t M, int32_t R, int32_t *llog2, int32_t *glog2)
{
    int ms;
    resolve_params(p, L, M, R, *llog2, *glog2, ms);
}

size_t search_workspace_bytes(int64_t nq, int32_t L, int32_t M, const sa_search_params &p, int32_t R)
{
    int llog2, glog2, max_sub;
    resolve_params(p, L, M, R, llog2, glog2, max_sub);
    return (size_t)nq * (bytes_per_slot(M, llog2, p.sync, R) << glog2);
}

namespace {

// flags[0]: some coordinate is not an integer of magnitude <= 2^24; flags[1], flags[2]:
// smallest and largest coordinate (as integers)
__global__ void integer_range_kernel(const float *x, int64_t n, int32_t d, int64_t ld, int32_t *flags)
{
    bool bad = false;
    int lo = INT_MAX, hi = INT_MIN;
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / d;
        const float v = x[r * ld + (e - r * d)];
        if (!(fabsf(v) <= 16777216.f) || v != rintf(v)) {
            bad = true;
        } else {
            lo = min(lo, (int)v);
            hi = max(hi, (int)v);
        }
    }
    if (bad) atomicOr(flags, 1);
    if (lo <= hi) {
        atomicMin(flags + 1, lo);
        atomicMax(flags + 2, hi);
    }
}

}  // namespace

int index_integer_range(const float *x, int64_t n, int32_t d, int64_t ld, int32_t *lo, int32_t *hi)
{
    *lo = 1;
    *hi = 0;
    if (n < 1 || d < 1) return SA_OK;
    int32_t *flags = nullptr;
    SA_HIP(hipMalloc(reinterpret_cast<void **>(&flags), 16));
    const int32_t init[3] = {0, INT_MAX, INT_MIN};
    int32_t res[3] = {1, 0, 0};
    hipError_t e = hipMemcpy(flags, init, 12, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int64_t blocks = std::min<int64_t>((n * d + 255) / 256, 8192);
        hipLaunchKernelGGL(integer_range_kernel, dim3((unsigned)blocks), dim3(256), 0, 0, x, n, d, ld, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(res, flags, 12, hipMemcpyDeviceToHost);
    (void)hipFree(flags);
    if (e != hipSuccess) return hip_fail(e, "integer range of the vectors");
    if (res[0] != 0 || res[1] > res[2]) return SA_OK;
    // squared differences of two coordinates in range and products of two: every partial
    // sum of d of them stays below 2^24
    const int64_t span = (int64_t)res[2] - res[1], mag = std::max<int64_t>(std::abs((int64_t)res[1]), std::abs((int64_t)res[2]));
    if (span * span * d < (int64_t(1) << 24) && mag * mag * d < (int64_t(1) << 24)) {
        *lo = res[1];
        *hi = res[2];
    }
    return SA_OK;
}

hipError_t resident_grid(const void *k, int block, uint32_t lds, int64_t njobs, int64_t *grid)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, uint32_t, int>, int64_t> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int64_t slots = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find({k, lds, dev});
        if (it != cache.end()) slots = it->second;
    }
    if (slots == 0) {
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        slots = std::max<int64_t>(1, (int64_t)per_cu * cus);
        std::lock_guard<std::mutex> g(mu);
        cache[{k, lds, dev}] = slots;
    }
    *grid = std::max<int64_t>(1, std::min(njobs, slots));
    return hipSuccess;
}

hipError_t lds_fill_log2(const void *k, int block, uint32_t base, int lmin, int lmax, int *out)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find({k, dev});
        if (it != cache.end()) {
            *out = it->second;
            return hipSuccess;
        }
    }
    int want = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&want, k, block, base + (4u << lmin));
    if (e != hipSuccess) return e;
    int l = lmin;
    for (int c = lmax; c > lmin; --c) {
        int got = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&got, k, block, base + (4u << c));
        if (e != hipSuccess) return e;
        if (got >= want) {
            l = c;
            break;
        }
    }
    std::lock_guard<std::mutex> g(mu);
    cache[{k, dev}] = l;
    *out = l;
    return hipSuccess;
}

int launch_search(const SearchLaunch &a, hipStream_t stream)
{
    int llog2, glog2, max_sub;
    resolve_params(a.p, a.L, a.M, a.R, llog2, glog2, max_sub);
    if (llog2 != 0 && (llog2 < 6 || llog2 > 14))
        return set_error(SA_EINVAL, "lds_hash_slots must be a power of two in [64, 16384] (or -1 for none)");
    if (glog2 < 6 || glog2 > 26) return set_error(SA_EINVAL, "ws_hash_slots must be a power of two in [64, 2^26]");
    if (a.p.rerank != 0 && glog2 < 13) return set_error(SA_EINVAL, "a re-rank needs ws_hash_slots >= 8192");
    if (llog2 > 0 && (int64_t(1) << llog2) / 2 < (int64_t)a.M * a.R + 1)
        return set_error(SA_EINVAL, "lds_hash_slots too small for M * R new vertices per local step");
    if ((int64_t(1) << glog2) * 3 / 4 < (int64_t)a.M * a.R + 1)
        return set_error(SA_EINVAL, "ws_hash_slots too small for M * R new vertices per local step");
    const size_t need = (size_t)a.nq * (bytes_per_slot(a.M, llog2, a.p.sync, a.R) << glog2);
    if (a.ws_bytes < need)
        return set_error(SA_ECAPACITY, "workspace of %zu bytes is smaller than the %zu bytes needed", a.ws_bytes, need);
    if (a.workspace == nullptr && need > 0) return set_error(SA_EINVAL, "workspace is NULL");
    if (((uintptr_t)a.workspace & 255u) != 0) return set_error(SA_EINVAL, "workspace must be 256-byte aligned");
    Layout Y = make_layout(a.L, a.M, llog2, search_detail::lanes_per_vector(a.d));
    if (Y.total > 160u * 1024u)
        return set_error(SA_ECAPACITY, "L=%d, M=%d need %u bytes of LDS per query (limit 163840); lower L, M or "
                         "lds_hash_slots", a.L, a.M, Y.total);
    KArgs A;
    A.codes = a.codes; A.scale = a.scale; A.ldc = a.ldc; A.vec32 = a.vec32; A.ld32 = a.ld32; A.rerank = a.p.rerank;
    A.adj = a.adj; A.queries = a.queries; A.ldq = a.ldq;
    A.qL = a.qL; A.qk = a.qk; A.order = a.order; A.ldo = a.ldo > 0 ? a.ldo : a.k;
    if (a.jobctr && a.p.rerank != 0) return set_error(SA_EUNSUPPORTED, "the persistent form takes no re-rank");
    if (a.nq > 0x7FFFFFFF) return set_error(SA_EINVAL, "nq=%lld out of range", (long long)a.nq);
    A.jobctr = a.jobctr; A.njobs = (int32_t)a.nq;
    A.ids = a.ids; A.dists = a.dists; A.stats = a.stats;
    A.ghash = reinterpret_cast<unsigned long long *>(a.workspace);
    A.n = a.n;
    A.idbits = 1;
    while ((int64_t(1) << A.idbits) < a.n) ++A.idbits;
    A.d = a.d; A.metric = a.metric; A.R = a.R; A.entry = a.entry; A.k = a.k; A.L = a.L; A.M = a.M;
    A.sync = a.p.sync; A.static_I = a.p.static_I; A.staged = a.p.staged ? 1 : 0; A.max_substeps = max_sub;
    A.rho = a.p.rho; A.glog2 = glog2; A.llog2 = llog2;
    // The single worker starts in the whole region, unless the region-sized tables of the
    // queries that can be resident at once (at most 256 CUs x 24 wavefronts) would take
    // more than half of the 256 MB Infinity Cache: then it starts in a table of at least
    // 8192 and 24 L slots (a search visits some 7-15 L vertices, so it stays under about
    // 40% full, where probe chains are still short), and the smaller tables keep the
    // claims out of HBM.  With fewer queries in flight the emptier region-sized table is
    // faster.  A query that outgrows its table moves into one twice as large, up to the
    // region's 2^glog2.
    if (a.p.ws_hash_init > 0 && compact_table(a.M, llog2, a.p.sync, a.R)) {
        // (used by one walker only; larger than the region means the region)
        const int t = ilog2_exact(a.p.ws_hash_init);
        if (t < 7 || (int64_t(1) << t) != a.p.ws_hash_init)
            return set_error(SA_EINVAL, "ws_hash_init must be a power of two >= 128");
        if ((int64_t(1) << t) * 3 / 4 < (int64_t)a.R + 1)
            return set_error(SA_EINVAL, "ws_hash_init too small for R new vertices per local step");
        A.glog2_init = std::min(t, glog2);
    } else {
        const int64_t resident = std::min<int64_t>(a.nq, 256 * 24);
        const bool crowded = resident * (int64_t(4) << glog2) > (int64_t(128) << 20);
        const int64_t want0 = std::max<int64_t>(8192, 24ll * a.L);
        int t = 10;
        while (t < glog2 && (int64_t(1) << t) < want0) ++t;
        A.glog2_init = crowded ? std::min(t, glog2) : glog2;
    }
    A.o_skey = Y.o_skey; A.o_srank = Y.o_srank; A.o_schk = Y.o_schk; A.o_pub = Y.o_pub;
    A.o_newkey = Y.o_newkey; A.o_claim = Y.o_claim; A.o_ctrl = Y.o_ctrl;
    A.o_hash = Y.o_hash; A.o_q = Y.o_q;
    if (a.nq == 0) return SA_OK;
    if (a.d > 1024) return set_error(SA_EUNSUPPORTED, "d=%d exceeds 1024", a.d);
    int rc;
    const bool compact = compact_table(a.M, llog2, a.p.sync, a.R);
    A.int_lo = a.int_lo; A.int_hi = a.int_hi; A.acc_pass = -1;
    if (compact) {
        if (a.dtype == SA_BF16) rc = launch_search_single_bf16(A, a.nq, stream);
        else if (a.dtype == SA_FP8E4M3) rc = launch_search_single_fp8(A, a.nq, stream);
        else if (a.int_lo <= a.int_hi && search_detail::lanes_per_vector(a.d) <= 16) {
            // integer-valued data: the queries that are integers in the same range in
            // float32 (exact), the others in double; each workgroup checks its query and
            // leaves it to the other pass if it is not its own
            A.acc_pass = 1;
            rc = launch_search_single_f32(A, a.nq, stream);
            A.acc_pass = 0;
            if (rc == SA_OK) rc = launch_search_single_f32(A, a.nq, stream);
        } else {
            rc = launch_search_single_f32(A, a.nq, stream);
        }
    } else {
        if (a.dtype == SA_BF16) rc = launch_search_multi_bf16(A, a.nq, a.M, Y.total, stream);
        else if (a.dtype == SA_FP8E4M3) rc = launch_search_multi_fp8(A, a.nq, a.M, Y.total, stream);
        else rc = launch_search_multi_f32(A, a.nq, a.M, Y.total, stream);
    }
    if (rc == SA_OK && a.p.rerank != 0) {
        // the list sits at the end of the slot list, which follows the table in each region
        const int64_t stride = (int64_t)bytes_per_slot(a.M, llog2, a.p.sync, a.R) << glog2;
        const int64_t list_off = ((int64_t)(compact ? 4 : 8) << glog2) + 4 * ((int64_t(1) << glog2) - 1025);
        rc = launch_rerank(a.vec32, a.ld32, a.queries, a.ldq, a.nq, a.d, a.metric, a.k, a.L, a.workspace, stride,
                           list_off, a.ids, a.dists, a.order, a.qk, A.ldo, stream);
    }
    if (rc == SA_OK && a.id_map) rc = launch_map_ids(a.ids, A.ldo, a.nq, a.k, a.order, a.qk, a.id_map, a.n, stream);
    return rc;
}

}  // namespace sa
