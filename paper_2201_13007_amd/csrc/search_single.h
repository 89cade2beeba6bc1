// Search with one worker (M = 1) and the visited set in the workspace: Algorithm 1, with
// the bookkeeping of Algorithm 3 at T = 1.  With a single worker the merge of Algorithm 3
// leaves the queue as it is, so the schedule (Algorithm 2) only moves the counters of
// global steps and merges.
//
// One 64-lane workgroup per query and no barrier.  Everything is sized for occupancy:
// the fewer registers a query needs, the more queries each SIMD keeps in flight to cover
// the latency of the random reads.
//
// Queue.  NI = ceil(L / 64) slots per lane hold the sorted 64-bit keys (order-preserving
// distance bits, id); entry p sits in slot p / 64 of lane p % 64.  The CHECKED flags are
// wave-uniform 64-bit masks, one per slot, so finding the first unchecked entry is scalar
// work.  The new entries of a step are merged in one pass: each destination computes how
// many of them land below it and pulls its old entry with a cross-lane permute.
//
// Visited set.  Open addressing over 32-bit entries (id + 1; zero is empty) in the
// query's workspace region, claimed with compare-and-swap; the first probe of a vertex
// goes to the line of its id block (see block_slot).  The table in use is a prefix
// of the region that doubles (rehashing the set) when it passes three quarters full.  A
// set-associative LDS filter of recently claimed or rejected ids (exact tags) sits in
// front of it: a neighbour found there is visited and needs no compare-and-swap.  When
// the query ends it clears the table in use with whole-line stores, which leaves the region zero for the next launch:
// clearing only the slots it filled would write each of their lines back a second time
// (they are long evicted by then), and listing them would cost writes of its own.
//
// Distances.  LPV lanes share one vector, each lane four float4 chunks (c = g, g + LPV,
// ...), accumulated in double precision (in float32 where the data and the query are
// integers that make every partial sum exact), summed into the group's last lane by DPP
// row shifts and broadcasts, and rounded once to float.  The query row sits in LDS.
#pragma once
#include "search_body.h"

namespace sa {
namespace single_detail {

using search_detail::KArgs;
using search_detail::NO_SLOT;

// LDS of a wavefront besides the filter of recently seen vertices: new keys, new ids, the
// query row
template <int LPV>
constexpr uint32_t single_lds_base()
{
    return 64 * 8 + 64 * 4 + 64 * LPV;
}

// log2 of the sets of the per-query LDS filter of recently seen vertices (one 32-bit word
// per set) that fits whatever the kernel's occupancy: the largest (up to 1024 sets, 4 KB)
// that keeps a wavefront's LDS within 160 KB / 28.  The launcher grows the filter beyond it
// (up to 2048 sets) where the kernel's registers hold fewer wavefronts per CU than that
// (lds_fill_log2), so that the LDS they leave idle serves the filter.
template <int LPV>
constexpr int seen_log2()
{
    int l = 10;
    while (l > 6 && single_lds_base<LPV>() + (4u << l) > 160u * 1024u / 28u) --l;
    return l;
}
using search_detail::VecSrc;
using search_detail::bpermute64;
using search_detail::distances;
using search_detail::rerank_list;
using search_detail::lanemask_lt;
using search_detail::low_bits;
using search_detail::rdlane64;

template <int NI>
struct Queue {
    uint64_t k[NI];    // keys; KEY_EMPTY past the end
    uint64_t chk[NI];  // CHECKED bits (wave-uniform)
    int len;
};

template <int NI>
__device__ __forceinline__ int first_unchecked(const Queue<NI> &Q)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const uint64_t b = low_bits(Q.len - 64 * i) & ~Q.chk[i];
        if (b) return 64 * i + __builtin_ctzll(b);
    }
    return 64 * NI;
}

// first unchecked position after p (p may be 64 NI)
template <int NI>
__device__ __forceinline__ int next_unchecked(const Queue<NI> &Q, int p)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int lo = p + 1 - 64 * i;   // positions of this slot below lo are excluded
        const uint64_t keep = lo <= 0 ? ~0ull : (lo >= 64 ? 0ull : (~0ull << lo));
        const uint64_t b = low_bits(Q.len - 64 * i) & ~Q.chk[i] & keep;
        if (b) return 64 * i + __builtin_ctzll(b);
    }
    return 64 * NI;
}

// Uniform position p: the key is read with a lane read in the branch of its slot, and a
// flag is set by a masked update of every slot.  Folding either into an access indexed by
// p / 64 would make the compiler move the arrays to scratch memory.
template <int NI>
__device__ __forceinline__ uint64_t get_key(const Queue<NI> &Q, int p)
{
    uint64_t r = KEY_EMPTY;
#pragma unroll
    for (int i = 0; i < NI; ++i)
        if (i == (p >> 6)) r = rdlane64(Q.k[i], p & 63);
    return r;
}

template <int NI>
__device__ __forceinline__ void mark_checked(Queue<NI> &Q, int p)
{
    const int s = p >> 6;
    const uint64_t bit = 1ull << (p & 63);
#pragma unroll
    for (int i = 0; i < NI; ++i) Q.chk[i] |= s == i ? bit : 0ull;
}

template <int NI>
__device__ __forceinline__ int count_less(const Queue<NI> &Q, uint64_t key)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) c += __popcll(__ballot(Q.k[i] < key));
    return c;
}

// Inserts the unchecked keys mk of the lanes in sbits (distinct, none in the queue),
// keeping at most L entries, and returns the update position: the best position one of
// them takes (L if none stays).  One pass for the whole batch: the key of rank r among
// them lands at f = (queue keys below it) + r; the landing positions form a bit mask per
// slot, and every other destination P takes the old entry at P - c(P), c(P) the number
// of landings below P, which lies in P's slot or the one before at lane (P - c(P)) mod
// 64.  stage (LDS, 64 keys) receives the batch sorted by rank.
template <int NI>
__device__ __forceinline__ int insert_batch(Queue<NI> &Q, int L, uint64_t mk, uint64_t sbits, uint64_t *stage)
{
    const int lane = __lane_id();
    const bool surv = (sbits >> lane) & 1ull;
    uint64_t land[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) land[i] = 0;
    int fmin = L;
    for (uint64_t b = sbits; b; b &= b - 1) {
        const int j = __builtin_ctzll(b);
        const uint64_t kj = rdlane64(mk, j);
        const int r = __popcll(__ballot(surv && mk < kj));
        const int f = count_less(Q, kj) + r;
        if (lane == 0) stage[r] = kj;
        fmin = min(fmin, f);
        const uint64_t bit = f < L ? 1ull << (f & 63) : 0ull;
#pragma unroll
        for (int i = 0; i < NI; ++i) land[i] |= (f >> 6) == i ? bit : 0ull;
    }
    __builtin_amdgcn_wave_barrier();
    if (fmin >= L) return L;
    const int nlen = min(L, Q.len + __popcll(sbits));
    const int i_first = fmin >> 6;
    int below = 0;   // landings in the slots under slot i
#pragma unroll
    for (int i = 0; i < NI; ++i)
        if (i < i_first) below += __popcll(land[i]);
    int base[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        base[i] = below;
        if (i >= i_first) below += __popcll(land[i]);
    }
#pragma unroll
    for (int i = NI - 1; i >= 0; --i) {
        if (i < i_first) continue;
        const int c = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(land[i] >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)land[i], (uint32_t)base[i]));
        const bool lands = (land[i] >> lane) & 1ull;
        const int src = (lane - c) & 63;
        const int addr = src << 2;
        const bool from_prev = lane < c;
        const uint64_t cur = bpermute64(addr, Q.k[i]);
        const uint64_t prv = i > 0 ? bpermute64(addr, Q.k[i > 0 ? i - 1 : 0]) : KEY_EMPTY;
        const uint64_t prv_chk = i > 0 ? Q.chk[i > 0 ? i - 1 : 0] : 0ull;
        const uint64_t sk = stage[c & 63];
        const int P = 64 * i + lane;
        const uint64_t ob = ((from_prev ? prv_chk : Q.chk[i]) >> src) & 1ull;
        const bool keep = P < nlen;
        Q.k[i] = keep ? (lands ? sk : (from_prev ? prv : cur)) : KEY_EMPTY;
        Q.chk[i] = __ballot(keep && !lands && ob);
    }
    Q.len = nlen;
    return fmin;
}

// Slots of vertex u in a table of 2^t entries (t >= 6).  The first probe keeps the 32
// vertices of one id block (u / 32) together in one 128-byte line, each at its own offset:
// neighbours that a breadth-first numbering gave nearby ids then share lines, within a
// step and from one step to the next, so a step's claims touch about half as many lines
// and most of them are still in the L2 from the step before.  Later probes move by an odd
// stride 32 r + 1 (r odd): a new line every time, and every slot of the table in turn.
__device__ __forceinline__ uint32_t block_slot(uint32_t u, int t)
{
    return ((((u >> 5) * 2654435761u) >> (37 - t)) << 5) | (u & 31u);
}

__device__ __forceinline__ uint32_t block_stride(uint32_t u, int t)
{
    const uint32_t r = (((u ^ 0x9E3779B9u) * 2654435761u) >> (37 - t)) | 1u;
    return ((r << 5) | 1u) & ((1u << t) - 1u);
}

// find or insert u; *fresh tells whether this call inserted it.  NO_SLOT: table full.
__device__ __forceinline__ uint32_t claim(uint32_t *T, int log2cap, uint32_t u, bool *fresh)
{
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t s = block_slot(u, log2cap);
    const uint32_t step = block_stride(u, log2cap);
    *fresh = false;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const uint32_t old = atomicCAS(&T[s], 0u, u + 1u);
        if (old == 0u) {
            *fresh = true;
            return s;
        }
        if (old == u + 1u) return s;
        s = (s + step) & mask;
    }
    return NO_SLOT;
}

// The rest of claim() after its first probe, given what that probe's compare-and-swap at
// block_slot(u, log2cap) returned: lets the caller issue the first probes of a step, go on
// with other loads, and read the results later.
__device__ __forceinline__ uint32_t claim_rest(uint32_t *T, int log2cap, uint32_t u, uint32_t old, bool *fresh)
{
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t s = block_slot(u, log2cap);
    *fresh = old == 0u;
    if (old == 0u || old == u + 1u) return s;
    const uint32_t step = block_stride(u, log2cap);
    for (uint32_t probe = 1; probe <= mask; ++probe) {
        s = (s + step) & mask;
        old = atomicCAS(&T[s], 0u, u + 1u);
        if (old == 0u) {
            *fresh = true;
            return s;
        }
        if (old == u + 1u) return s;
    }
    return NO_SLOT;
}

// Moves the visited set from the table in use (2^t1 entries) into one twice as large,
// 2^t2 entries at the same address (the region holds the largest; past the table in use
// it is zero).  The entries are copied out to scratch (the second half of the region) and
// the table is cleared; then they are inserted again and scratch is cleared.  Returns the
// number of entries moved.  The whole wavefront takes part.
__device__ __forceinline__ int grow_table(uint32_t *tbl, uint32_t *scratch, int t1, int t2)
{
    const int lane = __lane_id();
    int cnt = 0;
    for (int b = 0; b < (1 << t1); b += 64) {   // 2^t1 >= 64 entries
        const uint32_t e = tbl[b + lane];
        const uint64_t m = __ballot(e != 0u);
        if (e != 0u) scratch[cnt + __popcll(m & lanemask_lt())] = e;
        tbl[b + lane] = 0u;
        cnt += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < cnt; i += 64) {
        bool fresh;
        (void)claim(tbl, t2, scratch[i] - 1u, &fresh);
        scratch[i] = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    return cnt;
}

// Zeroes the first 2^t entries of tbl (2^t >= 64, 16-byte aligned) with 16-byte stores.
__device__ __forceinline__ void clear_table(uint32_t *tbl, int t)
{
    uint4 *const p = reinterpret_cast<uint4 *>(tbl);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int i = __lane_id(); i < (1 << (t - 2)); i += 64) p[i] = z;
}

template <int LPV, int NI, bool L2, int DT, bool ACC32>
__device__ __forceinline__ void single_query(const KArgs &A, int64_t qi, uint32_t *tbl)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint64_t *const nkey = reinterpret_cast<uint64_t *>(smem);    // [64] keys of new vertices
    int32_t *const sid = reinterpret_cast<int32_t *>(nkey + 64);   // [64] their ids
    float *const qs = reinterpret_cast<float *>(sid + 64);          // [16 LPV] the query
    // [SEEN] sets of recently claimed or rejected vertices: a vertex found here is visited and
    // needs no compare-and-swap in the workspace table.  A vertex's id u is mapped by
    // h = u * K_B mod 2^B, with K_B the odd number nearest 2^B / golden ratio (Fibonacci
    // hashing at B bits: one-to-one on ids of B bits, and ids close together land in sets far
    // apart); the top SEEN_LOG2 bits of h pick the set and the other tb = B - SEEN_LOG2 bits
    // are the tag, so a tag names one vertex exactly.  A set's word holds a count of valid
    // tags in its top two bits and up to W = min(3, 30 / tb) tags below, newest lowest; a new
    // tag pushes the oldest out.  (Ids of more than 15 + SEEN_LOG2 bits: no filter.)
    uint32_t *const seen = reinterpret_cast<uint32_t *>(qs + 16 * LPV);
    const int SEEN_LOG2 = A.seen_log2;
    const int SEEN = 1 << SEEN_LOG2;
    const int hbits = A.idbits > SEEN_LOG2 ? A.idbits : SEEN_LOG2 + 1;
    const int tbits = hbits - SEEN_LOG2;
    const bool filter = tbits <= 15;
    const uint32_t hmul = (2654435769u >> (32 - hbits)) | 1u;
    const uint32_t tmask = (1u << tbits) - 1u;
    const uint32_t ways = tbits <= 10 ? 3u : 2u;
    const uint32_t tagbits = filter ? (1u << (ways * tbits)) - 1u : 0u;

    const int lane = __lane_id();
    const int R = A.R, g2 = A.glog2;
    const int L = A.qL ? __builtin_amdgcn_readfirstlane(A.qL[qi]) : A.L;
    const int kq = A.qk ? __builtin_amdgcn_readfirstlane(A.qk[qi]) : A.k;
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    // the second half of the region: scratch while the table grows, and the list handed
    // to the re-rank kernel
    uint32_t *const slots = tbl + (1u << g2);
    // the table in use is the first 2^t2 entries of the region's 2^g2; it doubles when
    // the visited set would pass three quarters of it
    int t2 = A.glog2_init;
    int cap = (3 << t2) / 4;
    const VecSrc V{A.codes, A.scale, A.ldc};

    {
        const int nch = A.d >> 2;
        const float *qrow = A.queries + qi * A.ldq;
        const float lo = (float)A.int_lo, hi = (float)A.int_hi;
        bool outside = false;   // some coordinate is not an integer in [int_lo, int_hi]
        for (int c = lane; c < 4 * LPV; c += 64) {
            const float4 v = c < nch ? *reinterpret_cast<const float4 *>(qrow + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
            reinterpret_cast<float4 *>(qs)[c] = v;
            if (c < nch)
                outside |= !(v.x == rintf(v.x) && v.x >= lo && v.x <= hi) || !(v.y == rintf(v.y) && v.y >= lo && v.y <= hi) ||
                           !(v.z == rintf(v.z) && v.z >= lo && v.z <= hi) || !(v.w == rintf(v.w) && v.w >= lo && v.w <= hi);
        }
        // with two passes, each query is searched by exactly one of them
        if (A.acc_pass >= 0 && (__ballot(outside) == 0ull) != (A.acc_pass == 1)) return;
        if (lane == 0) sid[0] = A.entry;
        for (int i = lane; i < SEEN; i += 64) seen[i] = 0u;
    }
    __builtin_amdgcn_wave_barrier();

    // one worker: every local step expands one vertex, and every visited vertex has one
    // table slot, so the step count is the expansion count and the slot count is the
    // distance count
    int nslot = 0, substeps = 0, gsteps = 0, merges = 0, flags = 0;
    Queue<NI> Q;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        Q.k[i] = KEY_EMPTY;
        Q.chk[i] = 0;
    }
    // dist(P, Q); P goes into the queue and the visited set
    distances<LPV, L2, DT, ACC32>(V, A.d, qs, sid, 1, nkey);
    __builtin_amdgcn_wave_barrier();
    {
        const uint64_t k0 = nkey[0];
        if (lane == 0) Q.k[0] = k0;
        Q.len = 1;
        bool fresh = false;
        if (lane == 0) (void)claim(tbl, t2, (uint32_t)A.entry, &fresh);
        nslot = 1;
    }
    __builtin_amdgcn_wave_barrier();

    const int max_sub = A.max_substeps;
    const int32_t n = (int32_t)A.n;
    // Two walkers merging after every local step (Top-2, M = 2 with the every-step schedule,
    // R <= 32) also run here: the merge of their two local queues is the queue with both
    // expansions' new vertices inserted, so one queue serves.  Walker 0 expands the first
    // unchecked entry on lanes 0-31, walker 1 the second on lanes 32-63.
    const bool two = A.M == 2;
    // Two vectors per lane group in each pass of the distance loop (one round trip for 16
    // new vertices at d = 128 instead of two) where that pays for its registers, with up to
    // three queue slots per lane: float32 rows accumulated in float32 or wide enough
    // (d > 256) that a pass holds at most two vectors, and bf16 rows up to two slots (at
    // three the registers would cost two waves of seven).  Measured on 1M-row sets, d = 128
    // integer data: +2.3% (two walkers, L = 192) and +2.8% (one, L = 128) at one wave less;
    // d = 960: +2% at L = 64 and 128; d = 96 bf16: +2.8% (two walkers, L = 112, re-ranked);
    // d = 96 float32 in double 1-5% and fp8 1-4% slower.
    constexpr int GATHER_PB =
        (DT == SA_BF16 && NI <= 2) || (DT == SA_F32 && NI <= 3 && (ACC32 || LPV >= 32)) ? 2 : 1;
    // Gathers alongside the claims (SPEC) where the filter is the full 1024 sets, so that
    // few vertices that reach the table are already in it (with the 128 sets that d = 960
    // leaves room for, many are, and each wasted read is a 3.8 KB row: 30-60% slower), and
    // where the five registers it takes cost no wave that pays (not at NI = 7, 8; at NI = 3
    // with float32 accumulation the timed two-walker search went 0.5% slower at 5 waves).
    // Measured on 1M rows: d = 128 one walker +2.5% (L = 128), +2.3% (256), +3.4% (384);
    // d = 96 in double +4% (one walker, L = 128) and +3% (two, L = 192).
    constexpr bool SPEC = seen_log2<LPV>() >= 10 && NI != 7 && NI != 8 && !(ACC32 && NI == 3);
    const bool second = two && lane >= 32;
    int m = two && !A.staged ? 2 : 1;   // walkers active in the next step (staged: 1, then 2)
    int nexp = 0;
    // this lane's entry of an adjacency row (R <= 64); lanes past R load entry 0 and drop it
    const int aidx = two ? (lane & 31) : lane;
    const int32_t *const adj_lane = A.adj + (aidx < R ? aidx : 0);
    int32_t pv = -1, pv2 = -1, pu = -1;   // vertices whose rows are prefetched, and this lane's entry
    int cur = 0;
    bool stop = false;
    while (cur < Q.len && !stop) {
        gsteps++;
        int sub_in_step = 0;
        for (;;) {
            if (substeps >= max_sub) {
                flags |= SA_QFLAG_MAX_STEPS;
                stop = true;
                break;
            }
            substeps++;
            sub_in_step++;
            const int32_t v = key_id(get_key(Q, cur));
            mark_checked(Q, cur);
            int32_t v2 = -1;
            if (m == 2) {
                const int c2 = first_unchecked(Q);
                if (c2 < Q.len) {
                    v2 = key_id(get_key(Q, c2));
                    mark_checked(Q, c2);
                }
            }
            nexp += v2 >= 0 ? 2 : 1;
            const int32_t vl = second ? v2 : v;   // the vertex whose row this lane reads
            int32_t u = pu;
            if (vl != (second ? pv2 : pv)) u = adj_lane[(int64_t)(vl >= 0 ? vl : v) * R];
            // prefetch the rows of the next candidates while this step runs
            const int nxt = first_unchecked(Q);
            pv = nxt < Q.len ? key_id(get_key(Q, nxt)) : v;
            if (two) {
                const int nx2 = next_unchecked(Q, nxt);
                pv2 = nx2 < Q.len ? key_id(get_key(Q, nx2)) : pv;
            }
            pu = adj_lane[(int64_t)(second ? pv2 : pv) * R];
            if (aidx >= R || vl < 0 || u < 0 || u >= n) u = -1;   // idle walker, padding, malformed entries
            bool fresh = false;
            const uint32_t h = ((uint32_t)u * hmul) & (0xFFFFFFFFu >> (32 - hbits));
            const uint32_t hs = h >> tbits, tag = h & tmask;
            const uint32_t sw = u >= 0 && filter ? seen[hs] : 0u;
            const uint32_t cnt = sw >> 30;
            const bool known = (cnt > 0u && (sw & tmask) == tag) || (cnt > 1u && ((sw >> tbits) & tmask) == tag) ||
                               (cnt > 2u && ((sw >> (2 * tbits)) & tmask) == tag);
            const bool ask = u >= 0 && !known;
            // The first probe of each claim goes out now.  With SPEC the vectors of every vertex
            // that passed the filter are read while it is in flight: nearly all of them turn out
            // new, and the keys of the few found present are dropped after.  Without, the claims
            // settle first and only new vertices are read.
            uint32_t old = 0u;
            if (ask) old = atomicCAS(&tbl[block_slot((uint32_t)u, t2)], 0u, (uint32_t)u + 1u);
            if (ask && filter) seen[hs] = (min(cnt + 1u, ways) << 30) | (((sw << tbits) | tag) & tagbits);
            if (!SPEC && ask) (void)claim_rest(tbl, t2, (uint32_t)u, old, &fresh);
            const bool send = SPEC ? ask : fresh;   // the vertices whose vectors are read
            const uint64_t am = __ballot(send);
            const int nsend = __popcll(am);
            const int apos = __popcll(am & lanemask_lt());
            if (send) sid[apos] = u;
            __builtin_amdgcn_wave_barrier();
            distances<LPV, L2, DT, ACC32, GATHER_PB>(V, A.d, qs, sid, nsend, nkey);
            if (SPEC && ask) (void)claim_rest(tbl, t2, (uint32_t)u, old, &fresh);
            nslot += __popcll(__ballot(fresh));
            if (SPEC) {
                __builtin_amdgcn_wave_barrier();
                if (send && !fresh) nkey[apos] = KEY_EMPTY;
            }
            __builtin_amdgcn_wave_barrier();
            const uint64_t mk = lane < nsend ? nkey[lane] : KEY_EMPTY;
            __builtin_amdgcn_wave_barrier();
            // insert the survivors; the update position is the best place one of them takes
            const uint64_t worst = Q.len == L ? get_key(Q, L - 1) : KEY_EMPTY;
            const uint64_t sbits = __ballot(mk < worst);
            const int U = sbits ? insert_batch(Q, L, mk, sbits, nkey) : L;
            cur = first_unchecked(Q);
            if (nslot + (two ? 2 * R : R) > cap) {
                if (t2 < g2) {
                    // (one doubling suffices: nslot <= cap before, and at most 64 new < cap)
                    ++t2;
                    (void)grow_table(tbl, slots, t2 - 1, t2);
                    cap = (3 << t2) / 4;
                    flags |= SA_QFLAG_SPILLED;
                } else {
                    flags |= SA_QFLAG_CAPACITY;
                    stop = true;
                    break;
                }
            }
            bool merge_now;
            if (A.sync == SA_SYNC_BSP) merge_now = true;
            else if (A.sync == SA_SYNC_STATIC) merge_now = A.static_I > 0 && sub_in_step >= A.static_I;
            else merge_now = (double)U >= (double)L * A.rho;
            if (cur >= Q.len || merge_now) break;
        }
        merges++;   // the queue is S unchanged
        if (two) m = 2;
    }

    if (A.rerank != 0) {
        // hand the first nr entries of the final list to the re-rank kernel
        const int nr = A.rerank < 0 ? Q.len : min(A.rerank, Q.len);
        int32_t *const list = rerank_list(slots, g2);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            if (64 * i + lane < nr) list[1 + 64 * i + lane] = key_id(Q.k[i]);
        if (lane == 0) list[0] = nr;
    } else {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int p = 64 * i + lane;
            if (p < kq) {
                const bool ok = p < Q.len;
                A.ids[qi * A.ldo + p] = ok ? key_id(Q.k[i]) : -1;
                A.dists[qi * A.ldo + p] = ok ? key_dist(Q.k[i]) : __builtin_inff();
            }
        }
    }
    // leave the workspace zero-filled for the next launch
    clear_table(tbl, t2);
    if (lane == 0 && A.stats) {
        sa_query_stats st;
        st.global_steps = gsteps;
        st.substeps = substeps;
        st.expansions = nexp;
        st.dist_comps = nslot;
        st.merges = merges;
        st.flags = flags;
        st.t_start = t_start;
        st.t_end = __builtin_amdgcn_s_memrealtime();
        A.stats[qi] = st;
    }
}

// Workgroup b runs job b: query order[b] (or b), in workspace region b.  The hardware
// dispatcher hands out workgroups in index order as slots free up, so a batch ordered
// longest first is scheduled longest first.  (A persistent loop over jobs in one
// workgroup was measured: any loop around the search costs 17-36 more VGPRs, about a
// third of the occupancy this latency-bound search lives on.)
template <int LPV, int NI, bool L2, int DT, bool ACC32>
__global__ void __launch_bounds__(64) search_single(KArgs A)
{
    const int32_t job = blockIdx.x;
    uint32_t *const tbl = reinterpret_cast<uint32_t *>(A.ghash) + ((size_t)job << (A.glog2 + 1));
    single_query<LPV, NI, L2, DT, ACC32>(A, A.order ? A.order[job] : job, tbl);
}

// Persistent form: each resident workgroup takes jobs from the device counter until none
// is left, every one in its own workspace region (see KArgs::jobctr).
template <int LPV, int NI, bool L2, int DT, bool ACC32>
__global__ void __launch_bounds__(64) search_single_loop(KArgs A)
{
    uint32_t *const tbl = reinterpret_cast<uint32_t *>(A.ghash) + ((size_t)blockIdx.x << (A.glog2 + 1));
    for (;;) {
        int job = 0;
        if (__lane_id() == 0) job = atomicAdd(A.jobctr, 1);
        job = __builtin_amdgcn_readfirstlane(job);
        if (job >= A.njobs) break;
        // (loads after stores are vector loads: made wave-uniform again, or everything
        // derived from the query index would take vector registers)
        const int32_t qi = A.order ? __builtin_amdgcn_readfirstlane(A.order[job]) : job;
        single_query<LPV, NI, L2, DT, ACC32>(A, qi, tbl);
    }
    if (__lane_id() == 0) search_detail::release_jobs(A.jobctr);
}

template <int LPV, int NI, int DT, bool ACC32>
hipError_t launch1(const KArgs &A, int64_t nq, hipStream_t s)
{
    constexpr uint32_t base = single_lds_base<LPV>();
    KArgs B = A;
    if (A.jobctr) {
        auto k = A.metric == SA_L2 ? search_single_loop<LPV, NI, true, DT, ACC32>
                                   : search_single_loop<LPV, NI, false, DT, ACC32>;
        hipError_t e = lds_fill_log2(reinterpret_cast<const void *>(k), 64, base, seen_log2<LPV>(), 11, &B.seen_log2);
        if (e != hipSuccess) return e;
        const uint32_t lds = base + (4u << B.seen_log2);
        int64_t grid = nq;
        e = resident_grid(reinterpret_cast<const void *>(k), 64, lds, nq, &grid);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64), lds, s, B);
        return hipGetLastError();
    }
    auto k = A.metric == SA_L2 ? search_single<LPV, NI, true, DT, ACC32> : search_single<LPV, NI, false, DT, ACC32>;
    const hipError_t e = lds_fill_log2(reinterpret_cast<const void *>(k), 64, base, seen_log2<LPV>(), 11, &B.seen_log2);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)nq), dim3(64), base + (4u << B.seen_log2), s, B);
    return hipGetLastError();
}

template <int LPV, int DT, bool ACC32>
hipError_t launch1_ni(const KArgs &A, int64_t nq, hipStream_t s)
{
    const int ni = (A.L + 63) / 64;
    if (ni <= 1) return launch1<LPV, 1, DT, ACC32>(A, nq, s);
    if (ni <= 2) return launch1<LPV, 2, DT, ACC32>(A, nq, s);
    if (ni <= 3) return launch1<LPV, 3, DT, ACC32>(A, nq, s);
    if (ni <= 4) return launch1<LPV, 4, DT, ACC32>(A, nq, s);
    if (ni <= 5) return launch1<LPV, 5, DT, ACC32>(A, nq, s);
    if (ni <= 6) return launch1<LPV, 6, DT, ACC32>(A, nq, s);
    if (ni <= 7) return launch1<LPV, 7, DT, ACC32>(A, nq, s);
    if (ni <= 8) return launch1<LPV, 8, DT, ACC32>(A, nq, s);
    return launch1<LPV, 16, DT, ACC32>(A, nq, s);
}

// one instantiation per storage type, each in a file of its own (search_single_*.hip)
// float32 accumulation is compiled for float32 storage up to d = 256 (integer data such
// as 8-bit descriptors); the launcher asks for it only there
template <int LPV, int DT>
hipError_t launch_lpv(const KArgs &A, int64_t nq, hipStream_t s)
{
    if constexpr (DT == SA_F32 && LPV <= 16)
        if (A.acc_pass == 1) return launch1_ni<LPV, DT, true>(A, nq, s);
    return launch1_ni<LPV, DT, false>(A, nq, s);
}

template <int DT>
int launch_dt(const KArgs &A, int64_t nq, hipStream_t s)
{
    hipError_t e;
    switch (search_detail::lanes_per_vector(A.d)) {
    case 1: e = launch_lpv<1, DT>(A, nq, s); break;
    case 2: e = launch_lpv<2, DT>(A, nq, s); break;
    case 4: e = launch_lpv<4, DT>(A, nq, s); break;
    case 8: e = launch_lpv<8, DT>(A, nq, s); break;
    case 16: e = launch_lpv<16, DT>(A, nq, s); break;
    case 32: e = launch_lpv<32, DT>(A, nq, s); break;
    default: e = launch_lpv<64, DT>(A, nq, s); break;
    }
    if (e != hipSuccess) return hip_fail(e, "search kernel launch");
    return SA_OK;
}

}  // namespace single_detail
}  // namespace sa
