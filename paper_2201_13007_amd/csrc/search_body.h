// Intra-query parallel graph search (Speed-ANN, arXiv 2201.13007, Algorithm 3 with
// CheckMetrics of Algorithm 2; Algorithm 1 when there is one worker), for gfx950.
//
// One workgroup runs one query; worker t of Algorithm 3 is wavefront t.
//
// Each worker's local queue LS[t] (capacity L) lives in that wavefront's registers:
// NI = ceil(L / 64) slots per lane hold the sorted 64-bit keys (distance bits, id) and a
// 32-bit tag each, entry p in slot p / 64 of lane p % 64.  The tag holds the index of
// the S entry it was copied from (0xFFFF for vertices the worker inserted itself), MINE
// (the worker may expand it) and CHECKED.  Finding the first candidate to expand and
// counting smaller keys are ballots; a local step's new entries are merged in one pass
// of cross-lane permutes.  No memory round trip.
//
// Distances: LPV lanes share one vector, each lane four float4 chunks, accumulated in
// double precision (the single-worker kernel can also accumulate exact integer data in
// float32), summed by DPP row shifts and rounded once to float; the query sits in LDS for
// all workers.  Every gather and row load is issued unconditionally (from a
// clamped address): loads under lane conditions each get their own wait.
//
// Global steps with one active worker (every step when M = 1; the first step of a
// staged search) run on wavefront 0 alone, with no barrier: the merge of a single local
// queue into S leaves S equal to that queue, so S is the queue in registers.  With two
// or more workers S sits in LDS, the local steps proceed in lockstep between two
// barriers, and the merge ranks every surviving entry by counting smaller keys across
// the queues.
//
// The visited set is an open-addressing hash of 64-bit entries ((id + 1) << 32 | tag),
// zero meaning empty, kept in LDS or in a per-query region of the caller's workspace
// (a query moves it there when the LDS table passes half full).  A vertex reached by
// several workers in one local step goes to the lowest (worker, adjacency slot): claims
// carry that order in their tag and the smallest tag of the step wins (two phases around
// a barrier), which is the order a sequential emulation visits them in.  Workspace slots
// a query writes are listed and zeroed again before it ends, so the workspace stays
// zero-filled between launches.
#pragma once
#include "sa_internal.h"

#include <type_traits>

namespace sa {
namespace search_detail {

constexpr uint32_t META_SIDX = 0xFFFFu;
constexpr uint32_t META_MINE = 1u << 16;
constexpr uint32_t META_CHK = 1u << 17;
constexpr int MAXW = 16;
constexpr int PUBCAP = 512;   // new keys published per round of a merge
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;

struct Ctrl {
    int32_t U[MAXW];
    int32_t work[MAXW];
    int32_t nnew[MAXW];
    int32_t slen;
    int32_t hcount;   // visited vertices
    int32_t nexp;     // expansions
    int32_t mode;     // 0: visited set in LDS, 1: in the workspace
    int32_t flags;
    int32_t nslot;    // workspace-table slots written (zeroed again at the end)
    int32_t done;     // the search ended while one worker was active
    int32_t gsteps, substeps, merges, epoch;
    int32_t job;      // persistent form: the job the workgroup runs next
};

struct KArgs {
    const void *codes;           // stored vectors: rows of ldc elements of the index's dtype
    const float *scale;          // fp8: one scale per vector
    int64_t ldc;
    const float *vec32;          // float32 vectors for the re-rank
    int64_t ld32;
    int32_t rerank;
    const int32_t *adj;
    const float *queries;
    int64_t ldq;
    int32_t *ids;
    float *dists;
    sa_query_stats *stats;
    unsigned long long *ghash;   // per query: 2^glog2 table entries, then 2^glog2 slot indices
    int64_t n;
    int32_t d, metric, R, entry, k, L, M, sync, static_I, staged, max_substeps;
    double rho;
    int32_t glog2, llog2;        // llog2 == 0: no LDS table
    int32_t glog2_init;          // single worker: log2 of the table a query starts in (<= glog2)
    // single worker over integer-valued float32 vectors in [int_lo, int_hi] (see
    // index_integer_range): pass 1 takes the queries that are integers in that range and
    // accumulates in float32, pass 0 takes the others; -1: one pass takes every query
    int32_t int_lo, int_hi, acc_pass;
    int32_t idbits;              // vertex ids fit in idbits bits (2^idbits >= n)
    int32_t seen_log2;           // single-worker kernel: log2 of the seen filter's sets (set by its launcher)
    uint32_t o_skey, o_srank, o_schk, o_pub, o_newkey, o_claim, o_ctrl, o_hash, o_q;
    // batches: per-query L and k (null: L and k above) and the query each workgroup
    // runs (null: workgroup b runs query b)
    const int32_t *qL, *qk, *order;
    int64_t ldo;                 // row stride of ids and dists
    // persistent form (null: one workgroup per job): jobctr[0] hands out the jobs 0 ..
    // njobs - 1, jobctr[1] counts the workgroups that found none left; both are zero
    // before a launch and the last workgroup sets them back to zero
    int32_t *jobctr;
    int32_t njobs;
};

// Persistent form, end of a workgroup (one thread): the last one to finish puts the job
// counters back to zero for the next launch.
__device__ __forceinline__ void release_jobs(int32_t *ctr)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (atomicAdd(ctr + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(ctr, 0);
        atomicExch(ctr + 1, 0);
    }
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t hash_slot(uint32_t id, int log2cap)
{
    return (id * 2654435761u) >> (32 - log2cap);
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l)
{
    return ((uint64_t)rdlane((uint32_t)(v >> 32), l) << 32) | rdlane((uint32_t)v, l);
}
// Phase one of a claim: find or insert u, leaving the smallest tag of this local step
// in its slot.  Returns the slot, or NO_SLOT if the table is full; *fresh tells whether
// this call inserted u.
__device__ uint32_t visit_claim(unsigned long long *H, int log2cap, uint32_t u, uint32_t tag, uint32_t epoch,
                                bool *fresh)
{
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t s = hash_slot(u, log2cap);
    const unsigned long long want = ((unsigned long long)(u + 1) << 32) | tag;
    *fresh = false;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        unsigned long long old = atomicCAS(&H[s], 0ull, want);
        if (old == 0ull) {
            *fresh = true;
            return s;
        }
        if ((uint32_t)(old >> 32) == u + 1) {
            if (((uint32_t)old >> 10) == epoch) atomicMin(&H[s], want);
            return s;
        }
        s = (s + 1) & mask;
    }
    return NO_SLOT;
}

__device__ __forceinline__ unsigned long long read_slot_global(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lower_bound: number of entries of the sorted array a[0..n) smaller than key
__device__ __forceinline__ int lower_bound(const uint64_t *a, int n, uint64_t key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- cross-lane helpers

constexpr int DPP_ROW_SHR = 0x110;     // + n: row_shr:n
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

// lanes whose DPP source is invalid (outside the row or the enabled rows) keep `old`
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t v, uint32_t old)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, 0xF, false);
}

template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = dpp32<CTRL, ROWMASK>((uint32_t)b, 0u);
    const uint32_t hi = dpp32<CTRL, ROWMASK>((uint32_t)(b >> 32), 0u);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// sum of each group of LPV lanes, left in the group's last lane
template <int LPV>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (LPV >= 2) v += dpp_f64<DPP_ROW_SHR + 1>(v);
    if constexpr (LPV >= 4) v += dpp_f64<DPP_ROW_SHR + 2>(v);
    if constexpr (LPV >= 8) v += dpp_f64<DPP_ROW_SHR + 4>(v);
    if constexpr (LPV >= 16) v += dpp_f64<DPP_ROW_SHR + 8>(v);
    if constexpr (LPV >= 32) v += dpp_f64<DPP_ROW_BCAST15, 0xA>(v);
    if constexpr (LPV >= 64) v += dpp_f64<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

// the same sums in float32
template <int LPV>
__device__ __forceinline__ float group_sum_f32(float v)
{
    if constexpr (LPV >= 2) v += __uint_as_float(dpp32<DPP_ROW_SHR + 1>(__float_as_uint(v), 0u));
    if constexpr (LPV >= 4) v += __uint_as_float(dpp32<DPP_ROW_SHR + 2>(__float_as_uint(v), 0u));
    if constexpr (LPV >= 8) v += __uint_as_float(dpp32<DPP_ROW_SHR + 4>(__float_as_uint(v), 0u));
    if constexpr (LPV >= 16) v += __uint_as_float(dpp32<DPP_ROW_SHR + 8>(__float_as_uint(v), 0u));
    if constexpr (LPV >= 32) v += __uint_as_float(dpp32<DPP_ROW_BCAST15, 0xA>(__float_as_uint(v), 0u));
    if constexpr (LPV >= 64) v += __uint_as_float(dpp32<DPP_ROW_BCAST31, 0xC>(__float_as_uint(v), 0u));
    return v;
}

// bits [0, n) set, n in [0, 64]
__device__ __forceinline__ uint64_t low_bits(int n)
{
    return n <= 0 ? 0ull : (n >= 64 ? ~0ull : (~0ull >> (64 - n)));
}

__device__ __forceinline__ uint64_t bpermute64(int addr, uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// lanes per vector: the smallest power of two that leaves at most four float4 chunks per
// lane (d <= 1024)
__host__ __device__ inline int lanes_per_vector(int d)
{
    const int nch = d / 4;
    int lpv = 1;
    while (lpv < 64 && 4 * lpv < nch) lpv *= 2;
    return lpv;
}

// Where a kernel reads vectors: rows of ld elements of storage type DT (sa_dtype).
struct VecSrc {
    const void *p;
    const float *scale;   // SA_FP8E4M3 only
    int64_t ld;
};

// Coordinates 4c .. 4c+3 of a row as stored: this raw form is what stays in registers
// while the loads are in flight, and is decoded where the distance uses it.
template <int DT> struct Raw4T { using type = uint32_t; };
template <> struct Raw4T<SA_F32> { using type = float4; };
template <> struct Raw4T<SA_BF16> { using type = uint2; };
template <int DT> using Raw4 = typename Raw4T<DT>::type;

template <int DT>
__device__ __forceinline__ Raw4<DT> load_raw4(const VecSrc &V, int32_t id, int c)
{
    if constexpr (DT == SA_F32)
        return *reinterpret_cast<const float4 *>(static_cast<const float *>(V.p) + (int64_t)id * V.ld + 4 * c);
    else if constexpr (DT == SA_BF16)
        return *(reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(V.p) + (int64_t)id * V.ld) + c);
    else
        return *(reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(V.p) + (int64_t)id * V.ld) + c);
}

// Keys of the vectors ids[0..n) (n <= 64) to out[0..n), 64 / LPV vectors per pass; qs is
// the query, zero padded to 16 LPV floats.  The loads are issued unconditionally, from
// clamped addresses (a dropped id reads row 0): loads under lane conditions each get their
// own wait, which would turn one memory round trip into four.  (Written as a pass loop
// over arrays: the same steps as a per-vector helper cost some twenty more registers.)
// ACC32: accumulate in float32 (only where every partial sum is an integer below 2^24, so
// that the float32 sum is exact and equals the double one)
// PB: vectors per lane group in one pass (PB 64 / LPV a pass, each pass one memory round
// trip; each more in flight costs sixteen registers at d = 128)
template <int LPV, bool L2, int DT, bool ACC32 = false, int PB = 1>
__device__ __forceinline__ void distances(const VecSrc &V, int d, const float *qs, const int32_t *ids, int n,
                                          uint64_t *out)
{
    constexpr int VPW = 64 / LPV;
    const int lane = __lane_id(), grp = lane / LPV, g = lane % LPV;
    const int nch = d >> 2;
    for (int p0 = 0; p0 < n; p0 += VPW * PB) {
        Raw4<DT> x[PB][4];
        float sc[PB];
        int32_t id[PB];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
            const int idx = p0 + pp * VPW + grp;
            const int32_t raw = ids[idx & 63];
            id[pp] = idx < n ? raw : -1;
            const int32_t row = id[pp] < 0 ? 0 : id[pp];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = g + LPV * i;
                x[pp][i] = load_raw4<DT>(V, row, c < nch ? c : 0);
            }
            sc[pp] = DT == SA_FP8E4M3 ? V.scale[row] : 1.f;
        }
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
            using Acc = typename std::conditional<ACC32, float, double>::type;
            Acc acc = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool in = g + LPV * i < nch;
                const float4 a = reinterpret_cast<const float4 *>(qs)[g + LPV * i];
                // codes outside the row are taken as code 0, which is 0.0 in every storage
                // type; the selects act on the loaded registers themselves (on a decoded
                // copy they cost some twenty-five more registers)
                float bx, by, bz, bw;
                if constexpr (DT == SA_F32) {
                    bx = in ? x[pp][i].x : 0.f; by = in ? x[pp][i].y : 0.f;
                    bz = in ? x[pp][i].z : 0.f; bw = in ? x[pp][i].w : 0.f;
                } else if constexpr (DT == SA_BF16) {
                    const uint32_t lo = in ? x[pp][i].x : 0u, hi = in ? x[pp][i].y : 0u;
                    bx = __uint_as_float(lo << 16); by = __uint_as_float(lo & 0xFFFF0000u);
                    bz = __uint_as_float(hi << 16); bw = __uint_as_float(hi & 0xFFFF0000u);
                } else {
                    // e4m3 -> f16 bit pattern: same mantissa bits, exponent bias 15 instead
                    // of 7, so every value, subnormals included, comes out 2^-8 too small;
                    // 2^8 joins the scale, and s * 2^8 * v rounds once like s * value.  (The
                    // hardware fp8 conversion gives the same values but its vector results
                    // cost the caller about twenty registers.)  Codes 0x7F / 0xFF, NaN in
                    // e4m3, are never written and decode as 480 / -480 here.
                    const uint32_t w = in ? x[pp][i] : 0u;
                    const uint32_t h0 = ((w & 0x7Fu) << 7) | ((w & 0x80u) << 8);
                    const uint32_t h1 = ((w >> 8 & 0x7Fu) << 7) | ((w >> 8 & 0x80u) << 8);
                    const uint32_t h2 = ((w >> 16 & 0x7Fu) << 7) | ((w >> 16 & 0x80u) << 8);
                    const uint32_t h3 = ((w >> 24 & 0x7Fu) << 7) | ((w >> 24 & 0x80u) << 8);
                    const float s = sc[pp] * 256.f;
                    bx = s * (float)__builtin_bit_cast(_Float16, (uint16_t)h0);
                    by = s * (float)__builtin_bit_cast(_Float16, (uint16_t)h1);
                    bz = s * (float)__builtin_bit_cast(_Float16, (uint16_t)h2);
                    bw = s * (float)__builtin_bit_cast(_Float16, (uint16_t)h3);
                }
                if constexpr (L2) {
                    const Acc t0 = (Acc)a.x - (Acc)bx, t1 = (Acc)a.y - (Acc)by;
                    const Acc t2 = (Acc)a.z - (Acc)bz, t3 = (Acc)a.w - (Acc)bw;
                    acc += t0 * t0; acc += t1 * t1; acc += t2 * t2; acc += t3 * t3;
                } else {
                    acc += (Acc)a.x * (Acc)bx; acc += (Acc)a.y * (Acc)by;
                    acc += (Acc)a.z * (Acc)bz; acc += (Acc)a.w * (Acc)bw;
                }
            }
            if constexpr (ACC32) acc = group_sum_f32<LPV>(acc);
            else acc = group_sum<LPV>(acc);
            const int idx = p0 + pp * VPW + grp;
            if (g == LPV - 1 && idx < n) out[idx] = make_key(L2 ? (float)acc : (float)(-acc), id[pp]);
        }
    }
}

// Where a query leaves its final list for the re-rank: the last 1025 entries of its slot
// list (a count, then up to 1024 ids).  Slots stop at three quarters of a table of at
// least 4096, so the search never writes there; the re-rank zeroes it again.
__device__ __forceinline__ int32_t *rerank_list(uint32_t *slots, int glog2)
{
    return reinterpret_cast<int32_t *>(slots + (1u << glog2) - 1025u);
}

// ---------------------------------------------------------------- register queue

template <int NI>
struct RList {
    uint64_t k[NI];
    uint32_t m[NI];
};

template <int NI>
__device__ __forceinline__ void rl_clear(RList<NI> &l)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        l.k[i] = KEY_EMPTY;
        l.m[i] = 0;
    }
}

// entries with a key smaller than key (unused slots hold KEY_EMPTY)
template <int NI>
__device__ __forceinline__ int rl_count_less(const RList<NI> &l, uint64_t key)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) c += __popcll(__ballot(l.k[i] < key));
    return c;
}

// first entry the worker may expand (MINE and not CHECKED), or NI * 64
template <int NI>
__device__ __forceinline__ int rl_first_expandable(const RList<NI> &l)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const uint64_t b = __ballot((l.m[i] & (META_MINE | META_CHK)) == META_MINE);
        if (b) return i * 64 + __builtin_ctzll(b);
    }
    return NI * 64;
}

template <int NI>
__device__ __forceinline__ void rl_get(const RList<NI> &l, int p, uint64_t &key, uint32_t &meta)
{
    const int i = p >> 6, ln = p & 63;
    key = KEY_EMPTY;
    meta = 0;
#pragma unroll
    for (int ii = 0; ii < NI; ++ii)
        if (ii == i) {
            key = rdlane64(l.k[ii], ln);
            meta = rdlane(l.m[ii], ln);
        }
}

template <int NI>
__device__ __forceinline__ void rl_or_meta(RList<NI> &l, int p, uint32_t bits)
{
    const int i = p >> 6, ln = p & 63;
#pragma unroll
    for (int ii = 0; ii < NI; ++ii)
        if (ii == i && __lane_id() == ln) l.m[ii] |= bits;
}

// Inserts the keys mk of the lanes in sbits (distinct, none in the queue) as the worker's
// own unchecked entries, keeping at most L of the len + |sbits| entries; returns the
// update position: the best position one of them takes (L if none stays).  One pass for
// the whole batch: the key of rank r among them lands at f = (queue keys below it) + r;
// the landing positions form a bit mask per slot, and every other destination P takes the
// entry at P - c(P), c(P) the number of landings below P, which lies in P's slot or the
// one before at lane (P - c(P)) mod 64.  stage (LDS, 64 keys) receives the batch by rank.
template <int NI>
__device__ __forceinline__ int rl_insert_batch(RList<NI> &l, int L, int len, uint64_t mk, uint64_t sbits,
                                               uint64_t *stage)
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
        const int f = rl_count_less(l, kj) + r;
        if (lane == 0) stage[r] = kj;
        fmin = min(fmin, f);
        const uint64_t bit = f < L ? 1ull << (f & 63) : 0ull;
#pragma unroll
        for (int i = 0; i < NI; ++i) land[i] |= (f >> 6) == i ? bit : 0ull;
    }
    __builtin_amdgcn_wave_barrier();
    if (fmin >= L) return L;
    const int nlen = min(L, len + __popcll(sbits));
    const int i_first = fmin >> 6;
    int below = 0;
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
        const int addr = ((lane - c) & 63) << 2;
        const bool from_prev = lane < c;
        const uint64_t ck = bpermute64(addr, l.k[i]);
        const uint32_t cm = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)l.m[i]);
        const uint64_t pk = i > 0 ? bpermute64(addr, l.k[i > 0 ? i - 1 : 0]) : KEY_EMPTY;
        const uint32_t pm = i > 0 ? (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)l.m[i > 0 ? i - 1 : 0]) : 0u;
        const uint64_t sk = stage[c & 63];
        const bool keep = 64 * i + lane < nlen;
        l.k[i] = keep ? (lands ? sk : (from_prev ? pk : ck)) : KEY_EMPTY;
        l.m[i] = keep ? (lands ? (META_SIDX | META_MINE) : (from_prev ? pm : cm)) : 0u;
    }
    return fmin;
}

// Records workspace slots written by fresh claims of this wave (prefix over the wave,
// then one reservation) so they can be zeroed at the end of the query.
__device__ __forceinline__ void record_slots(bool rec, uint32_t slot, int32_t *base_counter, uint32_t *slots)
{
    const uint64_t b = __ballot(rec);
    if (!b) return;
    int base = 0;
    if (__lane_id() == 0) base = atomicAdd(base_counter, __popcll(b));
    base = __shfl(base, 0, 64);
    if (rec) slots[base + __popcll(b & lanemask_lt())] = slot;
}

// Moves the LDS visited table into the (zero-filled) workspace table.
__device__ void migrate_table(const unsigned long long *lh, int llog2, unsigned long long *gh, int glog2,
                              uint32_t *gslots, int32_t *nslot, int tid, int nthr)
{
    const uint32_t gm = (1u << glog2) - 1u;
    for (int base = 0; base < (1 << llog2); base += nthr) {
        const int i = base + tid;
        bool rec = false;
        uint32_t s = 0;
        if (i < (1 << llog2)) {
            const unsigned long long h = lh[i];
            if (h != 0ull) {
                s = hash_slot((uint32_t)(h >> 32) - 1u, glog2);
                while (atomicCAS(&gh[s], 0ull, h) != 0ull) s = (s + 1) & gm;
                rec = true;
            }
        }
        record_slots(rec, s, nslot, gslots);
    }
}

// Job `job` runs query order[job] (or job) in workspace region `region`.
// PB: vectors per lane group in each gather pass (see distances)
template <int LPV, int NI, int DT, int PB = 1>
__device__ __forceinline__ void search_body(const KArgs &A, int64_t job, int64_t region)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6, nthr = blockDim.x;
    const int64_t qi = A.order ? A.order[job] : job;
    const int L = A.qL ? A.qL[qi] : A.L, M = A.M, R = A.R;
    const int kq = A.qk ? A.qk[qi] : A.k;

    uint64_t *const skey_base = reinterpret_cast<uint64_t *>(smem + A.o_skey);
    int32_t *const srank = reinterpret_cast<int32_t *>(smem + A.o_srank);
    uint8_t *const schk_base = smem + A.o_schk;
    uint64_t *const pub = reinterpret_cast<uint64_t *>(smem + A.o_pub);   // [PUBCAP] published new keys
    uint64_t *const nkey = reinterpret_cast<uint64_t *>(smem + A.o_newkey) + w * 64;
    int32_t *const claim = reinterpret_cast<int32_t *>(smem + A.o_claim) + w * 64;
    Ctrl *const C = reinterpret_cast<Ctrl *>(smem + A.o_ctrl);
    unsigned long long *const lh = reinterpret_cast<unsigned long long *>(smem + A.o_hash);
    unsigned long long *const gh = A.ghash ? A.ghash + ((size_t)region << (A.glog2 + 1)) : nullptr;
    uint32_t *const gslots = gh ? reinterpret_cast<uint32_t *>(gh + (1ull << A.glog2)) : nullptr;

    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    const int max_sub = A.max_substeps;
    const int llog2 = A.llog2, glog2 = A.glog2;

    if (llog2 > 0)
        for (int i = tid; i < (1 << llog2); i += nthr) lh[i] = 0ull;
    if (tid == 0) {
        C->hcount = 1;
        C->nexp = 0;
        C->mode = llog2 > 0 ? 0 : 1;
        C->flags = 0;
        C->slen = 0;
        C->nslot = 0;
        C->done = 0;
        C->gsteps = C->substeps = C->merges = 0;
        C->epoch = 1;
    }
    // the query, zero padded to 16 LPV floats, shared by the workers
    float *const qs = reinterpret_cast<float *>(smem + A.o_q);
    {
        const float *qrow = A.queries + qi * A.ldq;
        const int nch = A.d >> 2;
        for (int c = tid; c < 4 * LPV; c += nthr)
            reinterpret_cast<float4 *>(qs)[c] =
                c < nch ? *reinterpret_cast<const float4 *>(qrow + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const bool l2 = A.metric == SA_L2;
    const VecSrc V{A.codes, A.scale, A.ldc};
    const int32_t n = (int32_t)A.n;
    // this lane's entry of an adjacency row (R <= 64); lanes past R load entry 0 and drop it
    const int32_t *const adj_lane = A.adj + (lane < R ? lane : 0);
    __syncthreads();

    RList<NI> ls;
    rl_clear(ls);
    int len = 0;
    int m = A.staged ? 1 : M;
    int32_t pv = -1, pu = -1;   // vertex whose adjacency row is prefetched, and this lane's entry of it

    // the start point: its distance, the list holding only it, and the visited set
    if (w == 0) {
        if (lane == 0) claim[0] = A.entry;
        __builtin_amdgcn_wave_barrier();
        if (l2) distances<LPV, true, DT>(V, A.d, qs, claim, 1, nkey);
        else distances<LPV, false, DT>(V, A.d, qs, claim, 1, nkey);
        __builtin_amdgcn_wave_barrier();
        const uint64_t k0 = nkey[0];
        bool fresh = false;
        uint32_t s0 = 0;
        if (lane == 0) {
            s0 = llog2 > 0 ? visit_claim(lh, llog2, (uint32_t)A.entry, 0u, 0u, &fresh)
                           : visit_claim(gh, glog2, (uint32_t)A.entry, 0u, 0u, &fresh);
        }
        if (llog2 == 0) record_slots(lane == 0, s0, &C->nslot, gslots);
        if (lane == 0) {
            ls.k[0] = k0;
            ls.m[0] = META_SIDX | META_MINE;
        }
        len = 1;
        if (m > 1 && lane == 0) {
            skey_base[0] = k0;
            schk_base[0] = 0;
            C->slen = 1;
        }
    }
    __syncthreads();

    // ------------------------------------------------------------ one active worker
    if (m == 1) {
        if (w == 0) {
            int substeps = 0, gsteps = 0, merges = 0, nexp = 0, hcount = 1;
            uint32_t epoch = 1;
            int mode = llog2 > 0 ? 0 : 1;
            bool done = false, stop = false;
            int cur = rl_first_expandable(ls);
            for (;;) {
                // S is this queue; all its unchecked entries belong to the one worker
                if (cur >= len) {
                    done = true;
                    break;
                }
                gsteps++;
                int sub_in_step = 0;
                for (;;) {
                    if (substeps >= max_sub) {
                        if (lane == 0) C->flags |= SA_QFLAG_MAX_STEPS;
                        stop = true;
                        break;
                    }
                    substeps++;
                    sub_in_step++;
                    uint64_t vkey;
                    uint32_t vmeta;
                    rl_get(ls, cur, vkey, vmeta);
                    rl_or_meta(ls, cur, META_CHK);
                    nexp++;
                    const int32_t v = key_id(vkey);
                    int32_t u = pu;
                    if (v != pv) u = adj_lane[(int64_t)v * R];
                    // prefetch the row of the next candidate while this step runs
                    const int nxt = rl_first_expandable(ls);
                    {
                        uint64_t nk = vkey;
                        uint32_t nm;
                        if (nxt < len) rl_get(ls, nxt, nk, nm);
                        pv = key_id(nk);
                        pu = adj_lane[(int64_t)pv * R];
                    }
                    if (lane >= R || u < 0 || u >= n) u = -1;   // padding and malformed entries
                    bool fresh = false;
                    uint32_t slot = NO_SLOT;
                    const uint32_t tag = (epoch << 10) | (uint32_t)lane;
                    if (u >= 0) slot = mode ? visit_claim(gh, glog2, (uint32_t)u, tag, epoch, &fresh)
                                            : visit_claim(lh, llog2, (uint32_t)u, tag, epoch, &fresh);
                    if (mode) record_slots(fresh, slot, &C->nslot, gslots);
                    const uint64_t cm = __ballot(fresh);
                    const int nclaim = __popcll(cm);
                    hcount += nclaim;
                    if (fresh) claim[__popcll(cm & lanemask_lt())] = u;
                    __builtin_amdgcn_wave_barrier();
                    if (l2) distances<LPV, true, DT, false, PB>(V, A.d, qs, claim, nclaim, nkey);
                    else distances<LPV, false, DT, false, PB>(V, A.d, qs, claim, nclaim, nkey);
                    __builtin_amdgcn_wave_barrier();
                    const uint64_t mk = lane < nclaim ? nkey[lane] : KEY_EMPTY;
                    __builtin_amdgcn_wave_barrier();
                    // insert the new entries; the update position is where the best lands
                    uint64_t worst = KEY_EMPTY;
                    if (len == L) {
                        uint32_t wm;
                        rl_get(ls, L - 1, worst, wm);
                    }
                    const uint64_t sbits = __ballot(lane < nclaim && mk < worst);
                    int U = L;
                    if (sbits) {
                        U = rl_insert_batch(ls, L, len, mk, sbits, nkey);
                        len = min(L, len + __popcll(sbits));
                    }
                    cur = rl_first_expandable(ls);
                    epoch++;
                    // keep the visited set below half (LDS) / three quarters (workspace)
                    const int need = hcount + R;
                    if (mode == 0 && need > (1 << llog2) / 2) {
                        if (gh == nullptr || need > (3 << glog2) / 4) {
                            if (lane == 0) C->flags |= SA_QFLAG_CAPACITY;
                            stop = true;
                            break;
                        }
                        migrate_table(lh, llog2, gh, glog2, gslots, &C->nslot, lane, 64);
                        mode = 1;
                        if (lane == 0) C->flags |= SA_QFLAG_SPILLED;
                    } else if (mode == 1 && need > (3 << glog2) / 4) {
                        if (lane == 0) C->flags |= SA_QFLAG_CAPACITY;
                        stop = true;
                        break;
                    }
                    bool merge_now;
                    if (A.sync == SA_SYNC_BSP) merge_now = true;
                    else if (A.sync == SA_SYNC_STATIC) merge_now = A.static_I > 0 && sub_in_step >= A.static_I;
                    else merge_now = (double)U >= (double)L * A.rho;
                    if (cur >= len || merge_now) break;
                }
                merges++;   // S becomes this queue unchanged
                if (stop) break;
                if (M > 1) {
                    m = 2;
                    break;
                }
            }
            if (!done && !stop) {
                // hand S to the workers through LDS
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int p = i * 64 + lane;
                    if (p < len) {
                        skey_base[p] = ls.k[i];
                        schk_base[p] = (ls.m[i] & META_CHK) ? 1 : 0;
                    }
                }
            }
            if (lane == 0) {
                C->done = (done || stop) ? 1 : 0;
                C->slen = len;
                C->hcount = hcount;
                C->nexp = nexp;
                C->mode = mode;
                C->gsteps = gsteps;
                C->substeps = substeps;
                C->merges = merges;
                C->epoch = (int)epoch;
            }
        }
        __syncthreads();
        m = 2;
    }

    // ------------------------------------------------------------ two or more workers
    int sb = 0;
    if (!C->done) {
        int substeps = C->substeps, gsteps = C->gsteps, merges = C->merges;
        uint32_t epoch = (uint32_t)C->epoch;
        pv = -1;
        for (;;) {
            uint64_t *S = skey_base + sb * L;
            uint8_t *Sc = schk_base + sb * L;
            const int slen = C->slen;
            // divide the unchecked entries of S among the m workers: the j-th unchecked
            // entry belongs to worker j mod m; every local queue starts as a copy of S
            int running = 0;
            rl_clear(ls);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int j = i * 64 + lane;
                const bool valid = j < slen;
                const uint8_t chk = valid ? Sc[j] : 1;
                const bool unc = valid && !chk;
                const uint64_t msk = __ballot(unc);
                const int r = running + __popcll(msk & lanemask_lt());
                running += __popcll(msk);
                if (w < m && valid) {
                    ls.k[i] = S[j];
                    ls.m[i] = (uint32_t)j | (chk ? META_CHK : 0u) | ((unc && (r % m) == w) ? META_MINE : 0u);
                }
            }
            for (int j = tid; j < slen; j += nthr) srank[j] = j + m * L;
            if (running == 0) break;   // every local queue is empty of unchecked work
            gsteps++;
            len = (w < m) ? slen : 0;
            int cur = (w < m) ? rl_first_expandable(ls) : NI * 64;
            __syncthreads();

            int sub_in_step = 0;
            bool stop = false;
            for (;;) {
                if (substeps >= max_sub) {
                    if (tid == 0) C->flags |= SA_QFLAG_MAX_STEPS;
                    stop = true;
                    break;
                }
                substeps++;
                sub_in_step++;
                const int mode = C->mode;
                const bool has = (w < m) && (cur < len);
                const uint32_t tag = (epoch << 10) | ((uint32_t)w << 6) | (uint32_t)lane;
                int32_t u = -1;
                uint32_t slot = NO_SLOT;
                bool fresh = false;
                if (has) {
                    // expand the first unchecked candidate of the local queue
                    uint64_t vkey;
                    uint32_t vmeta;
                    rl_get(ls, cur, vkey, vmeta);
                    rl_or_meta(ls, cur, META_CHK);
                    const uint32_t sidx = vmeta & META_SIDX;
                    if (lane == 0) {
                        if (sidx != META_SIDX) Sc[sidx] = 1;
                        atomicAdd(&C->nexp, 1);
                    }
                    const int32_t v = key_id(vkey);
                    u = pu;
                    if (v != pv) u = adj_lane[(int64_t)v * R];
                    const int nxt = rl_first_expandable(ls);
                    {
                        uint64_t nk = vkey;
                        uint32_t nm;
                        if (nxt < len) rl_get(ls, nxt, nk, nm);
                        pv = key_id(nk);
                        pu = adj_lane[(int64_t)pv * R];
                    }
                    if (lane >= R || u < 0 || u >= n) u = -1;
                    if (u >= 0) slot = mode ? visit_claim(gh, glog2, (uint32_t)u, tag, epoch, &fresh)
                                            : visit_claim(lh, llog2, (uint32_t)u, tag, epoch, &fresh);
                }
                __syncthreads();
                int U = L;
                if (has) {
                    bool claimed = false;
                    if (slot != NO_SLOT) {
                        unsigned long long h = mode ? read_slot_global(gh + slot) : lh[slot];
                        claimed = (uint32_t)h == tag;
                    }
                    // the visited count changes only between the two barriers of a local
                    // step, so every wave reads the same value in the decision below
                    const int nfresh = __popcll(__ballot(fresh));
                    if (lane == 0 && nfresh) atomicAdd(&C->hcount, nfresh);
                    if (mode) record_slots(fresh, slot, &C->nslot, gslots);
                    const uint64_t cm = __ballot(claimed);
                    const int nclaim = __popcll(cm);
                    if (claimed) claim[__popcll(cm & lanemask_lt())] = u;
                    __builtin_amdgcn_wave_barrier();
                    if (l2) distances<LPV, true, DT, false, PB>(V, A.d, qs, claim, nclaim, nkey);
                    else distances<LPV, false, DT, false, PB>(V, A.d, qs, claim, nclaim, nkey);
                    __builtin_amdgcn_wave_barrier();
                    const uint64_t mk = lane < nclaim ? nkey[lane] : KEY_EMPTY;
                    __builtin_amdgcn_wave_barrier();
                    uint64_t worst = KEY_EMPTY;
                    if (len == L) {
                        uint32_t wm;
                        rl_get(ls, L - 1, worst, wm);
                    }
                    const uint64_t sbits = __ballot(lane < nclaim && mk < worst);
                    if (sbits) {
                        U = rl_insert_batch(ls, L, len, mk, sbits, nkey);
                        len = min(L, len + __popcll(sbits));
                    }
                    cur = rl_first_expandable(ls);
                }
                if (lane == 0 && w < m) {
                    C->U[w] = U;
                    C->work[w] = cur < len;
                }
                epoch++;
                __syncthreads();
                // lane t reads worker t's flag and update position
                const bool any = __ballot(lane < m && C->work[lane] != 0) != 0;
                int sumU = lane < m ? C->U[lane] : 0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) sumU += __shfl_xor(sumU, off, 64);
                bool merge_now;
                if (A.sync == SA_SYNC_BSP) merge_now = true;
                else if (A.sync == SA_SYNC_STATIC) merge_now = A.static_I > 0 && sub_in_step >= A.static_I;
                else merge_now = (double)sumU / (double)m >= (double)L * A.rho;
                // keep the visited set below half (LDS) / three quarters (workspace) before
                // the next local step, which adds at most m * R entries
                const int need = C->hcount + m * R;
                if (mode == 0 && need > (1 << llog2) / 2) {
                    if (gh == nullptr || need > (3 << glog2) / 4) {
                        if (tid == 0) C->flags |= SA_QFLAG_CAPACITY;
                        stop = true;
                        break;
                    }
                    migrate_table(lh, llog2, gh, glog2, gslots, &C->nslot, tid, nthr);
                    __syncthreads();
                    if (tid == 0) {
                        C->mode = 1;
                        C->flags |= SA_QFLAG_SPILLED;
                    }
                    __syncthreads();
                } else if (mode == 1 && need > (3 << glog2) / 4) {
                    if (tid == 0) C->flags |= SA_QFLAG_CAPACITY;
                    stop = true;
                    break;
                }
                if (!any || merge_now) break;
            }

            // merge: S' = top-L of S and every worker's surviving new entries.  An S
            // entry's rank is its index plus, per worker, the new entries ahead of it in
            // that worker's queue (L if the worker truncated it away); a new entry's rank
            // is its position in its own queue plus the new entries of the other workers
            // below it.  A vertex is claimed by one worker only, so all new entries are
            // distinct keys: every worker publishes its own to LDS (PUBCAP at a time) and
            // each new entry counts the published keys below it, its own included.
            uint64_t *Sn = skey_base + (sb ^ 1) * L;
            uint8_t *Snc = schk_base + (sb ^ 1) * L;
            if (w < m) {
                int own = 0;
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int p = i * 64 + lane;
                    const bool valid = p < len;
                    const uint32_t sidx = valid ? ls.m[i] & META_SIDX : 0u;
                    if (valid && sidx != META_SIDX) atomicAdd(&srank[sidx], p - (int)sidx - L);
                    own += __popcll(__ballot(valid && sidx == META_SIDX));
                }
                if (lane == 0) C->nnew[w] = own;
            }
            __syncthreads();
            int first = 0, total_new = 0;   // this worker's place in the published order
#pragma unroll
            for (int t = 0; t < MAXW; ++t) {
                const int nn = t < m ? C->nnew[t] : 0;
                first += t < w ? nn : 0;
                total_new += nn;
            }
            int rk[NI];   // own position - own new entries below + published keys below
            {
                int nb = 0;
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int p = i * 64 + lane;
                    const bool isN = w < m && p < len && (ls.m[i] & META_SIDX) == META_SIDX;
                    const uint64_t nm = __ballot(isN);
                    rk[i] = p - (nb + __popcll(nm & lanemask_lt()));
                    nb += __popcll(nm);
                }
            }
            for (int c0 = 0; c0 < total_new; c0 += PUBCAP) {
                const int cn = min(PUBCAP, total_new - c0);
                if (w < m) {
                    int nb = first;
#pragma unroll
                    for (int i = 0; i < NI; ++i) {
                        const int p = i * 64 + lane;
                        const bool isN = p < len && (ls.m[i] & META_SIDX) == META_SIDX;
                        const uint64_t nm = __ballot(isN);
                        const int g = nb + __popcll(nm & lanemask_lt()) - c0;
                        if (isN && g >= 0 && g < cn) pub[g] = ls.k[i];
                        nb += __popcll(nm);
                    }
                }
                __syncthreads();
                if (w < m) {
#pragma unroll
                    for (int i = 0; i < NI; ++i) {
                        const int p = i * 64 + lane;
                        const bool isN = p < len && (ls.m[i] & META_SIDX) == META_SIDX;
                        if (__ballot(isN)) {
                            const uint64_t key = ls.k[i];
                            int below = 0;
                            for (int j = 0; j < cn; ++j) below += pub[j] < key ? 1 : 0;
                            rk[i] += below;
                        }
                    }
                }
                __syncthreads();
            }
            if (w < m) {
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int p = i * 64 + lane;
                    const bool isN = p < len && (ls.m[i] & META_SIDX) == META_SIDX;
                    if (isN && rk[i] < L) {
                        Sn[rk[i]] = ls.k[i];
                        Snc[rk[i]] = (ls.m[i] & META_CHK) ? 1 : 0;
                    }
                }
            }
            for (int j = tid; j < slen; j += nthr) {
                const int r = srank[j];
                if (r < L) {
                    Sn[r] = S[j];
                    Snc[r] = Sc[j];
                }
            }
            __syncthreads();
            if (tid == 0) C->slen = min(L, slen + total_new);
            sb ^= 1;
            merges++;
            if (A.staged && m < M) m = min(2 * m, M);
            __syncthreads();
            if (stop) break;   // a step limit or a full visited table ends the search after this merge
        }
        if (tid == 0) {
            C->gsteps = gsteps;
            C->substeps = substeps;
            C->merges = merges;
        }
    }

    __syncthreads();
    {
        const bool from_regs = C->done != 0;   // the search ended in wavefront 0's queue
        const int slen = C->slen;
        if (A.rerank != 0) {
            // hand the first nr entries of the final list to the re-rank kernel
            const int nr = A.rerank < 0 ? slen : min(A.rerank, slen);
            int32_t *const list = rerank_list(reinterpret_cast<uint32_t *>(gslots), glog2);
            if (from_regs) {
                if (w == 0) {
#pragma unroll
                    for (int i = 0; i < NI; ++i)
                        if (64 * i + lane < nr) list[1 + 64 * i + lane] = key_id(ls.k[i]);
                }
            } else {
                const uint64_t *S = skey_base + sb * L;
                for (int i = tid; i < nr; i += nthr) list[1 + i] = key_id(S[i]);
            }
            if (tid == 0) list[0] = nr;
        } else if (from_regs) {
            if (w == 0) {
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int p = i * 64 + lane;
                    if (p < kq) {
                        const bool ok = p < slen;
                        A.ids[qi * A.ldo + p] = ok ? key_id(ls.k[i]) : -1;
                        A.dists[qi * A.ldo + p] = ok ? key_dist(ls.k[i]) : __builtin_inff();
                    }
                }
            }
        } else {
            const uint64_t *S = skey_base + sb * L;
            for (int i = tid; i < kq; i += nthr) {
                if (i < slen) {
                    A.ids[qi * A.ldo + i] = key_id(S[i]);
                    A.dists[qi * A.ldo + i] = key_dist(S[i]);
                } else {
                    A.ids[qi * A.ldo + i] = -1;
                    A.dists[qi * A.ldo + i] = __builtin_inff();
                }
            }
        }
        // leave the workspace table zero-filled for the next launch
        const int ns = C->nslot;
        for (int i = tid; i < ns; i += nthr) {
            const uint32_t sl = gslots[i];
            gh[sl] = 0ull;
            gslots[i] = 0u;
        }
        if (tid == 0 && A.stats) {
            sa_query_stats st;
            st.global_steps = C->gsteps;
            st.substeps = C->substeps;
            st.expansions = C->nexp;
            st.dist_comps = C->hcount;
            st.merges = C->merges;
            st.flags = C->flags;
            st.t_start = t_start;
            st.t_end = __builtin_amdgcn_s_memrealtime();
            A.stats[qi] = st;
        }
    }
}

}  // namespace search_detail

int launch_rerank(const float *vec32, int64_t ld32, const float *queries, int64_t ldq, int64_t nq, int32_t d,
                  int32_t metric, int32_t k, int32_t L, void *ws, int64_t stride, int64_t list_off, int32_t *ids,
                  float *dists, const int32_t *order, const int32_t *qk, int64_t ldo, hipStream_t s);
int launch_search_single_f32(const search_detail::KArgs &A, int64_t nq, hipStream_t s);
int launch_search_single_bf16(const search_detail::KArgs &A, int64_t nq, hipStream_t s);
int launch_search_single_fp8(const search_detail::KArgs &A, int64_t nq, hipStream_t s);
int launch_search_multi_f32(const search_detail::KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s);
int launch_search_multi_bf16(const search_detail::KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s);
int launch_search_multi_fp8(const search_detail::KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s);

}  // namespace sa
