// Intra-query parallel graph search (Speed-ANN, arXiv 2201.13007, Algorithm 3 with
// CheckMetrics of Algorithm 2; Algorithm 1 when there is one worker), for gfx950.
//
// One workgroup runs one query; worker t of Algorithm 3 is wavefront t.  Per query the
// workgroup keeps in LDS:
//   S       the global queue, capacity L, as sorted 64-bit keys (distance bits, id) plus a
//           checked byte per entry (double buffered for the merge);
//   LS[t]   worker t's local queue, capacity L: keys plus a 32-bit tag holding the index
//           of the S entry it was copied from (0xFFFF for candidates the worker inserted
//           itself), MINE (the worker may expand it) and CHECKED bits;
//   visited an open-addressing hash of 64-bit entries (id << 32 | claim tag).  It moves to
//           a per-query region of the caller's workspace when it fills past one half.
//
// The workers advance in lockstep: in every local step each worker with work expands
// its first unchecked candidate, all workers place claims for the neighbours they find
// (two-phase, so that a vertex reached by several workers in one step goes to the
// lowest (worker, adjacency slot) — the order in which a sequential emulation would
// visit them), each worker computes the distances of the vertices it claimed, sorts them
// and merges them into its own queue, and after a barrier every thread evaluates the
// same merge decision.  The merge of the local queues into S ranks every surviving
// entry by counting smaller keys across the queues, so it needs no sort.
#include "sa_internal.h"

namespace sa {
namespace {

constexpr uint32_t META_SIDX = 0xFFFFu;
constexpr uint32_t META_MINE = 1u << 16;
constexpr uint32_t META_CHK = 1u << 17;
constexpr int MAXW = 16;
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;

struct Ctrl {
    int32_t lslen[MAXW];
    int32_t U[MAXW];
    int32_t work[MAXW];
    int32_t nnew[MAXW];
    int32_t slen;
    int32_t hcount;
    int32_t nexp;
    int32_t mode;   // 0: visited set in LDS, 1: in the workspace
    int32_t flags;
    int32_t pad[3];
};

struct KArgs {
    const float *vec;
    int64_t ld;
    const int32_t *adj;
    const float *queries;
    int64_t ldq;
    int32_t *ids;
    float *dists;
    sa_query_stats *stats;
    unsigned long long *ghash;
    int64_t n;
    int32_t d, metric, R, entry, k, L, M, sync, static_I, staged, max_substeps;
    double rho;
    int32_t glog2, llog2;
    uint32_t o_skey, o_srank, o_schk, o_lskey, o_lsmeta, o_newkey, o_claim, o_ctrl, o_hash;
};

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t hash_slot(uint32_t id, int log2cap)
{
    return (id * 2654435761u) >> (32 - log2cap);
}

// Phase one of a claim: find or insert u, leaving the smallest tag of this local step
// in its slot.  Returns the slot, or NO_SLOT if the table is full; *fresh tells whether
// this call inserted u.
template <bool GLOBAL>
__device__ uint32_t visit_claim(unsigned long long *H, int log2cap, uint32_t u, uint32_t tag, uint32_t epoch,
                                bool *fresh)
{
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t s = hash_slot(u, log2cap);
    const unsigned long long want = ((unsigned long long)u << 32) | tag;
    *fresh = false;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        unsigned long long old = atomicCAS(&H[s], (unsigned long long)KEY_EMPTY, want);
        if (old == KEY_EMPTY) {
            *fresh = true;
            return s;
        }
        if ((uint32_t)(old >> 32) == u) {
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

__device__ __forceinline__ uint64_t bitonic_sort64(uint64_t key)
{
    const int lane = __lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t other = (uint64_t)__shfl_xor((unsigned long long)key, j, 64);
            bool up = (lane & k) == 0;
            bool low = (lane & j) == 0;
            uint64_t mn = other < key ? other : key;
            uint64_t mx = other < key ? key : other;
            key = (low == up) ? mn : mx;
        }
    }
    return key;
}

// first index of the local queue holding an entry the worker may expand (MINE and not
// CHECKED), or len if none
__device__ __forceinline__ int first_expandable(const uint32_t *meta, int len)
{
    for (int base = 0; base < len; base += 64) {
        int p = base + __lane_id();
        bool ok = p < len && (meta[p] & (META_MINE | META_CHK)) == META_MINE;
        uint64_t m = __ballot(ok);
        if (m) return base + __builtin_ctzll(m);
    }
    return len;
}

// Distances from the query (q chunks in registers) to the vectors listed in ids[0..n),
// written as keys to out[0..n).  LPV lanes share one vector (float4 chunks c = g,
// g + LPV, ...); every lane accumulates its chunks in double precision, the group sums
// its lanes with a butterfly and the group's first lane rounds the sum once to float.
template <int LPV, int CPL>
__device__ void wave_distances(const KArgs &A, const float4 (&q)[CPL], const int32_t *ids, int n, uint64_t *out)
{
    constexpr int VPW = 64 / LPV;
    constexpr int PB = CPL >= 4 ? 1 : 4 / CPL;
    const int lane = __lane_id();
    const int grp = lane / LPV, g = lane % LPV;
    const int nch = A.d >> 2;
    const int npass = (n + VPW - 1) / VPW;
    for (int p0 = 0; p0 < npass; p0 += PB) {
        float4 xv[PB][CPL];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
            int idx = (p0 + pp) * VPW + grp;
            if (idx < n) {
                const float *row = A.vec + (int64_t)ids[idx] * A.ld;
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    int c = g + LPV * i;
                    if (c < nch) xv[pp][i] = *reinterpret_cast<const float4 *>(row + 4 * c);
                }
            }
        }
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
            int idx = (p0 + pp) * VPW + grp;
            double acc = 0.0;
            if (idx < n) {
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    int c = g + LPV * i;
                    if (c < nch) {
                        const float4 a = q[i], b = xv[pp][i];
                        if (A.metric == SA_L2) {
                            double t0 = (double)a.x - (double)b.x, t1 = (double)a.y - (double)b.y;
                            double t2 = (double)a.z - (double)b.z, t3 = (double)a.w - (double)b.w;
                            acc += t0 * t0; acc += t1 * t1; acc += t2 * t2; acc += t3 * t3;
                        } else {
                            acc += (double)a.x * (double)b.x; acc += (double)a.y * (double)b.y;
                            acc += (double)a.z * (double)b.z; acc += (double)a.w * (double)b.w;
                        }
                    }
                }
            }
#pragma unroll
            for (int off = LPV / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (g == 0 && idx < n) {
                float dist = A.metric == SA_L2 ? (float)acc : (float)(-acc);
                out[idx] = make_key(dist, ids[idx]);
            }
        }
    }
}

// Merge nnew sorted new keys (lane i holds the i-th, sorted copy in nk[]) into the
// worker's sorted queue (len entries), truncating to L.  Returns the update position:
// the 0-based position of the best new entry after truncation, or L.
__device__ int list_insert(uint64_t *lkey, uint32_t *lmeta, int len, int L, const uint64_t *nk, int nnew,
                           uint64_t mykey)
{
    const int lane = __lane_id();
    int mypos = L;
    if (lane < nnew) mypos = lane + lower_bound(lkey, len, mykey);
    int upd = __shfl(mypos, 0, 64);
    // move the old entries, highest chunk first: an entry only moves up, so every chunk
    // is read completely before anything lands on it
    int nchunk = (len + 63) >> 6;
    for (int c = nchunk - 1; c >= 0; --c) {
        int p = c * 64 + lane;
        uint64_t k = 0;
        uint32_t m = 0;
        int np = L;
        if (p < len) {
            k = lkey[p];
            m = lmeta[p];
            np = p + lower_bound(nk, nnew, k);
        }
        __builtin_amdgcn_wave_barrier();
        if (p < len && np < L && np != p) {
            lkey[np] = k;
            lmeta[np] = m;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < nnew && mypos < L) {
        lkey[mypos] = mykey;
        lmeta[mypos] = META_SIDX | META_MINE;
    }
    __builtin_amdgcn_wave_barrier();
    return (nnew > 0 && upd < L) ? upd : L;
}

template <int LPV, int CPL>
__global__ void __launch_bounds__(1024) search_kernel(KArgs A)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6, nthr = blockDim.x;
    const int64_t qi = blockIdx.x;
    const int L = A.L, M = A.M, R = A.R;

    uint64_t *const skey_base = reinterpret_cast<uint64_t *>(smem + A.o_skey);
    int32_t *const srank = reinterpret_cast<int32_t *>(smem + A.o_srank);
    uint8_t *const schk_base = smem + A.o_schk;
    uint64_t *const lskey_all = reinterpret_cast<uint64_t *>(smem + A.o_lskey);
    uint64_t *const lskey = lskey_all + (size_t)w * L;
    uint32_t *const lsmeta = reinterpret_cast<uint32_t *>(smem + A.o_lsmeta) + (size_t)w * L;
    uint64_t *const nkey = reinterpret_cast<uint64_t *>(smem + A.o_newkey) + w * 64;
    int32_t *const claim = reinterpret_cast<int32_t *>(smem + A.o_claim) + w * 64;
    Ctrl *const C = reinterpret_cast<Ctrl *>(smem + A.o_ctrl);
    unsigned long long *const lh = reinterpret_cast<unsigned long long *>(smem + A.o_hash);
    unsigned long long *const gh = A.ghash ? A.ghash + ((size_t)qi << A.glog2) : nullptr;

    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();

    for (int i = tid; i < (1 << A.llog2); i += nthr) lh[i] = KEY_EMPTY;
    if (tid == 0) {
        C->hcount = 0;
        C->nexp = 0;
        C->mode = 0;
        C->flags = 0;
        C->slen = 0;
    }
    float4 q[CPL];
    {
        const float *qrow = A.queries + qi * A.ldq;
        const int g = lane % LPV, nch = A.d >> 2;
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            int c = g + LPV * i;
            q[i] = c < nch ? *reinterpret_cast<const float4 *>(qrow + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    __syncthreads();
    if (w == 0) {
        // compute dist(P, Q), add P to S and mark it visited
        if (lane == 0) claim[0] = A.entry;
        __builtin_amdgcn_wave_barrier();
        wave_distances<LPV, CPL>(A, q, claim, 1, nkey);
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            bool fresh;
            visit_claim<false>(lh, A.llog2, (uint32_t)A.entry, 0u, 0u, &fresh);
            C->hcount = 1;
            skey_base[0] = nkey[0];
            schk_base[0] = 0;
            C->slen = 1;
        }
    }
    __syncthreads();

    int m = A.staged ? 1 : M;
    uint32_t epoch = 1;
    int substeps = 0, gsteps = 0, merges = 0;
    int sb = 0;
    const int max_sub = A.max_substeps;
    for (;;) {
        uint64_t *S = skey_base + sb * L;
        uint8_t *Sc = schk_base + sb * L;
        const int slen = C->slen;
        // divide the unchecked entries of S among the m workers: the j-th unchecked
        // entry belongs to worker j mod m; every local queue starts as a copy of S
        int running = 0;
        for (int base = 0; base < slen; base += 64) {
            int j = base + lane;
            bool valid = j < slen;
            uint8_t chk = valid ? Sc[j] : 1;
            bool unc = valid && !chk;
            uint64_t msk = __ballot(unc);
            int r = running + __popcll(msk & lanemask_lt());
            running += __popcll(msk);
            if (w < m && valid) {
                uint32_t meta = (uint32_t)j | (chk ? META_CHK : 0u) | ((unc && (r % m) == w) ? META_MINE : 0u);
                lsmeta[j] = meta;
                lskey[j] = S[j];
            }
        }
        for (int j = tid; j < slen; j += nthr) srank[j] = j + m * L;
        if (running == 0) break;   // every local queue is empty of unchecked work
        gsteps++;
        int mylen = slen;
        int cur = (w < m) ? first_expandable(lsmeta, mylen) : L;
        if (lane == 0 && w < m) C->lslen[w] = mylen;
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
            const bool has = (w < m) && (cur < mylen);
            const uint32_t tag = (epoch << 10) | ((uint32_t)w << 6) | (uint32_t)lane;
            int32_t u = -1;
            uint32_t slot = NO_SLOT;
            bool fresh = false;
            if (has) {
                // expand the first unchecked candidate of the local queue
                const uint32_t meta = lsmeta[cur];
                const int32_t v = key_id(lskey[cur]);
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    lsmeta[cur] = meta | META_CHK;
                    const uint32_t sidx = meta & META_SIDX;
                    if (sidx != META_SIDX) Sc[sidx] = 1;
                    atomicAdd(&C->nexp, 1);
                }
                if (lane < R) u = A.adj[(int64_t)v * R + lane];
                if (u >= A.n) u = -1;   // malformed row entries are ignored like padding
                if (u >= 0) {
                    slot = mode ? visit_claim<true>(gh, A.glog2, (uint32_t)u, tag, epoch, &fresh)
                                : visit_claim<false>(lh, A.llog2, (uint32_t)u, tag, epoch, &fresh);
                }
            }
            __syncthreads();
            int U = L;
            if (has) {
                bool claimed = false;
                if (slot != NO_SLOT) {
                    unsigned long long h = mode ? read_slot_global(gh + slot) : lh[slot];
                    claimed = (uint32_t)h == tag;
                }
                const uint64_t cm = __ballot(claimed);
                const int nclaim = __popcll(cm);
                // the visited count changes only between the two barriers of a local step,
                // so every wave reads the same value in the decision below
                const int nfresh = __popcll(__ballot(fresh));
                if (lane == 0 && nfresh) atomicAdd(&C->hcount, nfresh);
                if (claimed) claim[__popcll(cm & lanemask_lt())] = u;
                __builtin_amdgcn_wave_barrier();
                wave_distances<LPV, CPL>(A, q, claim, nclaim, nkey);
                __builtin_amdgcn_wave_barrier();
                uint64_t mk = lane < nclaim ? nkey[lane] : KEY_EMPTY;
                mk = bitonic_sort64(mk);
                __builtin_amdgcn_wave_barrier();
                nkey[lane] = mk;
                __builtin_amdgcn_wave_barrier();
                U = list_insert(lskey, lsmeta, mylen, L, nkey, nclaim, mk);
                mylen = min(L, mylen + nclaim);
                cur = first_expandable(lsmeta, mylen);
            }
            if (lane == 0 && w < m) {
                C->U[w] = U;
                C->work[w] = cur < mylen;
                C->lslen[w] = mylen;
            }
            epoch++;
            __syncthreads();
            bool any = false;
            int64_t sumU = 0;
            for (int t = 0; t < m; ++t) {
                any = any || C->work[t] != 0;
                sumU += C->U[t];
            }
            bool merge_now;
            if (A.sync == SA_SYNC_BSP) merge_now = true;
            else if (A.sync == SA_SYNC_STATIC) merge_now = A.static_I > 0 && sub_in_step >= A.static_I;
            else merge_now = (double)sumU / (double)m >= (double)L * A.rho;
            // keep the visited set at most half (LDS) / three quarters (workspace) full
            // before the next local step, which adds at most m * R entries
            const int need = C->hcount + m * R;
            if (mode == 0 && need > (1 << A.llog2) / 2) {
                if (gh == nullptr || need > (3 << A.glog2) / 4) {
                    if (tid == 0) C->flags |= SA_QFLAG_CAPACITY;
                    stop = true;
                    break;
                }
                for (int i = tid; i < (1 << A.glog2); i += nthr) gh[i] = KEY_EMPTY;
                __syncthreads();
                for (int i = tid; i < (1 << A.llog2); i += nthr) {
                    unsigned long long h = lh[i];
                    if (h != KEY_EMPTY) {
                        const uint32_t gm = (1u << A.glog2) - 1u;
                        uint32_t s = hash_slot((uint32_t)(h >> 32), A.glog2);
                        while (atomicCAS(&gh[s], (unsigned long long)KEY_EMPTY, h) != KEY_EMPTY) s = (s + 1) & gm;
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    C->mode = 1;
                    C->flags |= SA_QFLAG_SPILLED;
                }
                __syncthreads();
            } else if (mode == 1 && need > (3 << A.glog2) / 4) {
                if (tid == 0) C->flags |= SA_QFLAG_CAPACITY;
                stop = true;
                break;
            }
            if (!any || merge_now) break;
        }
        if (stop) break;

        // merge: S' = top-L of S and every worker's surviving new entries.  An S entry's
        // rank is its index plus, per worker, the new entries ahead of it in that
        // worker's queue (L if the worker truncated it away); a new entry's rank is its
        // position in its own queue plus the new entries of the other workers below it.
        uint64_t *Sn = skey_base + (sb ^ 1) * L;
        uint8_t *Snc = schk_base + (sb ^ 1) * L;
        if (w < m) {
            int nbefore = 0;
            for (int base = 0; base < mylen; base += 64) {
                const int p = base + lane;
                const bool valid = p < mylen;
                const uint32_t meta = valid ? lsmeta[p] : 0u;
                const uint32_t sidx = meta & META_SIDX;
                const bool isS = valid && sidx != META_SIDX;
                const bool isN = valid && sidx == META_SIDX;
                if (isS) atomicAdd(&srank[sidx], p - (int)sidx - L);
                const uint64_t nm = __ballot(isN);
                if (isN) {
                    const int nidx = nbefore + __popcll(nm & lanemask_lt());
                    const uint64_t key = lskey[p];
                    const int cS = p - nidx;
                    int rank = p;
                    for (int t = 0; t < m && rank < L; ++t) {
                        if (t == w) continue;
                        rank += lower_bound(lskey_all + (size_t)t * L, C->lslen[t], key) - cS;
                    }
                    if (rank < L) {
                        Sn[rank] = key;
                        Snc[rank] = (meta & META_CHK) ? 1 : 0;
                    }
                }
                nbefore += __popcll(nm);
            }
            if (lane == 0) C->nnew[w] = nbefore;
        }
        __syncthreads();
        for (int j = tid; j < slen; j += nthr) {
            const int r = srank[j];
            if (r < L) {
                Sn[r] = S[j];
                Snc[r] = Sc[j];
            }
        }
        int total = slen;
        for (int t = 0; t < m; ++t) total += C->nnew[t];
        __syncthreads();
        if (tid == 0) C->slen = min(L, total);
        sb ^= 1;
        merges++;
        if (A.staged && m < M) m = min(2 * m, M);
        __syncthreads();
    }

    __syncthreads();
    {
        const uint64_t *S = skey_base + sb * L;
        const int slen = C->slen;
        for (int i = tid; i < A.k; i += nthr) {
            if (i < slen) {
                A.ids[qi * A.k + i] = key_id(S[i]);
                A.dists[qi * A.k + i] = key_dist(S[i]);
            } else {
                A.ids[qi * A.k + i] = -1;
                A.dists[qi * A.k + i] = __builtin_inff();
            }
        }
        if (tid == 0 && A.stats) {
            sa_query_stats st;
            st.global_steps = gsteps;
            st.substeps = substeps;
            st.expansions = C->nexp;
            st.dist_comps = C->hcount;
            st.merges = merges;
            st.flags = C->flags;
            st.t_start = t_start;
            st.t_end = __builtin_amdgcn_s_memrealtime();
            A.stats[qi] = st;
        }
    }
}

struct Layout {
    uint32_t o_skey, o_srank, o_schk, o_lskey, o_lsmeta, o_newkey, o_claim, o_ctrl, o_hash, total;
};

uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

Layout make_layout(int L, int M, int llog2)
{
    Layout Y;
    uint32_t o = 0;
    Y.o_skey = o; o += 2u * 8u * L;
    Y.o_srank = o; o += 4u * L;
    Y.o_schk = o; o = align_up(o + 2u * L, 16);
    Y.o_lskey = o; o += 8u * M * L;
    Y.o_lsmeta = o; o += 4u * M * L;
    o = align_up(o, 16);
    Y.o_newkey = o; o += 8u * 64u * M;
    Y.o_claim = o; o += 4u * 64u * M;
    Y.o_ctrl = o; o += align_up(sizeof(Ctrl), 16);
    Y.o_hash = o; o += 8u << llog2;
    Y.total = o;
    return Y;
}

int ilog2_exact(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

void resolve_params(const sa_search_params &in, int L, int M, int R, int &llog2, int &glog2, int &max_sub)
{
    max_sub = in.max_substeps > 0 ? in.max_substeps : (1 << 22);
    if (in.lds_hash_slots > 0) llog2 = ilog2_exact(in.lds_hash_slots);
    else llog2 = M <= 2 ? 11 : 12;
    if (in.ws_hash_slots > 0) glog2 = ilog2_exact(in.ws_hash_slots);
    else {
        // the visited set holds at most 1 + E * R vertices after E expansions, and E stays
        // close to L; 64 L slots keep three quarters of the table above 1.5 L * 32
        int64_t want = 64ll * L;
        if (want < 4096) want = 4096;
        glog2 = ilog2_exact(want);
    }
    (void)R;
}

template <int LPV, int CPL>
hipError_t launch_t(const KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s)
{
    auto k = search_kernel<LPV, CPL>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)nq), dim3(64 * M), lds, s, A);
    return hipGetLastError();
}

}  // namespace

size_t search_workspace_bytes(int64_t nq, int32_t L, int32_t M, const sa_search_params &p, int32_t R)
{
    int llog2, glog2, max_sub;
    resolve_params(p, L, M, R, llog2, glog2, max_sub);
    return (size_t)nq * ((size_t)8 << glog2);
}

int launch_search(const SearchLaunch &a, hipStream_t stream)
{
    int llog2, glog2, max_sub;
    resolve_params(a.p, a.L, a.M, a.R, llog2, glog2, max_sub);
    if (llog2 < 6 || llog2 > 14) return set_error(SA_EINVAL, "lds_hash_slots must be a power of two in [64, 16384]");
    if (glog2 < 6 || glog2 > 26) return set_error(SA_EINVAL, "ws_hash_slots must be a power of two in [64, 2^26]");
    if ((int64_t(1) << llog2) / 2 < (int64_t)a.M * a.R + 1)
        return set_error(SA_EINVAL, "lds_hash_slots too small for M * R new vertices per local step");
    size_t need = (size_t)a.nq * ((size_t)8 << glog2);
    if (a.ws_bytes < need)
        return set_error(SA_ECAPACITY, "workspace of %zu bytes is smaller than the %zu bytes needed", a.ws_bytes, need);
    if (a.workspace == nullptr && need > 0) return set_error(SA_EINVAL, "workspace is NULL");
    if (((uintptr_t)a.workspace & 255u) != 0) return set_error(SA_EINVAL, "workspace must be 256-byte aligned");
    Layout Y = make_layout(a.L, a.M, llog2);
    if (Y.total > 160u * 1024u)
        return set_error(SA_ECAPACITY, "L=%d, M=%d need %u bytes of LDS per query (limit 163840); lower L, M or "
                         "lds_hash_slots", a.L, a.M, Y.total);
    KArgs A;
    A.vec = a.vec; A.ld = a.ld; A.adj = a.adj; A.queries = a.queries; A.ldq = a.ldq;
    A.ids = a.ids; A.dists = a.dists; A.stats = a.stats;
    A.ghash = reinterpret_cast<unsigned long long *>(a.workspace);
    A.n = a.n;
    A.d = a.d; A.metric = a.metric; A.R = a.R; A.entry = a.entry; A.k = a.k; A.L = a.L; A.M = a.M;
    A.sync = a.p.sync; A.static_I = a.p.static_I; A.staged = a.p.staged ? 1 : 0; A.max_substeps = max_sub;
    A.rho = a.p.rho; A.glog2 = glog2; A.llog2 = llog2;
    A.o_skey = Y.o_skey; A.o_srank = Y.o_srank; A.o_schk = Y.o_schk; A.o_lskey = Y.o_lskey;
    A.o_lsmeta = Y.o_lsmeta; A.o_newkey = Y.o_newkey; A.o_claim = Y.o_claim; A.o_ctrl = Y.o_ctrl;
    A.o_hash = Y.o_hash;
    if (a.nq == 0) return SA_OK;
    const int nch = a.d / 4;
    hipError_t e;
    if (nch <= 8) e = launch_t<8, 1>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 16) e = launch_t<16, 1>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 32) e = launch_t<32, 1>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 64) e = launch_t<64, 1>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 128) e = launch_t<64, 2>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 256) e = launch_t<64, 4>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 512) e = launch_t<64, 8>(A, a.nq, a.M, Y.total, stream);
    else if (nch <= 1024) e = launch_t<64, 16>(A, a.nq, a.M, Y.total, stream);
    else return set_error(SA_EUNSUPPORTED, "d=%d exceeds 4096", a.d);
    if (e != hipSuccess) return hip_fail(e, "search kernel launch");
    return SA_OK;
}

}  // namespace sa
