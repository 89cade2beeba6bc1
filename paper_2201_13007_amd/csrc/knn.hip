// Exact k nearest neighbours by linear scan (Sec. 2.1: the naive solution that checks
// every point).  Used for ground truth and for the candidate lists of graph
// construction.
//
// A workgroup owns TQ = 32 queries and streams all base rows in tiles of TX = 64.  The
// d dimensions go through LDS in chunks of 32; each thread accumulates 2 x 4
// (query, base) pairs in double precision, one dimension after the other in index order
// with separately rounded multiply and add, and rounds each sum once to float — the
// same arithmetic as a plain sequential loop, so the keys are reproducible bit for bit.
// Each query keeps its current top-k (sorted keys in LDS) and a threshold; tile
// results below the threshold go to a per-query buffer that is sorted and merged into
// the top-k whenever it could overflow.
#include "sa_internal.h"

namespace sa {
namespace {

constexpr int TQ = 32;
constexpr int TX = 64;
constexpr int DC = 32;
constexpr int NT = 256;
constexpr int BUF = 128;   // per-query candidate buffer; flushed when > BUF - TX

__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int n, uint64_t key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long shx(unsigned long long v, int j) { return __shfl_xor(v, j, 64); }

// sort 128 keys held two per lane (element lane and lane + 64), ascending
__device__ void sort128(unsigned long long &lo, unsigned long long &hi)
{
    const int lane = __lane_id();
    for (int k = 2; k <= 128; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j == 64) {
                unsigned long long mn = lo < hi ? lo : hi, mx = lo < hi ? hi : lo;
                lo = mn;
                hi = mx;
            } else {
                unsigned long long olo = shx(lo, j), ohi = shx(hi, j);
                {
                    const int e = lane;
                    bool up = (e & k) == 0, low = (e & j) == 0;
                    unsigned long long mn = olo < lo ? olo : lo, mx = olo < lo ? lo : olo;
                    lo = (low == up) ? mn : mx;
                }
                {
                    const int e = lane + 64;
                    bool up = (e & k) == 0, low = (e & j) == 0;
                    unsigned long long mn = ohi < hi ? ohi : hi, mx = ohi < hi ? hi : ohi;
                    hi = (low == up) ? mn : mx;
                }
            }
        }
    }
}

// merge the cnt keys of buf (unsorted) into the sorted list top[0..*len), keeping k
__device__ void flush_query(uint64_t *top, int *len, uint64_t *buf, int cnt, int k)
{
    const int lane = __lane_id();
    unsigned long long lo = lane < cnt ? buf[lane] : KEY_EMPTY;
    unsigned long long hi = lane + 64 < cnt ? buf[lane + 64] : KEY_EMPTY;
    sort128(lo, hi);
    __builtin_amdgcn_wave_barrier();
    buf[lane] = lo;
    buf[lane + 64] = hi;
    __builtin_amdgcn_wave_barrier();
    const int n = *len;
    // positions of the new keys in the merged order
    int plo = k, phi = k;
    if (lane < cnt) plo = lane + lower_bound_u64(top, n, lo);
    if (lane + 64 < cnt) phi = lane + 64 + lower_bound_u64(top, n, hi);
    // move old entries up, highest chunk first (see the search kernel's queue insert)
    for (int c = (n + 63) / 64 - 1; c >= 0; --c) {
        int p = c * 64 + lane;
        uint64_t key = 0;
        int np = k;
        if (p < n) {
            key = top[p];
            np = p + lower_bound_u64(buf, cnt, key);
        }
        __builtin_amdgcn_wave_barrier();
        if (p < n && np < k && np != p) top[np] = key;
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < cnt && plo < k) top[plo] = lo;
    if (lane + 64 < cnt && phi < k) top[phi] = hi;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) *len = min(k, n + cnt);
}

struct KnnArgs {
    const float *base;
    int64_t n, ld;
    const float *queries;
    int64_t nq, ldq;
    int32_t d, k, kpad, metric, exclude_self;
    int32_t *ids;
    float *dists;
};

__global__ void __launch_bounds__(NT) knn_kernel(KnnArgs A)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *Qs = reinterpret_cast<float *>(smem);                      // [TQ][DC+1]
    float *Xs = Qs + TQ * (DC + 1);                                    // [TX][DC+1]
    uint64_t *top = reinterpret_cast<uint64_t *>(Xs + TX * (DC + 1)); // [TQ][kpad]
    uint64_t *buf = top + (size_t)TQ * A.kpad;                         // [TQ][BUF]
    int *toplen = reinterpret_cast<int *>(buf + (size_t)TQ * BUF);     // [TQ]
    int *cnt = toplen + TQ;                                            // [TQ]
    uint64_t *thr = reinterpret_cast<uint64_t *>(cnt + TQ + 2);        // [TQ] (8-aligned below)
    int *need = cnt + TQ;                                              // [1]

    const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
    const int tq = tid >> 4, tx = tid & 15;   // queries tq, tq + 16; bases tx + 16 b
    const int64_t q0 = (int64_t)blockIdx.x * TQ;

    for (int i = tid; i < TQ; i += NT) {
        toplen[i] = 0;
        cnt[i] = 0;
        thr[i] = KEY_EMPTY;
    }
    if (tid == 0) *need = 0;
    __syncthreads();

    for (int64_t xb = 0; xb < A.n; xb += TX) {
        double acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int dc = 0; dc < A.d; dc += DC) {
            const int dlen = min(DC, A.d - dc);
            for (int i = tid; i < TQ * DC; i += NT) {
                int r = i / DC, c = i % DC;
                int64_t qr = q0 + r;
                Qs[r * (DC + 1) + c] = (qr < A.nq && c < dlen) ? A.queries[qr * A.ldq + dc + c] : 0.f;
            }
            for (int i = tid; i < TX * DC; i += NT) {
                int r = i / DC, c = i % DC;
                int64_t xr = xb + r;
                Xs[r * (DC + 1) + c] = (xr < A.n && c < dlen) ? A.base[xr * A.ld + dc + c] : 0.f;
            }
            __syncthreads();
            for (int c = 0; c < dlen; ++c) {
                double qv[2], xv[4];
#pragma unroll
                for (int a = 0; a < 2; ++a) qv[a] = (double)Qs[(tq + 16 * a) * (DC + 1) + c];
#pragma unroll
                for (int b = 0; b < 4; ++b) xv[b] = (double)Xs[(tx + 16 * b) * (DC + 1) + c];
                if (A.metric == SA_L2) {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            double t = qv[a] - xv[b];
                            acc[a][b] += t * t;
                        }
                } else {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] += qv[a] * xv[b];
                }
            }
            __syncthreads();
        }
        // filter against the per-query thresholds
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int qr = tq + 16 * a;
            const int64_t qg = q0 + qr;
            if (qg >= A.nq) continue;
            const uint64_t t = thr[qr];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t xg = xb + tx + 16 * b;
                if (xg >= A.n || (A.exclude_self && xg == qg)) continue;
                const float dist = A.metric == SA_L2 ? (float)acc[a][b] : (float)(-acc[a][b]);
                const uint64_t key = make_key(dist, (int32_t)xg);
                if (key < t) {
                    int pos = atomicAdd(&cnt[qr], 1);
                    buf[(size_t)qr * BUF + pos] = key;
                    if (pos + 1 > BUF - TX) atomicOr(need, 1);
                }
            }
        }
        __syncthreads();
        const bool last = xb + TX >= A.n;
        if (*need || last) {
            for (int qr = wv; qr < TQ; qr += NT / 64) {
                const int c = cnt[qr];
                if (c == 0) continue;
                flush_query(top + (size_t)qr * A.kpad, &toplen[qr], buf + (size_t)qr * BUF, c, A.k);
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    cnt[qr] = 0;
                    if (toplen[qr] >= A.k) thr[qr] = top[(size_t)qr * A.kpad + A.k - 1];
                }
            }
            __syncthreads();
            if (tid == 0) *need = 0;
            __syncthreads();
        }
    }
    for (int i = tid; i < TQ * A.k; i += NT) {
        const int qr = i / A.k, j = i % A.k;
        const int64_t qg = q0 + qr;
        if (qg >= A.nq) continue;
        if (j < toplen[qr]) {
            const uint64_t key = top[(size_t)qr * A.kpad + j];
            A.ids[qg * A.k + j] = key_id(key);
            A.dists[qg * A.k + j] = key_dist(key);
        } else {
            A.ids[qg * A.k + j] = -1;
            A.dists[qg * A.k + j] = __builtin_inff();
        }
    }
}

}  // namespace

int launch_knn(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq, int64_t ldq,
               int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists, hipStream_t stream)
{
    if (nq == 0) return SA_OK;
    KnnArgs A;
    A.base = base; A.n = n; A.ld = ld; A.queries = queries; A.nq = nq; A.ldq = ldq;
    A.d = d; A.k = k; A.metric = metric; A.exclude_self = exclude_self; A.ids = ids; A.dists = dists;
    A.kpad = (k + 63) / 64 * 64;
    size_t lds = sizeof(float) * (size_t)(TQ + TX) * (DC + 1);
    lds = (lds + 15) / 16 * 16;
    lds += 8ull * TQ * A.kpad + 8ull * TQ * BUF + 4ull * (TQ + TQ + 2) + 8ull * TQ;
    lds = (lds + 15) / 16 * 16;
    if (lds > 160u * 1024u) return set_error(SA_EINVAL, "k=%d needs too much LDS", k);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(knn_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(knn)");
    const int64_t blocks = (nq + TQ - 1) / TQ;
    hipLaunchKernelGGL(knn_kernel, dim3((unsigned)blocks), dim3(NT), lds, stream, A);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "knn kernel launch");
    return SA_OK;
}

}  // namespace sa
