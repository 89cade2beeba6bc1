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
#include "knn_select.h"

namespace sa {
namespace {

using knn_detail::flush_query;

constexpr int TQ = 32;
constexpr int TX = 64;
constexpr int DC = 32;
constexpr int NT = 256;
constexpr int BUF = 128;   // per-query candidate buffer; flushed when > BUF - TX

struct KnnArgs {
    const float *base;
    int64_t n, ld;
    const float *queries;
    int64_t nq, ldq;
    int32_t d, k, kpad, metric, exclude_self;
    const int32_t *qmap;   // job j is query qmap[j] (its row, its self id, its output row); null: j
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
                const int64_t qs = qr < A.nq && A.qmap ? A.qmap[qr] : qr;
                Qs[r * (DC + 1) + c] = (qr < A.nq && c < dlen) ? A.queries[qs * A.ldq + dc + c] : 0.f;
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
            const int64_t self = A.qmap ? A.qmap[qg] : qg;
            const uint64_t t = thr[qr];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t xg = xb + tx + 16 * b;
                if (xg >= A.n || (A.exclude_self && xg == self)) continue;
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
        const int64_t orow = A.qmap ? A.qmap[qg] : qg;
        if (j < toplen[qr]) {
            const uint64_t key = top[(size_t)qr * A.kpad + j];
            A.ids[orow * A.k + j] = key_id(key);
            A.dists[orow * A.k + j] = key_dist(key);
        } else {
            A.ids[orow * A.k + j] = -1;
            A.dists[orow * A.k + j] = __builtin_inff();
        }
    }
}

}  // namespace

int launch_knn_scan(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq, int64_t ldq,
               int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists, hipStream_t stream,
               const int32_t *qmap)
{
    if (nq == 0) return SA_OK;
    KnnArgs A;
    A.base = base; A.n = n; A.ld = ld; A.queries = queries; A.nq = nq; A.ldq = ldq;
    A.d = d; A.k = k; A.metric = metric; A.exclude_self = exclude_self; A.ids = ids; A.dists = dists;
    A.qmap = qmap;
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
