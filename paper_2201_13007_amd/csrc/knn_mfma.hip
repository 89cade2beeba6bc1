// Exact k nearest neighbours on the matrix cores for integer-valued data, and the choice
// between this path and the double-precision scan of knn.hip.
//
// Exactness.  When every coordinate is an integer in [-255, 255] and d <= 256, bf16 holds
// each coordinate exactly, each product is an integer below 2^16 and every partial sum of
// a dot product stays below 256 * 255^2 < 2^24 in magnitude, so the fp32 accumulators of
// v_mfma_f32_16x16x32_bf16 hold the exact integer dot product whatever order the
// additions take.  The squared distance |q|^2 + |x|^2 - 2 q.x (or -q.x for the inner
// product) is then formed in 32-bit integers and rounded once to float, which is the key
// the scan produces, bit for bit.
//
// Work split.  A workgroup of four wavefronts owns MQ = 64 queries, whose bf16 rows stay
// in registers as the A operands (4 row blocks x d/32 k-steps).  The base streams in
// tiles of MT = 64 rows; wavefront w multiplies rows 16w .. 16w+15 of each tile against
// all 64 queries, loading its B operands from memory straight into a ring of registers
// that runs one or two tiles ahead of the products.
//
// Selection.  A product passes a cheap integer test first: u <= B_q with u = |x|^2 - 2 q.x
// and B_q = T_q - |q|^2, where T_q bounds from above every integer distance whose float
// rounding does not exceed the query's current k-th distance.  Only passing products
// build a 64-bit key and enter the query's LDS buffer, which is sorted and merged into
// the query's top-k list as in the scan.
//
// Float data (d <= 1024, k <= 96; above d = 128 the chunks of 32 dimensions are loaded per
// tile instead of held in registers).  Each coordinate is split into bf16 parts x = h + l + r
// (h and l rounded to nearest even, so |x - h| <= 2^-8 |x| and |r| <= 2^-16 |x|) and
// q.x is approximated by qh.xh + qh.xl + ql.xh on the matrix cores with fp32 accumulation.
// Its error is at most c |q| |x| with c = 3.1 2^-16 + (3d + 2) 2^-24 (the omitted terms,
// then every fp32 rounding of the 3d products), so every approximate distance is within E_q of the exact
// one, with E_q from |q| and the largest |x| (doubled for safety).  For L2 all points are
// first moved by the base mean (distances unchanged, norms and so the bound smaller).  The
// candidate kernel keeps the kc = 128 smallest approximate keys; the exact kernel rescores
// them with the scan's own FP64 arithmetic and keeps the k smallest exact keys.  Every
// point outside the list is then at least (kc-th approximate distance - E_q) away; if
// that exceeds the k-th exact key, none can enter the k best, and the result is the
// scan's, bit for bit.  The queries that cannot show that margin (ties within the bound)
// are listed and rescored by the scan alone.
#include "knn_select.h"

#include <climits>

namespace sa {
namespace {

using knn_detail::flush_query;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int MQ = 64;                 // queries per workgroup
constexpr int MT = 64;                 // base rows per tile
constexpr int MNT = 256;               // four wavefronts
constexpr int MBUF = 128;              // candidates buffered per query; flushed when > MBUF - MT
// the integer kernel's buffer: with its sorted lists k keys long (not rounded up), a
// workgroup then takes 76 KB of LDS at k = 65 and two fit on a CU (at 128 and a rounded
// list, 133 KB: one workgroup, one wavefront per SIMD, nothing to hide a barrier or a load)
constexpr int MBUF_I = 80;
constexpr int32_t NORM_PAD = 1 << 30;  // norm of padding rows

struct PrepArgs {
    const float *x;
    int64_t n, ld, rows;  // rows: n rounded up to the tile size
    int32_t d, dpad, metric;
    __bf16 *out;          // rows x dpad
    int32_t *norm;        // rows
    int32_t *bad;
};

// One wavefront per row: the bf16 copy (zero padded to dpad columns and `rows` rows), the
// exact integer squared norm (0 for the inner product, NORM_PAD for padding rows), and a
// flag raised by any value that is not an integer in [-255, 255] (NaN included).
__global__ void __launch_bounds__(256) knn_prep_kernel(PrepArgs P)
{
    const int lane = __lane_id();
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= P.rows) return;
    int sum = 0;
    bool bad = false;
    for (int c = lane; c < P.dpad; c += 64) {
        float v = 0.f;
        if (row < P.n && c < P.d) v = P.x[row * P.ld + c];
        const bool ok = fabsf(v) <= 255.f && v == rintf(v);
        bad |= !ok;
        const int iv = ok ? (int)v : 0;
        sum += iv * iv;
        P.out[row * P.dpad + c] = (__bf16)(ok ? v : 0.f);
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (bad) atomicOr(P.bad, 1);
    if (lane == 0) P.norm[row] = row < P.n ? (P.metric == SA_L2 ? sum : 0) : NORM_PAD;
}

// Upper bound, minus |q|^2, on the integer distances whose float rounding is at most the
// distance of key thr.  Distances here are roundings of integers, so the float is
// integral; below 2^24 it is exact, above it one unit in the last place covers every
// integer that rounds down onto it.  INT_MAX while the list is not full.
__device__ inline int prefilter_bound(uint64_t thr, int32_t qnorm)
{
    if (thr == KEY_EMPTY) return INT_MAX;
    const float f = key_dist(thr);
    int64_t t = (int64_t)f;
    const float a = fabsf(f);
    if (a >= 16777216.f) t += int64_t(1) << ((int)((__float_as_uint(a) >> 23) & 0xFF) - 127 - 23);
    t -= qnorm;
    return t > INT_MAX ? INT_MAX : (int)t;
}

struct MArgs {
    const __bf16 *xb;    // base rows, xrows x dpad
    const int32_t *xn;   // their norms
    const __bf16 *qb;    // query rows, a multiple of MQ rows x dpad
    const int32_t *qn;
    int64_t n, nq, xrows;
    int32_t dpad, k, kpad, exclude_self;
    int32_t *ids;
    float *dists;
};

template <int KS, bool L2>
__global__ void __launch_bounds__(MNT) knn_mfma_kernel(MArgs A)
{
    constexpr int NB = KS <= 4 ? 3 : 2;  // register ring: tiles in flight + the one in use
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint64_t *top = reinterpret_cast<uint64_t *>(smem);   // [MQ][kpad] sorted best keys
    uint64_t *buf = top + (size_t)MQ * A.kpad;             // [MQ][MBUF_I] unsorted candidates
    uint64_t *thr = buf + (size_t)MQ * MBUF_I;             // [MQ] k-th key (or empty)
    int *cnt = reinterpret_cast<int *>(thr + MQ);          // [MQ] buffered candidates
    int *len = cnt + MQ;                                   // [MQ] length of top
    int *bnd = len + MQ;                                   // [MQ] B_q of the prefilter
    int *qns = bnd + MQ;                                   // [MQ] |q|^2
    int *need = qns + MQ;  // 1 + index of the last tile in which a buffer passed MBUF_I - MT

    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * MQ;
    for (int i = tid; i < MQ; i += MNT) {
        cnt[i] = 0;
        len[i] = 0;
        thr[i] = KEY_EMPTY;
        bnd[i] = q0 + i < A.nq ? INT_MAX : INT_MIN;  // padding queries take nothing
        qns[i] = A.qn[q0 + i];
    }
    if (tid == 0) *need = 0;

    bf16x8 a[4][KS];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const __bf16 *p = A.qb + (q0 + rb * 16 + (lane & 15)) * A.dpad + 8 * (lane >> 4);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a[rb][ks] = *reinterpret_cast<const bf16x8 *>(p + ks * 32);
    }
    __syncthreads();
    // lane holds output rows 4 (lane / 16) + r of each row block, column lane % 16
    int bq[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) bq[rb][r] = bnd[rb * 16 + 4 * (lane >> 4) + r];

    const int64_t ntile = A.xrows / MT;
    bf16x8 b[NB][KS];
    int bn[NB];
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) {
        const int64_t row = (j < ntile ? j : ntile - 1) * MT + 16 * w + (lane & 15);
        const __bf16 *p = A.xb + row * A.dpad + 8 * (lane >> 4);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[j][ks] = *reinterpret_cast<const bf16x8 *>(p + ks * 32);
        bn[j] = A.xn[row];
    }

    for (int64_t t0 = 0; t0 < ntile; t0 += NB) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int64_t t = t0 + j;
            if (t >= ntile) break;
            {
                // refill the slot freed by the previous tile; past the end, reload the last tile
                const int jn = (j + NB - 1) % NB;
                const int64_t tn = t + NB - 1 < ntile ? t + NB - 1 : ntile - 1;
                const int64_t row = tn * MT + 16 * w + (lane & 15);
                const __bf16 *p = A.xb + row * A.dpad + 8 * (lane >> 4);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) b[jn][ks] = *reinterpret_cast<const bf16x8 *>(p + ks * 32);
                bn[jn] = A.xn[row];
            }
            f32x4 acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb][ks], b[j][ks], acc[rb], 0, 0, 0);
            const int64_t col = t * MT + 16 * w + (lane & 15);
            const int nx = bn[j];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int dneg = (int)(-acc[rb][r]);  // -q.x, exact
                    const int u = L2 ? nx + 2 * dneg : dneg;
                    if (u <= bq[rb][r]) {
                        const int row = rb * 16 + 4 * (lane >> 4) + r;
                        if (col < A.n && !(A.exclude_self && col == q0 + row)) {
                            const uint64_t key = make_key((float)(qns[row] + u), (int32_t)col);
                            if (key < thr[row]) {
                                const int pos = atomicAdd(&cnt[row], 1);
                                buf[(size_t)row * MBUF_I + pos] = key;
                                if (pos + 1 > MBUF_I - MT) *need = (int)(t + 1);
                            }
                        }
                    }
                }
            __syncthreads();
            // every wavefront reads the same value: a later tile can only write after the
            // barrier that follows a flush
            const bool last = t + 1 == ntile;
            if (*need == (int)(t + 1) || last) {
                for (int qr = w; qr < MQ; qr += MNT / 64) {
                    const int c = cnt[qr];
                    if (c == 0) continue;
                    flush_query(top + (size_t)qr * A.kpad, &len[qr], buf + (size_t)qr * MBUF_I, c, A.k);
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0) {
                        cnt[qr] = 0;
                        if (len[qr] >= A.k) {
                            const uint64_t th = top[(size_t)qr * A.kpad + A.k - 1];
                            thr[qr] = th;
                            bnd[qr] = prefilter_bound(th, qns[qr]);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) bq[rb][r] = bnd[rb * 16 + 4 * (lane >> 4) + r];
            }
        }
    }
    for (int i = tid; i < MQ * A.k; i += MNT) {
        const int qr = i / A.k, j = i % A.k;
        const int64_t qg = q0 + qr;
        if (qg >= A.nq) continue;
        if (j < len[qr]) {
            const uint64_t key = top[(size_t)qr * A.kpad + j];
            A.ids[qg * A.k + j] = key_id(key);
            A.dists[qg * A.k + j] = key_dist(key);
        } else {
            A.ids[qg * A.k + j] = -1;
            A.dists[qg * A.k + j] = __builtin_inff();
        }
    }
}

// ---------------------------------------------------------------- float data

constexpr int KC = 128;        // candidates kept per query (k <= 96)

// column sums of the base in double (L2 centring): one block per row chunk
__global__ void __launch_bounds__(256) knn_colsum_kernel(const float *x, int64_t n, int d, int64_t ld, int64_t chunk,
                                                         double *sum)
{
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = r0 + chunk < n ? r0 + chunk : n;
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += (double)x[r * ld + c];
        atomicAdd(sum + c, acc);
    }
}

// float -> bf16 bits, rounded to nearest even (finite inputs; an overflow rounds to inf)
__device__ __forceinline__ uint16_t bf16_rne_bits(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

struct FPrepArgs {
    const float *x;
    int64_t n, ld, rows;
    int32_t d, dpad;
    const double *colsum;  // L2: subtract colsum / n_base from every coordinate (null: none)
    double n_base;
    __bf16 *hi, *lo;      // rows x dpad
    float *norm2;         // rows: |x|^2 (rounded once from double)
    unsigned *max_norm2;  // bits of the largest |x|^2 (non-negative floats order as unsigned)
    int32_t *bad;         // any non-finite value
};

__global__ void __launch_bounds__(256) knn_prep_float_kernel(FPrepArgs P)
{
    const int lane = __lane_id();
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= P.rows) return;
    double sum = 0.0;
    bool bad = false;
    for (int c = lane; c < P.dpad; c += 64) {
        float v = 0.f;
        if (row < P.n && c < P.d) v = P.x[row * P.ld + c];
        if (!(fabsf(v) <= 3.0e38f)) {
            bad = true;
            v = 0.f;
        }
        if (P.colsum && row < P.n && c < P.d) v -= (float)(P.colsum[c] / P.n_base);
        // nonzero magnitudes below 2^-60 could give subnormal bf16 parts, which the matrix
        // cores may flush: such data goes to the scan
        if (v != 0.f && fabsf(v) < 0x1p-60f) bad = true;
        const uint16_t hb = bf16_rne_bits(v);
        const float hf = __uint_as_float((uint32_t)hb << 16);
        const uint16_t lb = bf16_rne_bits(v - hf);   // v - hf is exact
        P.hi[row * P.dpad + c] = __builtin_bit_cast(__bf16, hb);
        P.lo[row * P.dpad + c] = __builtin_bit_cast(__bf16, lb);
        sum += (double)v * (double)v;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (bad) atomicOr(P.bad, 1);
    if (lane == 0) {
        const float nf = (float)sum;
        P.norm2[row] = row < P.n ? nf : __builtin_inff();
        if (row < P.n) atomicMax(P.max_norm2, __float_as_uint(nf));
    }
}

struct FArgs {
    const __bf16 *xh, *xl;   // base parts, xrows x dpad
    const float *xn;         // base |x|^2
    const __bf16 *qh, *ql;   // query parts, a multiple of MQ rows x dpad
    const float *qn;
    int64_t n, nq, xrows;
    int32_t dpad, kc, kpad, exclude_self;
    int32_t *cand;           // nq x kc candidate ids (approximate order)
    float *cand_d;           // their approximate distances
    int32_t *cand_len;       // nq
};

// The candidate pass: as knn_mfma_kernel, with three bf16 products per block and the
// approximate distance |q|^2 + |x|^2 - 2 q.x (or -q.x) in fp32.
template <int KS, bool L2>
__global__ void __launch_bounds__(MNT) knn_mfma_float_kernel(FArgs A)
{
    constexpr int NB = 3;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint64_t *top = reinterpret_cast<uint64_t *>(smem);   // [MQ][kpad]
    uint64_t *buf = top + (size_t)MQ * A.kpad;             // [MQ][MBUF]
    uint64_t *thr = buf + (size_t)MQ * MBUF;               // [MQ]
    int *cnt = reinterpret_cast<int *>(thr + MQ);          // [MQ]
    int *len = cnt + MQ;                                   // [MQ]
    float *qns = reinterpret_cast<float *>(len + MQ);      // [MQ]
    int *need = reinterpret_cast<int *>(qns + MQ);

    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * MQ;
    for (int i = tid; i < MQ; i += MNT) {
        cnt[i] = 0;
        len[i] = 0;
        thr[i] = q0 + i < A.nq ? KEY_EMPTY : 0ull;   // padding queries take nothing
        qns[i] = A.qn[q0 + i];
    }
    if (tid == 0) *need = 0;

    bf16x8 ah[4][KS], al[4][KS];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t off = (q0 + rb * 16 + (lane & 15)) * A.dpad + 8 * (lane >> 4);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            ah[rb][ks] = *reinterpret_cast<const bf16x8 *>(A.qh + off + ks * 32);
            al[rb][ks] = *reinterpret_cast<const bf16x8 *>(A.ql + off + ks * 32);
        }
    }
    __syncthreads();

    const int64_t ntile = A.xrows / MT;
    bf16x8 bh[NB][KS], bl[NB][KS];
    float bn[NB];
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) {
        const int64_t row = (j < ntile ? j : ntile - 1) * MT + 16 * w + (lane & 15);
        const int64_t off = row * A.dpad + 8 * (lane >> 4);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bh[j][ks] = *reinterpret_cast<const bf16x8 *>(A.xh + off + ks * 32);
            bl[j][ks] = *reinterpret_cast<const bf16x8 *>(A.xl + off + ks * 32);
        }
        bn[j] = A.xn[row];
    }

    for (int64_t t0 = 0; t0 < ntile; t0 += NB) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int64_t t = t0 + j;
            if (t >= ntile) break;
            {
                const int jn = (j + NB - 1) % NB;
                const int64_t tn = t + NB - 1 < ntile ? t + NB - 1 : ntile - 1;
                const int64_t row = tn * MT + 16 * w + (lane & 15);
                const int64_t off = row * A.dpad + 8 * (lane >> 4);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    bh[jn][ks] = *reinterpret_cast<const bf16x8 *>(A.xh + off + ks * 32);
                    bl[jn][ks] = *reinterpret_cast<const bf16x8 *>(A.xl + off + ks * 32);
                }
                bn[jn] = A.xn[row];
            }
            f32x4 acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb][ks], bh[j][ks], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb][ks], bl[j][ks], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rb][ks], bh[j][ks], acc[rb], 0, 0, 0);
                }
            const int64_t col = t * MT + 16 * w + (lane & 15);
            const float nx = bn[j];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rb * 16 + 4 * (lane >> 4) + r;
                    if (col < A.n && !(A.exclude_self && col == q0 + row)) {
                        const float dt = L2 ? (qns[row] + nx) - 2.f * acc[rb][r] : -acc[rb][r];
                        const uint64_t key = make_key(dt, (int32_t)col);
                        if (key < thr[row]) {
                            const int pos = atomicAdd(&cnt[row], 1);
                            buf[(size_t)row * MBUF + pos] = key;
                            if (pos + 1 > MBUF - MT) *need = (int)(t + 1);
                        }
                    }
                }
            __syncthreads();
            const bool last = t + 1 == ntile;
            if (*need == (int)(t + 1) || last) {
                for (int qr = w; qr < MQ; qr += MNT / 64) {
                    const int c = cnt[qr];
                    if (c == 0) continue;
                    flush_query(top + (size_t)qr * A.kpad, &len[qr], buf + (size_t)qr * MBUF, c, A.kc);
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0) {
                        cnt[qr] = 0;
                        if (len[qr] >= A.kc) thr[qr] = top[(size_t)qr * A.kpad + A.kc - 1];
                    }
                }
                __syncthreads();
            }
        }
    }
    for (int i = tid; i < MQ * A.kc; i += MNT) {
        const int qr = i / A.kc, j = i % A.kc;
        const int64_t qg = q0 + qr;
        if (qg >= A.nq) continue;
        const bool ok = j < len[qr];
        const uint64_t key = ok ? top[(size_t)qr * A.kpad + j] : KEY_EMPTY;
        A.cand[qg * A.kc + j] = ok ? key_id(key) : -1;
        A.cand_d[qg * A.kc + j] = ok ? key_dist(key) : __builtin_inff();
        if (j == 0) A.cand_len[qg] = len[qr];
    }
}

struct EArgs {
    const float *base;
    int64_t n, ld;
    const float *queries;
    int64_t nq, ldq;
    int32_t d, k, kc, metric;
    const int32_t *cand;
    const float *cand_d;
    const int32_t *cand_len;
    const float *qn;            // |q|^2 per query (the candidate pass's)
    const unsigned *max_norm2;
    int32_t *ids;
    float *dists;
    int32_t *failed;            // count of queries whose list could not show the margin
    int32_t *failed_list;       // those queries, in any order
};

// One wavefront per query: the exact keys of the candidates with the scan's arithmetic
// (double, index order, separately rounded multiply and add, one rounding to float) and
// the k smallest, then the margin test.  A point outside the list has an approximate
// distance of at least the list's last one, so its exact distance is at least that less
// E_q; if that exceeds the k-th exact key by more than a few float units (the keys are
// roundings), no outside point can enter the k best.
__global__ void __launch_bounds__(64) knn_exact_kernel(EArgs E)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *qs = reinterpret_cast<float *>(smem);
    const int lane = __lane_id();
    const int64_t q = blockIdx.x;
    const int nc = E.cand_len[q];
    const int32_t *cd = E.cand + q * E.kc;
    for (int c = lane; c < E.d; c += 64) qs[c] = E.queries[q * E.ldq + c];
    __builtin_amdgcn_wave_barrier();
    unsigned long long key[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = lane + 64 * h;
        key[h] = KEY_EMPTY;
        if (j < nc && j < E.kc) {
            const int32_t id = cd[j];
            const float *x = E.base + (int64_t)id * E.ld;
            double acc = 0.0;
            if (E.metric == SA_L2) {
                for (int c = 0; c < E.d; ++c) {
                    const double t = (double)qs[c] - (double)x[c];
                    acc += t * t;
                }
            } else {
                for (int c = 0; c < E.d; ++c) acc += (double)qs[c] * (double)x[c];
            }
            key[h] = make_key(E.metric == SA_L2 ? (float)acc : (float)(-acc), id);
        }
    }
    knn_detail::sort128(key[0], key[1]);
    if (nc >= E.kc) {
        // (for L2 the last term also covers the rounding of the centred coordinates)
        const double c = 3.1 / 65536.0 + (3.0 * E.d + 2.0) / 16777216.0;
        const double nq_ = sqrt((double)E.qn[q]), nm = sqrt((double)__uint_as_float(*E.max_norm2));
        // (the last term: fp32 products and partial sums below 2^-126 that may be flushed)
        const double tiny = (3.0 * E.d + 2.0) * 0x1p-126;
        const double err = E.metric == SA_L2 ? 2.0 * (2.0 * c * nq_ * nm + 8.0 / 16777216.0 * (nq_ + nm) * (nq_ + nm) + 2.0 * tiny)
                                             : 2.0 * (c * nq_ * nm + 2.0 / 16777216.0 * nq_ * nm + tiny);
        const int kk = E.k - 1;
        const unsigned long long kth = __shfl(kk < 64 ? key[0] : key[1], kk & 63, 64);
        const double Kk = key_dist(kth);
        const double last = E.cand_d[q * E.kc + E.kc - 1];
        if (!(last - err > Kk + fabs(Kk) * (1.0 / 1048576.0))) {
            if (lane == 0) E.failed_list[atomicAdd(E.failed, 1)] = (int32_t)q;
            return;
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = lane + 64 * h;
        if (j < E.k) {
            const bool ok = key[h] != KEY_EMPTY;
            E.ids[q * E.k + j] = ok ? key_id(key[h]) : -1;
            E.dists[q * E.k + j] = ok ? key_dist(key[h]) : __builtin_inff();
        }
    }
}

// The candidate pass for larger d (128 < d <= 1024): the same products, with the query
// and base parts of each 32-dimension chunk loaded per tile (queries from the caches,
// the next chunk's operands in flight while the current chunk's products run).
template <bool L2>
__global__ void __launch_bounds__(MNT) knn_mfma_float_kloop_kernel(FArgs A)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint64_t *top = reinterpret_cast<uint64_t *>(smem);
    uint64_t *buf = top + (size_t)MQ * A.kpad;
    uint64_t *thr = buf + (size_t)MQ * MBUF;
    int *cnt = reinterpret_cast<int *>(thr + MQ);
    int *len = cnt + MQ;
    float *qns = reinterpret_cast<float *>(len + MQ);
    int *need = reinterpret_cast<int *>(qns + MQ);

    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * MQ;
    for (int i = tid; i < MQ; i += MNT) {
        cnt[i] = 0;
        len[i] = 0;
        thr[i] = q0 + i < A.nq ? KEY_EMPTY : 0ull;
        qns[i] = A.qn[q0 + i];
    }
    if (tid == 0) *need = 0;
    __syncthreads();

    const int nks = A.dpad / 32;
    const int64_t ntile = A.xrows / MT;
    const int koff = 8 * (lane >> 4);
    int64_t qoff[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) qoff[rb] = (q0 + rb * 16 + (lane & 15)) * A.dpad + koff;
    for (int64_t t = 0; t < ntile; ++t) {
        const int64_t xoff = (t * MT + 16 * w + (lane & 15)) * A.dpad + koff;
        f32x4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x8 ah[2][4], al[2][4], bh[2], bl[2];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            ah[0][rb] = *reinterpret_cast<const bf16x8 *>(A.qh + qoff[rb]);
            al[0][rb] = *reinterpret_cast<const bf16x8 *>(A.ql + qoff[rb]);
        }
        bh[0] = *reinterpret_cast<const bf16x8 *>(A.xh + xoff);
        bl[0] = *reinterpret_cast<const bf16x8 *>(A.xl + xoff);
        for (int ks = 0; ks < nks; ks += 2) {
            // chunk ks + 1 in flight while chunk ks multiplies, then the other way round
            const int k1 = ks + 1 < nks ? ks + 1 : ks;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                ah[1][rb] = *reinterpret_cast<const bf16x8 *>(A.qh + qoff[rb] + 32 * k1);
                al[1][rb] = *reinterpret_cast<const bf16x8 *>(A.ql + qoff[rb] + 32 * k1);
            }
            bh[1] = *reinterpret_cast<const bf16x8 *>(A.xh + xoff + 32 * k1);
            bl[1] = *reinterpret_cast<const bf16x8 *>(A.xl + xoff + 32 * k1);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0][rb], bh[0], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0][rb], bl[0], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[0][rb], bh[0], acc[rb], 0, 0, 0);
            }
            if (ks + 1 >= nks) break;
            const int k2 = ks + 2 < nks ? ks + 2 : ks + 1;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                ah[0][rb] = *reinterpret_cast<const bf16x8 *>(A.qh + qoff[rb] + 32 * k2);
                al[0][rb] = *reinterpret_cast<const bf16x8 *>(A.ql + qoff[rb] + 32 * k2);
            }
            bh[0] = *reinterpret_cast<const bf16x8 *>(A.xh + xoff + 32 * k2);
            bl[0] = *reinterpret_cast<const bf16x8 *>(A.xl + xoff + 32 * k2);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1][rb], bh[1], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1][rb], bl[1], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[1][rb], bh[1], acc[rb], 0, 0, 0);
            }
        }
        const int64_t col = t * MT + 16 * w + (lane & 15);
        const float nx = A.xn[t * MT + 16 * w + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rb * 16 + 4 * (lane >> 4) + r;
                if (col < A.n && !(A.exclude_self && col == q0 + row)) {
                    const float dt = L2 ? (qns[row] + nx) - 2.f * acc[rb][r] : -acc[rb][r];
                    const uint64_t key = make_key(dt, (int32_t)col);
                    if (key < thr[row]) {
                        const int pos = atomicAdd(&cnt[row], 1);
                        buf[(size_t)row * MBUF + pos] = key;
                        if (pos + 1 > MBUF - MT) *need = (int)(t + 1);
                    }
                }
            }
        __syncthreads();
        const bool last = t + 1 == ntile;
        if (*need == (int)(t + 1) || last) {
            for (int qr = w; qr < MQ; qr += MNT / 64) {
                const int c = cnt[qr];
                if (c == 0) continue;
                flush_query(top + (size_t)qr * A.kpad, &len[qr], buf + (size_t)qr * MBUF, c, A.kc);
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    cnt[qr] = 0;
                    if (len[qr] >= A.kc) thr[qr] = top[(size_t)qr * A.kpad + A.kc - 1];
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < MQ * A.kc; i += MNT) {
        const int qr = i / A.kc, j = i % A.kc;
        const int64_t qg = q0 + qr;
        if (qg >= A.nq) continue;
        const bool ok = j < len[qr];
        const uint64_t key = ok ? top[(size_t)qr * A.kpad + j] : KEY_EMPTY;
        A.cand[qg * A.kc + j] = ok ? key_id(key) : -1;
        A.cand_d[qg * A.kc + j] = ok ? key_dist(key) : __builtin_inff();
        if (j == 0) A.cand_len[qg] = len[qr];
    }
}

using FKernel = void (*)(FArgs);

FKernel pick_float_kernel(int ks, int metric)
{
    switch (ks) {
    case 1: return metric == SA_L2 ? knn_mfma_float_kernel<1, true> : knn_mfma_float_kernel<1, false>;
    case 2: return metric == SA_L2 ? knn_mfma_float_kernel<2, true> : knn_mfma_float_kernel<2, false>;
    case 3: return metric == SA_L2 ? knn_mfma_float_kernel<3, true> : knn_mfma_float_kernel<3, false>;
    case 4: return metric == SA_L2 ? knn_mfma_float_kernel<4, true> : knn_mfma_float_kernel<4, false>;
    default: return metric == SA_L2 ? knn_mfma_float_kloop_kernel<true> : knn_mfma_float_kloop_kernel<false>;
    }
}

using MKernel = void (*)(MArgs);

template <int KS>
MKernel pick(int metric)
{
    return metric == SA_L2 ? knn_mfma_kernel<KS, true> : knn_mfma_kernel<KS, false>;
}

MKernel pick_kernel(int ks, int metric)
{
    switch (ks) {
    case 1: return pick<1>(metric);
    case 2: return pick<2>(metric);
    case 3: return pick<3>(metric);
    case 4: return pick<4>(metric);
    case 6: return pick<6>(metric);
    case 8: return pick<8>(metric);
    default: return nullptr;
    }
}

struct DeviceBlock {
    void *p = nullptr;
    ~DeviceBlock()
    {
        if (p) (void)hipFree(p);
    }
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Runs the matrix-core path if every coordinate qualifies; *ran tells whether it did.
int launch_knn_mfma(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq,
                    int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists,
                    bool *ran, hipStream_t s)
{
    *ran = false;
    int ks = (d + 31) / 32;
    if (ks == 5) ks = 6;
    if (ks == 7) ks = 8;
    const int dpad = 32 * ks;
    const int64_t xrows = (n + MT - 1) / MT * MT;
    const bool shared_q = queries == base && ldq == ld && nq <= n;
    const int64_t qrows = shared_q ? xrows : (nq + MQ - 1) / MQ * MQ;
    const size_t xb_bytes = align256((size_t)xrows * dpad * 2), xn_bytes = align256((size_t)xrows * 4);
    const size_t qb_bytes = shared_q ? 0 : align256((size_t)qrows * dpad * 2);
    const size_t qn_bytes = shared_q ? 0 : align256((size_t)qrows * 4);
    DeviceBlock mem;
    if (hipMalloc(&mem.p, xb_bytes + xn_bytes + qb_bytes + qn_bytes + 256) != hipSuccess) {
        (void)hipGetLastError();
        mem.p = nullptr;
        return set_error(SA_ENOMEM, "hipMalloc of the bf16 copies failed");
    }
    unsigned char *m = static_cast<unsigned char *>(mem.p);
    __bf16 *xb = reinterpret_cast<__bf16 *>(m);
    int32_t *xn = reinterpret_cast<int32_t *>(m + xb_bytes);
    __bf16 *qb = shared_q ? xb : reinterpret_cast<__bf16 *>(m + xb_bytes + xn_bytes);
    int32_t *qn = shared_q ? xn : reinterpret_cast<int32_t *>(m + xb_bytes + xn_bytes + qb_bytes);
    int32_t *bad = reinterpret_cast<int32_t *>(m + xb_bytes + xn_bytes + qb_bytes + qn_bytes);

    SA_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    PrepArgs P{base, n, ld, xrows, d, dpad, metric, xb, xn, bad};
    hipLaunchKernelGGL(knn_prep_kernel, dim3((unsigned)((xrows + 3) / 4)), dim3(256), 0, s, P);
    SA_HIP(hipGetLastError());
    if (!shared_q) {
        PrepArgs Q{queries, nq, ldq, qrows, d, dpad, metric, qb, qn, bad};
        hipLaunchKernelGGL(knn_prep_kernel, dim3((unsigned)((qrows + 3) / 4)), dim3(256), 0, s, Q);
        SA_HIP(hipGetLastError());
    }
    int32_t flag = 0;
    SA_HIP(hipMemcpyAsync(&flag, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    if (flag) return SA_OK;

    MArgs A;
    A.xb = xb; A.xn = xn; A.qb = qb; A.qn = qn;
    A.n = n; A.nq = nq; A.xrows = xrows;
    A.dpad = dpad; A.k = k; A.kpad = k; A.exclude_self = exclude_self;
    A.ids = ids; A.dists = dists;
    const size_t lds = 8ull * MQ * A.kpad + 8ull * MQ * MBUF_I + 8ull * MQ + 4ull * 4 * MQ + 16;
    if (lds > 160u * 1024u) return set_error(SA_EINVAL, "k=%d needs too much LDS", k);
    MKernel kern = pick_kernel(ks, metric);
    if (!kern) return set_error(SA_EUNSUPPORTED, "d=%d", d);
    SA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)((nq + MQ - 1) / MQ)), dim3(MNT), lds, s, A);
    SA_HIP(hipGetLastError());
    SA_HIP(hipStreamSynchronize(s));
    *ran = true;
    return SA_OK;
}

// The float path for d <= 1024 and k <= 96; *ran is false on non-finite data (the caller
// then runs the scan).  Queries that cannot show their margin are rescored by the scan
// here.  Synchronous.
int launch_knn_mfma_float(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq,
                          int64_t ldq, int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists,
                          bool *ran, hipStream_t s)
{
    *ran = false;
    const int ks = (d + 31) / 32;
    const int dpad = 32 * ks;
    const int kc = KC;
    const int64_t xrows = (n + MT - 1) / MT * MT;
    const bool shared_q = queries == base && ldq == ld && nq <= n;
    const int64_t qrows = shared_q ? xrows : (nq + MQ - 1) / MQ * MQ;
    const size_t xp = align256((size_t)xrows * dpad * 2), xn_b = align256((size_t)xrows * 4);
    const size_t qp = shared_q ? 0 : align256((size_t)qrows * dpad * 2), qn_b = shared_q ? 0 : align256((size_t)qrows * 4);
    const size_t cand_b = align256((size_t)nq * kc * 4), len_b = align256((size_t)nq * 4);
    const size_t mu_b = align256((size_t)d * 8);
    DeviceBlock mem;
    const size_t total = 2 * xp + xn_b + 2 * qp + qn_b + 2 * cand_b + 2 * len_b + mu_b + 256;
    if (hipMalloc(&mem.p, total) != hipSuccess) {
        (void)hipGetLastError();
        mem.p = nullptr;
        return set_error(SA_ENOMEM, "hipMalloc of the bf16 parts failed");
    }
    unsigned char *m = static_cast<unsigned char *>(mem.p);
    __bf16 *xh = reinterpret_cast<__bf16 *>(m); m += xp;
    __bf16 *xl = reinterpret_cast<__bf16 *>(m); m += xp;
    float *xn = reinterpret_cast<float *>(m); m += xn_b;
    __bf16 *qh = shared_q ? xh : reinterpret_cast<__bf16 *>(m); m += qp;
    __bf16 *ql = shared_q ? xl : reinterpret_cast<__bf16 *>(m); m += qp;
    float *qn = shared_q ? xn : reinterpret_cast<float *>(m); m += qn_b;
    int32_t *cand = reinterpret_cast<int32_t *>(m); m += cand_b;
    float *cand_d = reinterpret_cast<float *>(m); m += cand_b;
    int32_t *cand_len = reinterpret_cast<int32_t *>(m); m += len_b;
    int32_t *failed_list = reinterpret_cast<int32_t *>(m); m += len_b;
    double *colsum = reinterpret_cast<double *>(m); m += mu_b;
    unsigned *flags = reinterpret_cast<unsigned *>(m);   // [0] max |x|^2, [1] bad, [2] failed, [3] unused norm
    SA_HIP(hipMemsetAsync(flags, 0, 16, s));
    const double *mu = nullptr;
    if (metric == SA_L2) {
        // distances do not change when every point moves by the base mean, and the bound,
        // which grows with the norms, shrinks
        SA_HIP(hipMemsetAsync(colsum, 0, (size_t)d * 8, s));
        const int64_t chunk = (n + 4095) / 4096;
        hipLaunchKernelGGL(knn_colsum_kernel, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(256), 0, s, base, n, d,
                           ld, chunk, colsum);
        SA_HIP(hipGetLastError());
        mu = colsum;
    }
    FPrepArgs P{base, n, ld, xrows, d, dpad, mu, (double)n, xh, xl, xn, flags, reinterpret_cast<int32_t *>(flags + 1)};
    hipLaunchKernelGGL(knn_prep_float_kernel, dim3((unsigned)((xrows + 3) / 4)), dim3(256), 0, s, P);
    SA_HIP(hipGetLastError());
    if (!shared_q) {
        // queries do not take part in the largest |x|: their maximum goes to an unused word
        FPrepArgs Q{queries, nq, ldq, qrows, d, dpad, mu, (double)n, qh, ql, qn, flags + 3,
                    reinterpret_cast<int32_t *>(flags + 1)};
        hipLaunchKernelGGL(knn_prep_float_kernel, dim3((unsigned)((qrows + 3) / 4)), dim3(256), 0, s, Q);
        SA_HIP(hipGetLastError());
    }
    FArgs A;
    A.xh = xh; A.xl = xl; A.xn = xn; A.qh = qh; A.ql = ql; A.qn = qn;
    A.n = n; A.nq = nq; A.xrows = xrows;
    A.dpad = dpad; A.kc = kc; A.kpad = (kc + 63) / 64 * 64; A.exclude_self = exclude_self;
    A.cand = cand; A.cand_d = cand_d; A.cand_len = cand_len;
    const size_t lds = 8ull * MQ * A.kpad + 8ull * MQ * MBUF + 8ull * MQ + 3ull * 4 * MQ + 16;
    FKernel kern = pick_float_kernel(ks, metric);
    if (!kern || lds > 160u * 1024u) return SA_OK;
    SA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)((nq + MQ - 1) / MQ)), dim3(MNT), lds, s, A);
    SA_HIP(hipGetLastError());
    EArgs E{base, n, ld, queries, nq, ldq, d, k, kc, metric, cand, cand_d, cand_len, qn, flags, ids, dists,
            reinterpret_cast<int32_t *>(flags + 2), failed_list};
    hipLaunchKernelGGL(knn_exact_kernel, dim3((unsigned)nq), dim3(64), 4 * (size_t)dpad, s, E);
    SA_HIP(hipGetLastError());
    unsigned hf[3] = {0, 0, 0};
    SA_HIP(hipMemcpyAsync(hf, flags, 12, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    if (hf[1] != 0) return SA_OK;
    if (hf[2] > 0) {
        // the listed queries' rows are written by the scan; every other row is final
        const int rc = launch_knn_scan(base, n, d, ld, queries, (int64_t)hf[2], ldq, k, metric, exclude_self, ids,
                                       dists, s, failed_list);
        if (rc != SA_OK) return rc;
        SA_HIP(hipStreamSynchronize(s));
        knn_rescanned = hf[2];
    }
    *ran = true;
    return SA_OK;
}

}  // namespace

thread_local int64_t knn_rescanned = 0;

int launch_knn(const float *base, int64_t n, int32_t d, int64_t ld, const float *queries, int64_t nq, int64_t ldq,
               int32_t k, int32_t metric, int32_t exclude_self, int32_t *ids, float *dists, int32_t path,
               int32_t *path_used, hipStream_t stream)
{
    if (path_used) *path_used = SA_KNN_AUTO;
    knn_rescanned = 0;
    if (path != SA_KNN_AUTO && path != SA_KNN_SCAN && path != SA_KNN_MFMA)
        return set_error(SA_EINVAL, "unknown kNN path %d", path);
    if (nq == 0) return SA_OK;
    const bool int_shape = n >= 1 && d <= 256 && k <= 128;    // integer-valued data
    const bool flt_shape = n >= 1 && d <= 1024 && k <= 96;    // any finite data
    if (path == SA_KNN_MFMA && !int_shape && !flt_shape)
        return set_error(SA_EUNSUPPORTED, "the MFMA kNN path needs n >= 1 and d <= 256, k <= 128 (integer data) or "
                         "d <= 1024, k <= 96 (n=%lld, d=%d, k=%d)", (long long)n, d, k);
    if (path != SA_KNN_SCAN) {
        bool ran = false;
        if (int_shape) {
            const int rc = launch_knn_mfma(base, n, d, ld, queries, nq, ldq, k, metric, exclude_self, ids, dists,
                                           &ran, stream);
            if (rc != SA_OK) return rc;
        }
        // not integer data (or too wide for it): the float path, where its shape allows
        if (!ran && flt_shape) {
            const int rf = launch_knn_mfma_float(base, n, d, ld, queries, nq, ldq, k, metric, exclude_self, ids,
                                                 dists, &ran, stream);
            if (rf != SA_OK) return rf;
        }
        if (ran) {
            if (path_used) *path_used = SA_KNN_MFMA;
            return SA_OK;
        }
        if (path == SA_KNN_MFMA)
            return set_error(SA_EUNSUPPORTED, "the MFMA kNN path needs integer coordinates in [-255, 255] (d <= 256, "
                             "k <= 128) or finite floats with d <= 1024 and k <= 96");
    }
    const int rc = launch_knn_scan(base, n, d, ld, queries, nq, ldq, k, metric, exclude_self, ids, dists, stream);
    if (rc != SA_OK) return rc;
    SA_HIP(hipStreamSynchronize(stream));
    if (path_used) *path_used = SA_KNN_SCAN;
    return SA_OK;
}

}  // namespace sa
