// Exact re-rank of a search's final list (the search_params rerank option): every query's
// search leaves the ids of the first nr entries of its final list in its workspace region
// (see rerank_list in search_body.h); one wavefront per query recomputes their distances
// from the float32 vectors, writes the first k by key and zeroes the list again.
#include "search_body.h"

namespace sa {
namespace {

using search_detail::VecSrc;
using search_detail::distances;
using search_detail::lanes_per_vector;

struct RArgs {
    const float *vec32;
    int64_t ld32;
    const float *queries;
    int64_t ldq;
    int32_t d, k;
    unsigned char *ws;
    int64_t stride, list_off;   // bytes per workspace region, and of the list within it
    int32_t *ids;
    float *dists;
    const int32_t *order, *qk;  // batches: the query of region b, per-query k (null: b, k)
    int64_t ldo;                // row stride of ids and dists
};

__device__ __forceinline__ uint64_t wave_min64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

template <int LPV, int NI, bool L2>
__global__ void __launch_bounds__(64) rerank_kernel(RArgs R)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint64_t *const nkey = reinterpret_cast<uint64_t *>(smem);    // [64]
    int32_t *const sid = reinterpret_cast<int32_t *>(nkey + 64);   // [64]
    float *const qs = reinterpret_cast<float *>(sid + 64);          // [16 LPV]
    const int lane = __lane_id();
    const int64_t job = blockIdx.x;
    const int64_t qi = R.order ? R.order[job] : job;
    const int kq = R.qk ? R.qk[qi] : R.k;
    int32_t *const list = reinterpret_cast<int32_t *>(R.ws + job * R.stride + R.list_off);
    {
        const int nch = R.d >> 2;
        const float *qrow = R.queries + qi * R.ldq;
        for (int c = lane; c < 4 * LPV; c += 64)
            reinterpret_cast<float4 *>(qs)[c] =
                c < nch ? *reinterpret_cast<const float4 *>(qrow + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int nr = list[0];
    const VecSrc X{R.vec32, nullptr, R.ld32};
    uint64_t ek[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        ek[i] = KEY_EMPTY;
        if (64 * i < nr) {
            const int cnt = min(64, nr - 64 * i);
            const int32_t id = list[1 + 64 * i + lane];   // the region holds 1024 ids
            sid[lane] = lane < cnt ? id : 0;
            __builtin_amdgcn_wave_barrier();
            distances<LPV, L2, SA_F32>(X, R.d, qs, sid, cnt, nkey);
            __builtin_amdgcn_wave_barrier();
            ek[i] = lane < cnt ? nkey[lane] : KEY_EMPTY;
            __builtin_amdgcn_wave_barrier();
        }
    }
    // the first k exact keys, one selection round each
    for (int r = 0; r < kq; ++r) {
        uint64_t best = ek[0];
#pragma unroll
        for (int i = 1; i < NI; ++i) best = ek[i] < best ? ek[i] : best;
        best = wave_min64(best);
#pragma unroll
        for (int i = 0; i < NI; ++i) ek[i] = ek[i] == best ? KEY_EMPTY : ek[i];
        if (lane == 0) {
            R.ids[qi * R.ldo + r] = best == KEY_EMPTY ? -1 : key_id(best);
            R.dists[qi * R.ldo + r] = best == KEY_EMPTY ? __builtin_inff() : key_dist(best);
        }
    }
    for (int j = lane; j <= nr; j += 64) list[j] = 0;   // leave the workspace zero-filled
}

template <int LPV, int NI>
hipError_t launch1(const RArgs &R, bool l2, int64_t nq, hipStream_t s)
{
    auto k = l2 ? rerank_kernel<LPV, NI, true> : rerank_kernel<LPV, NI, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)nq), dim3(64), 64 * 8 + 64 * 4 + 64 * LPV, s, R);
    return hipGetLastError();
}

template <int LPV>
hipError_t launch1_ni(const RArgs &R, bool l2, int L, int64_t nq, hipStream_t s)
{
    const int ni = (L + 63) / 64;
    if (ni <= 1) return launch1<LPV, 1>(R, l2, nq, s);
    if (ni <= 2) return launch1<LPV, 2>(R, l2, nq, s);
    if (ni <= 4) return launch1<LPV, 4>(R, l2, nq, s);
    if (ni <= 6) return launch1<LPV, 6>(R, l2, nq, s);
    if (ni <= 8) return launch1<LPV, 8>(R, l2, nq, s);
    return launch1<LPV, 16>(R, l2, nq, s);
}

}  // namespace

int launch_rerank(const float *vec32, int64_t ld32, const float *queries, int64_t ldq, int64_t nq, int32_t d,
                  int32_t metric, int32_t k, int32_t L, void *ws, int64_t stride, int64_t list_off, int32_t *ids,
                  float *dists, const int32_t *order, const int32_t *qk, int64_t ldo, hipStream_t s)
{
    RArgs R{vec32, ld32, queries, ldq, d, k, static_cast<unsigned char *>(ws), stride, list_off, ids, dists,
            order, qk, ldo > 0 ? ldo : k};
    const bool l2 = metric == SA_L2;
    hipError_t e;
    switch (lanes_per_vector(d)) {
    case 1: e = launch1_ni<1>(R, l2, L, nq, s); break;
    case 2: e = launch1_ni<2>(R, l2, L, nq, s); break;
    case 4: e = launch1_ni<4>(R, l2, L, nq, s); break;
    case 8: e = launch1_ni<8>(R, l2, L, nq, s); break;
    case 16: e = launch1_ni<16>(R, l2, L, nq, s); break;
    case 32: e = launch1_ni<32>(R, l2, L, nq, s); break;
    default: e = launch1_ni<64>(R, l2, L, nq, s); break;
    }
    if (e != hipSuccess) return hip_fail(e, "re-rank kernel launch");
    return SA_OK;
}

}  // namespace sa
