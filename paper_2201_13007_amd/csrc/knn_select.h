// Top-k selection shared by the exact-search kernels: a sorted list of the best keys per
// query and an unsorted buffer of candidates, merged by one wavefront at a time.
#pragma once
#include "sa_internal.h"

namespace sa {
namespace knn_detail {

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
__device__ inline void sort128(unsigned long long &lo, unsigned long long &hi)
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

// merge the cnt <= 128 keys of buf (unsorted) into the sorted list top[0..*len), keeping k
__device__ inline void flush_query(uint64_t *top, int *len, uint64_t *buf, int cnt, int k)
{
    const int lane = __lane_id();
    unsigned long long lo = lane < cnt ? buf[lane] : KEY_EMPTY;
    unsigned long long hi = lane + 64 < cnt ? buf[lane + 64] : KEY_EMPTY;
    sort128(lo, hi);
    __builtin_amdgcn_wave_barrier();
    // only the cnt real keys go back (the rest sort to the end as empty): the buffer may be
    // shorter than 128
    if (lane < cnt) buf[lane] = lo;
    if (lane + 64 < cnt) buf[lane + 64] = hi;
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

}  // namespace knn_detail
}  // namespace sa
