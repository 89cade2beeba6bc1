// Reduced-precision copies of the vectors (the storage types of sa_dtype), written from
// the format definitions: bf16 keeps the upper half of the float32 pattern rounded to
// nearest even; fp8 e4m3 (finite variant: bias 7, three mantissa bits, subnormals
// m * 2^-9, largest 448) takes a per-vector scale amax / 448, and each coordinate divided
// by it is rounded to nearest even and saturated.
#include "sa_internal.h"

namespace sa {
namespace {

__device__ __forceinline__ uint32_t to_bf16(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (b >> 16) | 0x40u;   // quiet NaN
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ uint32_t to_e4m3(float x)
{
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a < 448.f)) return sign | 0x7Eu;
    if (a < 0.015625f) return sign | (uint32_t)rintf(a * 512.f);   // below 2^-6: units of 2^-9
    int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;          // a in [2^e, 2^(e+1)), e in [-6, 8]
    const float frac = a * __uint_as_float((uint32_t)(127 - e) << 23); // a / 2^e, exact, in [1, 2)
    uint32_t m = (uint32_t)rintf((frac - 1.f) * 8.f);
    if (m == 8u) {
        m = 0u;
        ++e;
    }
    return sign | ((uint32_t)(e + 7) << 3) | m;
}

// one wavefront per row
__global__ void __launch_bounds__(256) quantize_kernel(const float *x, int64_t n, int d, int64_t ld, int dtype,
                                                       void *codes, int64_t ldc, float *scale)
{
    const int lane = __lane_id();
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const float *r = x + row * ld;
    float s = 1.f;
    if (dtype == SA_FP8E4M3) {
        float amax = 0.f;
        for (int c = lane; c < d; c += 64) amax = fmaxf(amax, fabsf(r[c]));
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        s = amax > 0.f ? amax / 448.f : 1.f;
    }
    for (int c = lane; c < ldc; c += 64) {
        const float v = c < d ? r[c] : 0.f;
        if (dtype == SA_BF16) static_cast<uint16_t *>(codes)[row * ldc + c] = (uint16_t)to_bf16(v);
        else static_cast<uint8_t *>(codes)[row * ldc + c] = (uint8_t)to_e4m3(v / s);
    }
    if (lane == 0) scale[row] = s;
}

}  // namespace

int launch_quantize(const float *x, int64_t n, int32_t d, int64_t ld, int32_t dtype, void *codes, int64_t ldc,
                    float *scale, hipStream_t stream)
{
    if (n == 0) return SA_OK;
    hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, x, n, d, ld, dtype,
                       codes, ldc, scale);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

}  // namespace sa
