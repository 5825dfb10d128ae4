// Device-side helpers shared by the libmips kernels: outward rounding,
// the bfloat16 and OCP E4M3 screen encodings, and wave-level primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef int intx8_t __attribute__((ext_vector_type(8)));
typedef int intx4_t __attribute__((ext_vector_type(4)));

namespace mips {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kTile = 32;     // items (and users) per matrix-core tile edge

// ---------------------------------------------------------------------------
// Outward rounding of non-negative float64 quantities to float32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float next_up_f32(float y) {
    // next float toward +inf for finite y
    uint32_t b = __float_as_uint(y);
    if (y == 0.0f) return __uint_as_float(1u);
    return __uint_as_float((b >> 31) ? b - 1u : b + 1u);
}

__device__ __forceinline__ float round_up_f32(double x) {
    float y = (float)x;                       // round to nearest
    if ((double)y < x) y = next_up_f32(y);
    return y;
}

// Smallest float >= x * (1 + 2^-40): absorbs the float64 rounding of sums of
// squares and square roots (relative error far below 2^-40 for f <= 256).
__device__ __forceinline__ float norm_up_f32(double x) {
    return round_up_f32(x * (1.0 + 0x1p-40));
}

// ---------------------------------------------------------------------------
// bfloat16, round to nearest even (finite inputs).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7FFFu + lsb;
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// ---------------------------------------------------------------------------
// OCP E4M3 ("FN": bias 7, no infinities, max finite 448, min normal 2^-6,
// subnormal step 2^-9).  Encoding rounds to nearest even and saturates to
// +-448; inputs here are pre-scaled so |x| <= 448.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float e4m3_decode(uint32_t byte) {
    uint32_t s = (byte >> 7) & 1u, e = (byte >> 3) & 15u, m = byte & 7u;
    float mag = (e == 0) ? (float)m * 0x1p-9f
                         : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return s ? -mag : mag;
}

__device__ __forceinline__ uint32_t e4m3_encode(float x) {
    uint32_t sign = (__float_as_uint(x) >> 31) << 7;
    float a = __builtin_fabsf(x);
    if (!(a > 0.0f)) return sign;                     // zero (NaN is rejected earlier)
    if (a >= 448.0f) return sign | 0x7Eu;            // saturate to 448
    uint32_t b = __float_as_uint(a);
    int e = (int)((b >> 23) & 255u) - 127;           // unbiased exponent
    if (e < -6) {
        // subnormal range: value = m * 2^-9, m in [0, 8]
        float q = a * 0x1p9f;                         // exact (power-of-two scaling)
        float r = __builtin_rintf(q);                 // nearest, ties to even
        uint32_t m = (uint32_t)r;                     // m == 8 is the smallest normal
        return sign | m;                              // m=8 -> e=1,m=0 pattern 0b0001000
    }
    // normal: keep 3 mantissa bits with round-to-nearest-even on the float bits
    uint32_t lsb = (b >> 20) & 1u;
    uint32_t rb = b + 0x7FFFFu + lsb;
    int e2 = (int)((rb >> 23) & 255u) - 127;
    uint32_t m3 = (rb >> 20) & 7u;
    if (e2 > 8 || (e2 == 8 && m3 > 6)) return sign | 0x7Eu;  // above 448 after rounding
    return sign | ((uint32_t)(e2 + 7) << 3) | m3;
}

// Power-of-two scale exponent k for a row whose largest magnitude is amax:
// the smallest k with amax * 2^-k <= 448, clamped to the E8M0 range
// [-127, 127] (0 for a zero row).
__device__ __forceinline__ int e4m3_row_scale_exp(float amax) {
    if (!(amax > 0.0f)) return 0;
    int ex;
    (void)__builtin_frexpf(amax, &ex);               // amax = m 2^ex, m in [0.5, 1)
    int k = (ex - 1) - 8;                             // amax 2^-k in [256, 512)
    if (__builtin_ldexpf(amax, -k) > 448.0f) ++k;    // now in [128, 448]
    if (k < -127) k = -127;
    if (k > 127) k = 127;
    return k;
}

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// Value held by lane (lane ^ 32), by the VALU lane-swap of the two wave
// halves (v_permlane32_swap: with both operands equal, the first result holds
// the lower half's values in both halves and the second the upper half's).
__device__ __forceinline__ uint32_t xor32_u(uint32_t v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() < 32) ? r[1] : r[0];
}
__device__ __forceinline__ float xor32_f(float v) { return __uint_as_float(xor32_u(__float_as_uint(v))); }
__device__ __forceinline__ int xor32_i(int v) { return (int)xor32_u((uint32_t)v); }
__device__ __forceinline__ double xor32_d(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = xor32_u((uint32_t)b), hi = xor32_u((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Order-preserving maps for atomic max on non-negative floating point.
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    if (!(v >= 0.0)) return;
    atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

}  // namespace mips
