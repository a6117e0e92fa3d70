// Low-precision number formats on the device (bf16, fp16, OCP e4m3fn).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mxlu {

enum { kFmtBf16 = 0, kFmtFp16 = 1 };

// ---- FP64 -> 16-bit format, round to nearest even, directly from the FP64
// bits (no intermediate FP32 rounding).  MANT stored mantissa bits, BIAS
// exponent bias; overflow gives infinity; FP64 values below half the smallest
// subnormal give zero.
template <int MANT, int BIAS>
__device__ __forceinline__ uint16_t f64_to_ieee16(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
    const uint64_t a = u & 0x7fffffffffffffffull;
    constexpr int EXPBITS = 15 - MANT;
    constexpr uint16_t INF = (uint16_t)(((1u << EXPBITS) - 1u) << MANT);
    if (a >= 0x7ff0000000000000ull) {                        // inf or NaN
        return (a == 0x7ff0000000000000ull) ? (uint16_t)(sign | INF)
                                            : (uint16_t)(sign | INF | (1u << (MANT - 1)));
    }
    const int e2 = (int)(a >> 52);
    if (e2 == 0) return sign;                                // FP64 zero/subnormal
    const int e = e2 - 1023;
    const uint64_t full = (a & 0x000fffffffffffffull) | 0x0010000000000000ull;
    constexpr int EMIN = 1 - BIAS, EMAX = BIAS;
    int shift = 52 - MANT;
    int biased;
    if (e >= EMIN) {
        biased = e + BIAS;
    } else {
        shift += EMIN - e;                                   // subnormal target
        biased = 0;
    }
    if (shift >= 64) return sign;
    uint64_t q = full >> shift;
    const uint64_t rem = full & ((1ull << shift) - 1ull);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1ull))) ++q;
    uint32_t bits;
    if (biased == 0) {
        bits = (uint32_t)q;            // q == 2^MANT lands on the smallest normal
    } else {
        if (q == (2ull << MANT)) {     // mantissa overflow
            q >>= 1;
            ++biased;
        }
        if (biased > EMAX + BIAS) return (uint16_t)(sign | INF);
        bits = ((uint32_t)biased << MANT) | ((uint32_t)q & ((1u << MANT) - 1u));
    }
    return (uint16_t)(sign | bits);
}

template <int FMT>
__device__ __forceinline__ uint16_t f64_to_lp(double x) {
    return FMT == kFmtBf16 ? f64_to_ieee16<7, 127>(x) : f64_to_ieee16<10, 15>(x);
}

// ---- 16-bit format <-> FP32 (FP32 holds every bf16/fp16 value exactly).
template <int FMT>
__device__ __forceinline__ float lp_to_f32(uint16_t h) {
    if (FMT == kFmtBf16) return __uint_as_float((uint32_t)h << 16);
    return (float)__builtin_bit_cast(_Float16, h);
}

// FP32 -> 16-bit, round to nearest even (finite inputs).
template <int FMT>
__device__ __forceinline__ uint16_t f32_to_lp(float f) {
    if (FMT == kFmtBf16) {
        const uint32_t u = __float_as_uint(f);
        const uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)((u + bias) >> 16);
    }
    return __builtin_bit_cast(uint16_t, (_Float16)f);
}

// ---- FP32 -> OCP e4m3fn, round to nearest even, saturating at +-448 (the
// format has no infinities; 0x7f/0xff are NaN).  Written from the format
// definition: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits, subnormals
// at exponent field 0 with quantum 2^-9.
__device__ __forceinline__ uint8_t f32_to_e4m3(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    const uint32_t a = u & 0x7fffffffu;
    if (a >= 0x7f800000u) return (uint8_t)(sign | 0x7e);     // inf -> 448 (NaN not expected)
    const int e2 = (int)(a >> 23);
    if (e2 == 0) return sign;                                // FP32 zero/subnormal (< 2^-126)
    const int e = e2 - 127;
    const uint32_t full = (a & 0x7fffffu) | 0x800000u;       // 24 bits
    int shift = 23 - 3;
    int biased;
    if (e >= -6) {
        biased = e + 7;
    } else {
        shift += -6 - e;
        biased = 0;
    }
    if (shift >= 32) return sign;
    uint32_t q = full >> shift;
    const uint32_t rem = full & ((1u << shift) - 1u);
    const uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1u))) ++q;
    uint32_t bits;
    if (biased == 0) {
        bits = q;
    } else {
        if (q == 16u) {
            q >>= 1;
            ++biased;
        }
        bits = ((uint32_t)biased << 3) | (q & 7u);
        if (biased > 15 || bits > 0x7eu) bits = 0x7eu;       // saturate at 448
    }
    return (uint8_t)(sign | bits);
}

// Smallest power of two s with amax / s <= 448 (s = 1 for amax = 0).
// The ratio is formed in FP64 so that the power-of-two test is exact.
// E8M0 exponent e of the MX block scale 2^e: the smallest e with
// amax / 2^e <= 448, limited to [-127, 127]; 0 for an all-zero block.
__device__ __forceinline__ int mx_block_exp(float amax) {
    if (!(amax > 0.0f)) return 0;
    int e;
    const double m = frexp((double)amax / 448.0, &e);
    const int k = (m == 0.5) ? e - 1 : e;
    return k < -127 ? -127 : (k > 127 ? 127 : k);
}

__device__ __forceinline__ float fp8_tile_scale(float amax) {
    if (!(amax > 0.0f)) return 1.0f;
    const double r = (double)amax / 448.0;
    int e;
    const double m = frexp(r, &e);        // r = m 2^e, m in [0.5, 1)
    return (float)ldexp(1.0, (m == 0.5) ? e - 1 : e);
}

}  // namespace mxlu
