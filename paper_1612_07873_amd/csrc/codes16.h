// 16-bit storage codes shared by the kernels that keep links, clover terms or
// vectors as FP16 or BF16 pairs (one complex number per 32-bit word, real part
// in the low half).  Decoding is exact; encoding rounds to nearest even.
#pragma once

#include "qmg_internal.h"

namespace qmg {

// FP32 -> binary16, round to nearest even, written out from the formats (a
// plain conversion was lowered to a mixed-precision FMA whose rounding did not
// match round-to-nearest-even on every value): normal results round at
// mantissa bit 13 and re-bias the exponent (127 -> 15); results below 2^-14
// are multiples of 2^-24, rounded by rintf; from 65520 up the result is Inf.
__device__ __forceinline__ uint16_t f32_to_h16(float f) {
    const uint32_t x = __float_as_uint(f);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) return (uint16_t)(sign | (ax > 0x7f800000u ? 0x7e00u : 0x7c00u));   // NaN, Inf
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);                                  // overflow
    if (ax >= 0x38800000u) {                                                                   // normal
        const uint32_t r = ax + 0x0fffu + ((ax >> 13) & 1u) - 0x38000000u;
        return (uint16_t)(sign | (r >> 13));
    }
    return (uint16_t)(sign | (uint32_t)rintf(__uint_as_float(ax) * 16777216.0f));             // subnormal, zero
}
__device__ __forceinline__ float h16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
__device__ __forceinline__ uint16_t f32_to_b16(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float b16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// storage formats: complex128, complex64, FP16 pairs, BF16 pairs (the values of qmg_prec)
enum { FMT_F64 = 0, FMT_F32 = 1, FMT_H16 = 2, FMT_B16 = 3 };

template <int F> __device__ __forceinline__ float dec16(uint16_t v) {
    return F == FMT_H16 ? h16_to_f32(v) : b16_to_f32(v);
}
template <int F> __device__ __forceinline__ uint16_t enc16(float v) {
    return F == FMT_H16 ? f32_to_h16(v) : f32_to_b16(v);
}
template <int F> __device__ __forceinline__ cpx<float> dec_pair(uint32_t w) {
    return cpx<float>{dec16<F>((uint16_t)(w & 0xffffu)), dec16<F>((uint16_t)(w >> 16))};
}
template <int F> __device__ __forceinline__ uint32_t enc_pair(float re, float im) {
    return (uint32_t)enc16<F>(re) | ((uint32_t)enc16<F>(im) << 16);
}

// An encoder that met a NaN or Inf input (or a scale beyond FP32) records it
// in the per-device word nf (a vector atomic OR), which the next blocking
// call or qmg_sync turns into QMG_ERR_NONFINITE.
__device__ __forceinline__ void note_nonfinite(unsigned* nf, bool bad) {
    if (bad) atomicOr(nf, 1u);
}

}  // namespace qmg
