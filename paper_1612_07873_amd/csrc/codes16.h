// 16-bit storage codes shared by the kernels that keep links, clover terms or
// vectors as FP16 or BF16 pairs (one complex number per 32-bit word, real part
// in the low half).  Decoding is exact; encoding rounds to nearest even.
#pragma once

#include "qmg_internal.h"

namespace qmg {

__device__ __forceinline__ uint16_t f32_to_h16(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
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

}  // namespace qmg
