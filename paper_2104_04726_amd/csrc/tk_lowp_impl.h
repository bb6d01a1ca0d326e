// Encodings, storage codecs and matrix-instruction wrappers shared by the reduced-precision kernels
// (included by the translation units of the reduced-precision GEMM and by tk_lowp.hip; everything
// here is internal to each of them).
#pragma once
#include "tk_common.h"
#include "tk_lowp.h"

namespace tk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------- encodings
__device__ __forceinline__ uint16_t enc_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // RNE
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float dec_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t enc_f16(float x) {
    _Float16 h = (_Float16)x;                 // RNE conversion instruction
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float dec_f16(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// OCP E4M3: s eeee mmm, bias 7; exponent field 0 is subnormal (m * 2^-9); 0x7f / 0xff is NaN
__device__ __forceinline__ uint8_t enc_e4m3(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    const float a = fabsf(x);
    if (!(a == a)) return sign | 0x7f;
    if (a >= 464.0f) return sign | 0x7e;                 // saturate (448 and above round to 448)
    if (a < 0.015625f) {                                 // below 2^-6: subnormal grid of 2^-9
        const int m = (int)rintf(a * 512.0f);            // 0..8 (8 is the smallest normal, 0x08)
        return sign | (uint8_t)m;
    }
    const uint32_t ua = __float_as_uint(a);
    int e = (int)((ua >> 23) & 0xffu) - 127;
    uint32_t mant = ua & 0x7fffffu;
    const uint32_t r = mant + 0x7ffffu + ((mant >> 20) & 1u);   // RNE to 3 mantissa bits
    uint32_t m3 = (r >> 20) & 7u;
    if (r & 0x800000u) {
        ++e;
        m3 = 0;
    }
    const int E = e + 7;                                  // 1..15 here (a < 464)
    return sign | (uint8_t)(E << 3) | (uint8_t)m3;
}
// decode by the hardware conversion (v_cvt_f32_fp8), which reads gfx950's FP8 bytes as OCP E4M3 like
// the matrix instructions do; exact (every E4M3 value is a binary32 value)
__device__ __forceinline__ float dec_e4m3(uint8_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

template <int P> struct Codec;
template <> struct Codec<LP_BF16> {
    typedef uint16_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_bf16(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_bf16(h); }
};
template <> struct Codec<LP_F16> {
    typedef uint16_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_f16(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_f16(h); }
};
template <> struct Codec<LP_FP8> {
    typedef uint8_t S;
    static __device__ __forceinline__ S enc(float x) { return enc_e4m3(x); }
    static __device__ __forceinline__ float dec(S h) { return dec_e4m3(h); }
};

// eight consecutive elements: 16 bytes for 16-bit types, 8 bytes for FP8
template <int P> struct Vec8 { typedef uint4 T; };
template <> struct Vec8<LP_FP8> { typedef uint2 T; };

template <int P>
__device__ __forceinline__ f32x4 mfma32(const typename Vec8<P>::T& a, const typename Vec8<P>::T& b, f32x4 c);
template <>
__device__ __forceinline__ f32x4 mfma32<LP_BF16>(const uint4& a, const uint4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma32<LP_F16>(const uint4& a, const uint4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma32<LP_FP8>(const uint2& a, const uint2& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0,
                                                      0, 0);
}

__device__ __forceinline__ int64_t coloff(const Desc& d, int64_t c) {
    return (c / d.seg) * d.segstride + (c % d.seg);
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    if (G < 16) return b;
    const int64_t q = G / 8, r = G % 8;
    const int64_t x = b % 8, idx = b / 8;
    return x * q + (x < r ? x : r) + idx;
}

}  // namespace
}  // namespace tk
