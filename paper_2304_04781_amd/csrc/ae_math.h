// Scalar numerics shared by the autoencoder kernels (training and inference):
// bfloat16 rounding, the GELU activation and its derivative.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wv {

typedef __bf16 ae_bf16x2 __attribute__((ext_vector_type(2)));
typedef float ae_f32x2 __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest even (v_cvt_pk_bf16_f32; finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x)
{
    const ae_bf16x2 b = __builtin_convertvector((ae_f32x2{x, 0.0f}), ae_bf16x2);
    return (uint16_t)(__builtin_bit_cast(uint32_t, b) & 0xFFFFu);
}
// two floats -> packed bfloat16 pair (x in the low half)
__device__ __forceinline__ uint32_t f2bf2(float x, float y)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((ae_f32x2{x, y}), ae_bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// bfloat16 bits of the largest bfloat16 <= x and of the smallest bfloat16 >= x
// (finite x): truncation toward zero, moved one step away from zero when the
// dropped bits are nonzero and zero lies on the wrong side
__device__ __forceinline__ uint16_t bf16_down(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u >> 16) + (((u >> 31) != 0u && (u & 0xFFFFu) != 0u) ? 1u : 0u));
}
__device__ __forceinline__ uint16_t bf16_up(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u >> 16) + (((u >> 31) == 0u && (u & 0xFFFFu) != 0u) ? 1u : 0u));
}

// erf(x) by the rational-exponential approximation of Abramowitz & Stegun 7.1.26
// (Hastings): |error| <= 1.5e-7, far below the bfloat16 rounding of the hidden
// layer that follows every use. Branch-free: one reciprocal and one exp2.
__device__ __forceinline__ float erf_as(float x)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float y = fmaf(1.061405429f, t, -1.453152027f);
    y = fmaf(y, t, 1.421413741f);
    y = fmaf(y, t, -0.284496736f);
    y = fmaf(y, t, 0.254829592f);
    y *= t;
    const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
    return copysignf(fmaf(-y, e, 1.0f), x);
}

// GELU(x) = x Phi(x) = max(x, 0) - |x| Phi(-|x|), with Phi(-a) = erfc(a / sqrt 2) / 2 from the
// same approximation (argument scale and the 1/2 folded into its constants)
__device__ __forceinline__ float gelu(float x)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, ax, 1.0f));
    float y = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
    y = fmaf(y, t, 0.5f * 1.421413741f);
    y = fmaf(y, t, 0.5f * -0.284496736f);
    y = fmaf(y, t, 0.5f * 0.254829592f);
    y *= t;
    const float e = __builtin_amdgcn_exp2f(x * (x * (-0.5f * 1.4426950408889634f)));
    return fmaf(-ax, y * e, fmaxf(x, 0.0f));
}
__device__ __forceinline__ float gelu_prime(float x)
{
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
           x * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f) * 0.39894228040143268f;
}

}  // namespace wv
