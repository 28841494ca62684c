// Message arithmetic of the on-chip BP decoders, as policies: the same
// decoder runs eq. (1) in FP32 min-sum (F32) or on saturating b-bit
// integers (Fixed), the hardware setting in which the paper counts a PE's
// cost (Sections I and V).
//
// Fixed: every message is an integer in [-Q, Q], Q = 2^(b-1) - 1, held
// exactly in an FP32 register (all sums, products by a/16 and the +-1/2 of
// the rounding stay far below 2^24).  The channel is clamp(round(LLR 2^F));
// each sum of eq. (1) saturates; the scaled minimum is
// sign(x) sign(y) floor((a min(|x|, |y|) + 8) / 16), a = round(16 alpha),
// unsaturated; +-Q stands for the +-inf of frozen rows; hard decisions keep
// the exact sum's sign.
#pragma once

#include <hip/hip_runtime.h>

namespace pbp {
namespace arith {
namespace {

// sign(y) min(|x|, |y|): y clamped to [-|x|, |x|] (a selection, exact)
__device__ __forceinline__ float clampm(float x, float y)
{
    return __builtin_amdgcn_fmed3f(-fabsf(x), y, fabsf(x));
}

// alpha carrying the sign of x.  The min-sum term of eq. (1),
// alpha sign(x) sign(y) min(|x|, |y|), is salpha(x) * clampm(x, y): one
// product, rounded once and symmetrically in sign.  A PE's two terms with
// the same first operand share salpha, so a PE costs 11 FP32 operations.  A
// zero result may carry either sign; no value or decision depends on it.
__device__ __forceinline__ float salpha(float x, float alpha)
{
    return __builtin_copysignf(alpha, x);
}

// alpha: the PE's scale (F32: alpha; Fixed: round(16 alpha) / 16, exact);
// q: Q (Fixed only); frac: fraction bits of the channel quantizer (Fixed).
struct F32 {
    static constexpr bool kFixed = false;
    __device__ static __forceinline__ float big(float) { return __builtin_inff(); }
    __device__ static __forceinline__ float channel(float v, int, float) { return v; }
    __device__ static __forceinline__ void pe(float La, float Lb, float Ra, float Rb,
                                              float alpha, float, float &la,
                                              float &lbv, float &ra, float &rb)
    {
        const float s = Lb + Rb;
        const float aLa = salpha(La, alpha);
        const float g1 = aLa * clampm(La, Ra);
        la = aLa * clampm(La, s);
        lbv = Lb + g1;
        ra = salpha(Ra, alpha) * clampm(Ra, s);
        rb = Rb + g1;
    }
};

struct Fixed {
    static constexpr bool kFixed = true;
    __device__ static __forceinline__ float big(float q) { return q; }
    __device__ static __forceinline__ float sat(float v, float q)
    {
        return __builtin_amdgcn_fmed3f(v, -q, q);
    }
    // clamp(round(LLR 2^F), -Q, Q), halves away from zero (the product by
    // 2^F is exact)
    __device__ static __forceinline__ float channel(float v, int frac, float q)
    {
        return sat(roundf(ldexpf(v, frac)), q);
    }
    // sign(x) sign(y) floor((a/16) min(|x|, |y|) + 1/2), a/16 the PE's scale
    // (the argument a): the magnitude (a/16) min + 1/2 is a multiple of 1/32
    // far below 2^24, so the fma is exact, and the sign bits of x and y are
    // applied once to the rounded magnitude
    __device__ static __forceinline__ float term(float a, float x, float y)
    {
        const float r = floorf(__builtin_fmaf(a, fminf(fabsf(x), fabsf(y)), 0.5f));
        return __builtin_copysignf(
            r, __uint_as_float(__float_as_uint(x) ^ __float_as_uint(y)));
    }
    // one PE of eq. (1): every sum saturates, the scaled minima do not
    __device__ static __forceinline__ void pe(float La, float Lb, float Ra, float Rb,
                                              float a, float q, float &la,
                                              float &lbv, float &ra, float &rb)
    {
        const float s = sat(Lb + Rb, q);
        const float g1 = term(a, La, Ra);
        la = term(a, La, s);
        lbv = sat(Lb + g1, q);
        ra = term(a, Ra, s);
        rb = sat(Rb + g1, q);
    }
};

}  // namespace
}  // namespace arith
}  // namespace pbp
