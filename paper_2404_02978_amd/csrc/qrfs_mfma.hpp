// qrfs_mfma.hpp -- MFMA operand types and the basis / operand-split
// helpers shared by the fused and the two-phase contraction kernels.
#pragma once

#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"

namespace qrfs {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// x = hi + mid (+ lo) in bf16, each part the rounding (to nearest even) of
// the remainder left by the parts before it; split for two values at once:
// plane i of (x0, x1) as one packed word, x0 in the low half (the element
// order of the MFMA operands).  One pair conversion per plane; the
// remainders take each half back to binary32 by a shift or a mask.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int NPL>
__device__ __forceinline__ void split_bf16x2(float x0, float x1, uint32_t part[NPL]) {
    float r0 = x0, r1 = x1;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        const f32x2 r = {r0, r1};
        const bf16x2 h = __builtin_convertvector(r, bf16x2);
        const uint32_t u = __builtin_bit_cast(uint32_t, h);
        part[i] = u;
        if (i + 1 < NPL) {
            r0 -= __uint_as_float(u << 16);
            r1 -= __uint_as_float(u & 0xffff0000u);
        }
    }
}

// Eight values (one MFMA operand register group) into NPL operand planes:
// word j of each plane holds elements 2j and 2j + 1.
template <int NPL>
__device__ __forceinline__ void split8_bf16(const float (&v)[8], bf16x8 (&o)[NPL]) {
    uint32_t w[NPL][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t part[NPL];
        split_bf16x2<NPL>(v[2 * j], v[2 * j + 1], part);
#pragma unroll
        for (int i = 0; i < NPL; ++i) w[i][j] = part[i];
    }
#pragma unroll
    for (int i = 0; i < NPL; ++i) o[i] = __builtin_bit_cast(bf16x8, w[i]);
}

// FP16x3 operands: x = hi + lo in fp16.  hi is x rounded to nearest fp16,
// the remainder x - hi is exact in binary32, and lo is its rounding:
// |x - hi - lo| <= 2^-22 |x| in the normal fp16 range and below 2^-25
// absolute where hi or lo is an fp16 subnormal.  The caller keeps
// |x| < 2^15.  Two values at once: hi and lo each as one packed word,
// x0 in the low half (the element order of the MFMA operands).
// Two forms with the same values: FEW forms the remainder with one
// v_fma_mix_f32 per value that reads hi as an fp16 operand (4 instructions
// per pair, for loops bound by vector issue); otherwise hi is converted
// back and subtracted (6 per pair, plain code the scheduler can interleave
// with MFMAs, where the inline-asm form serialises).
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x16 mfma_f16(f16x8 a, f16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

template <bool FEW>
__device__ __forceinline__ void split_f16x2(float x0, float x1, uint32_t part[2]) {
    const f32x2 x = {x0, x1};
    const f16x2 hv = __builtin_convertvector(x, f16x2);
    const uint32_t h = __builtin_bit_cast(uint32_t, hv);
    f32x2 r;
    if constexpr (FEW) {
        float r0, r1;
        // r = x - hi with hi read as fp16 from its half of the packed word
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r0) : "v"(h), "v"(x0));
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
            : "=v"(r1)
            : "v"(h), "v"(x1));
        r = f32x2{r0, r1};
    } else {
        r = x - __builtin_convertvector(hv, f32x2);
    }
    part[0] = h;
    part[1] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, f16x2));
}

template <bool FEW = true>
__device__ __forceinline__ void split8_f16(const float (&v)[8], f16x8 (&o)[2]) {
    uint32_t w[2][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t part[2];
        split_f16x2<FEW>(v[2 * j], v[2 * j + 1], part);
        w[0][j] = part[0];
        w[1][j] = part[1];
    }
    o[0] = __builtin_bit_cast(f16x8, w[0]);
    o[1] = __builtin_bit_cast(f16x8, w[1]);
}

// Power-of-two scale 2^s (and 2^-s) that brings a largest magnitude m into
// [2^13, 2^14), so FP16x3 basis values (at most 2 m) stay below the fp16
// maximum; s is clamped to [-100, 100] (1 for m = 0).
__device__ __forceinline__ void f16_scale(double m, double& scale, float& unscale) {
    int s = 0;
    if (m > 0.0) {
        s = 13 - ilogb(m);
        s = s < -100 ? -100 : (s > 100 ? 100 : s);
    }
    scale = ldexp(1.0, s);
    unscale = ldexpf(1.0f, -s);
}

template <int BASIS>
__device__ __forceinline__ void basis_pair(double t, double amp, float& cb, float& sb) {
    float r = frac_rev_f32(t);
    if (BASIS == BASIS_DIFF) {
        float sh = __builtin_amdgcn_sinf(0.5f * r);  // sin(pi r), squared below
        cb = -2.0f * sh * sh;                         // cos(2 pi r) - 1
        sb = __builtin_amdgcn_sinf(r);
    } else {
        cb = __builtin_amdgcn_cosf(r);
        sb = __builtin_amdgcn_sinf(r);
    }
    float fa = (float)amp;
    cb *= fa;
    sb *= fa;
}

}  // namespace qrfs
