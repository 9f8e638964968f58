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

// x = hi + mid (+ lo) in bf16, each part the rounding of the remainder
template <int NPL>
__device__ __forceinline__ void split_bf16(float x, __bf16 part[NPL]) {
    float r = x;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        __bf16 h = (__bf16)r;
        part[i] = h;
        r -= (float)h;
    }
}

template <int BASIS>
__device__ __forceinline__ void basis_pair(double t, double amp, float& cb, float& sb) {
    float r = (float)frac_centered(t);
    if (BASIS == BASIS_DIFF) {
        float sh = __builtin_amdgcn_sinf(0.5f * r);  // sin(pi r)
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
