// qrfs_peaks.hip -- throughput probes for the roofline denominators (gfx950).
//
// Each probe is a bounded amount of independent work of one instruction
// class: register-only MFMA chains (four accumulators per wave, so the
// matrix core never waits on a result), register-only FMA chains (eight per
// lane) and a streaming copy.  The caller times a launch and divides the
// nominal work it reports by the time.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "qrfs_peaks.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kChains = 4;     // accumulators per wave (MFMA)
constexpr int kFmaChains = 8;  // independent chains per lane (VALU)

// Operand value of (lane, chain j, element e, operand o) when the probe runs
// on varied data: a multiple of 1/16 in [-1, 1) from an integer hash, so
// every product and every partial sum is exact in binary32.
__device__ __forceinline__ float probe_value(int lane, int j, int e, int o) {
    uint32_t h = (uint32_t)lane * 0x9E3779B1u ^ (uint32_t)(j * 16 + e) * 0x85EBCA6Bu ^
                 (uint32_t)o * 0xC2B2AE35u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (float)((int)((h >> 7) & 31u) - 16) * 0.0625f;
}

// KIND: 0 bf16, 1 fp16, 2 FP32 operands.  x != 0: every operand equals x;
// x == 0: each chain has its own varied operands, so consecutive MFMAs read
// different data, as real contractions do (the matrix cores draw more
// power, and the clock can drop, when their inputs change).
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_peak_mfma(int iters, float x,
                                                        float* __restrict__ out) {
    typedef typename std::conditional<KIND == 2, float,
                                      typename std::conditional<KIND == 1, f16x8, bf16x8>::type>::type
        Op;
    const int lane = threadIdx.x & 63;
    Op a[kChains], b[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        if constexpr (KIND == 2) {
            a[j] = x != 0.0f ? x : probe_value(lane, j, 0, 0);
            b[j] = x != 0.0f ? x : probe_value(lane, j, 0, 1);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                typedef typename std::conditional<KIND == 1, _Float16, __bf16>::type E;
                a[j][e] = (E)(x != 0.0f ? x : probe_value(lane, j, e, 0));
                b[j][e] = (E)(x != 0.0f ? x : probe_value(lane, j, e, 1));
            }
        }
    }
    f32x16 c[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) c[j][i] = 0.0f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            if constexpr (KIND == 2)
                c[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], b[j], c[j], 0, 0, 0);
            else if constexpr (KIND == 1)
                c[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[j], b[j], c[j], 0, 0, 0);
            else
                c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[j], c[j], 0, 0, 0);
        }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) s += c[j][i];
    out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_peak_fma(int iters, T x, T y,
                                                       float* __restrict__ out) {
    T a[kFmaChains];
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) a[j] = T(0);
    // unrolled so that the loop's scalar instructions are few against the FMAs
#pragma unroll 8
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < kFmaChains; ++j) a[j] = fma_t(a[j], x, y);
    T s = T(0);
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) s += a[j];
    out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// blocks walk 16 KiB chunks (four 16-byte loads in flight per thread, the
// four consecutive 4 KiB pieces of the chunk), then the tail
__global__ __launch_bounds__(kThreads) void k_peak_copy(const float4* __restrict__ src,
                                                        float4* __restrict__ dst, int64_t n4) {
    constexpr int64_t kChunk = 4 * kThreads;
    const int64_t nchunk = n4 / kChunk;
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int64_t i = c * kChunk + threadIdx.x;
        const float4 v0 = src[i], v1 = src[i + kThreads], v2 = src[i + 2 * kThreads],
                     v3 = src[i + 3 * kThreads];
        dst[i] = v0;
        dst[i + kThreads] = v1;
        dst[i + 2 * kThreads] = v2;
        dst[i + 3 * kThreads] = v3;
    }
    for (int64_t i = nchunk * kChunk + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

}  // namespace

extern "C" int qrfs_peak_blocks(int kind, int64_t* blocks) {
    if (!blocks) return -1;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -3;
    hipError_t e;
    switch (kind) {
        case QRFS_PEAK_MFMA_BF16:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_mfma<0>, kThreads, 0);
            break;
        case QRFS_PEAK_MFMA_FP16:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_mfma<1>, kThreads, 0);
            break;
        case QRFS_PEAK_MFMA_F32:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_mfma<2>, kThreads, 0);
            break;
        case QRFS_PEAK_VALU_F32:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_fma<float>, kThreads, 0);
            break;
        case QRFS_PEAK_VALU_F64:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_fma<double>, kThreads, 0);
            break;
        case QRFS_PEAK_HBM_COPY:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_peak_copy, kThreads, 0);
            break;
        default:
            return -1;
    }
    if (e != hipSuccess || per < 1) return -3;
    *blocks = (int64_t)cus * per;
    return 0;
}

extern "C" int qrfs_peak_launch(int kind, int64_t blocks, int32_t iters, float x, float y,
                                float* out, const float* src, float* dst, int64_t n,
                                double* work, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    // blocks x 256 work-items must fit in 32 bits
    if (!work || blocks < 1 || blocks >= (int64_t)1 << 24) return -1;
    const dim3 grid((unsigned)blocks), block(kThreads);
    const double lanes = (double)blocks * kThreads;
    const double waves = (double)blocks * (kThreads / 64);
    if (kind == QRFS_PEAK_HBM_COPY) {
        if (!src || !dst || n < 4 || n % 4 != 0) return -1;
        hipLaunchKernelGGL(k_peak_copy, grid, block, 0, st, (const float4*)src, (float4*)dst,
                           n / 4);
        *work = 8.0 * (double)n;  // 4 B read + 4 B written per float
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    if (!out || iters < 0) return -1;
    switch (kind) {
        case QRFS_PEAK_MFMA_BF16:
            hipLaunchKernelGGL(k_peak_mfma<0>, grid, block, 0, st, (int)iters, x, out);
            *work = waves * iters * kChains * (2.0 * 32 * 32 * 16);
            break;
        case QRFS_PEAK_MFMA_FP16:
            hipLaunchKernelGGL(k_peak_mfma<1>, grid, block, 0, st, (int)iters, x, out);
            *work = waves * iters * kChains * (2.0 * 32 * 32 * 16);
            break;
        case QRFS_PEAK_MFMA_F32:
            hipLaunchKernelGGL(k_peak_mfma<2>, grid, block, 0, st, (int)iters, x, out);
            *work = waves * iters * kChains * (2.0 * 32 * 32 * 2);
            break;
        case QRFS_PEAK_VALU_F32:
            hipLaunchKernelGGL(k_peak_fma<float>, grid, block, 0, st, (int)iters, x, y, out);
            *work = lanes * iters * kFmaChains * 2.0;
            break;
        case QRFS_PEAK_VALU_F64:
            hipLaunchKernelGGL(k_peak_fma<double>, grid, block, 0, st, (int)iters, (double)x,
                               (double)y, out);
            *work = lanes * iters * kFmaChains * 2.0;
            break;
        default:
            return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
