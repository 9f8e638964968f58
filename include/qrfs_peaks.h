/*
 * qrfs_peaks.h -- C ABI of libqrfs_peaks, throughput probes for the roofline
 * denominators of the MI355X build.
 *
 * The rooflines of the kernels in libqrfs are quoted against the vendor's
 * nominal peaks (dense MFMA bf16 / fp16 2.5 PFLOP/s, FP32 MFMA 157.3 TFLOP/s,
 * FP32 and FP64 vector FMA 78.6 TFLOP/s unpacked, HBM 8 TB/s).  These probes
 * measure what the device at hand sustains for the same instruction classes,
 * so that a kernel can also be placed against a measured ceiling: the clock
 * a busy MI355X holds is below its nominal 2.4 GHz.  They are measuring
 * instruments, not part of the method of the paper.
 *
 * Conventions: pointers are DEVICE pointers owned by the caller; work is
 * enqueued on `stream` (a hipStream_t passed as void*, NULL = the null
 * stream); the caller times the launch (for example with events on that
 * stream).  Returns 0, or -1 on a bad argument (nothing enqueued), or -3 on
 * a launch error.
 */
#ifndef QRFS_PEAKS_H
#define QRFS_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define QRFS_PEAKS_API __attribute__((visibility("default")))
#else
#define QRFS_PEAKS_API
#endif

/* Probe kinds.
 *   MFMA_*: every wave of 256-thread blocks runs `iters` rounds of four
 *     independent 32x32 MFMA accumulations (v_mfma_f32_32x32x16_bf16,
 *     _f16, or v_mfma_f32_32x32x2f32); out[thread] = sum of the thread's 64
 *     accumulator values.  With x != 0 both operands equal x and out is
 *     64 * iters * Kd * x^2 (x rounded to the operand type, Kd = 16 for
 *     bf16 and fp16, 2 for FP32).  With x = 0 every chain multiplies its own
 *     varied operands (multiples of 1/16 in [-1, 1), exact products and
 *     sums), so out is iters times its value for one round: the matrix
 *     cores see changing data, as in a real contraction.
 *   VALU_*: every thread runs `iters` rounds of 8 independent fused
 *     multiply-adds a = a*x + y (binary32 or binary64, unpacked) from a = 0;
 *     out[thread] = sum of the 8 values (binary32).
 *   HBM_COPY: dst[i] = src[i] for i < n (n floats, n a multiple of 4),
 *     grid-stride, 16-byte accesses; iters, x, y and out unused. */
#define QRFS_PEAK_MFMA_BF16 0
#define QRFS_PEAK_MFMA_FP16 1
#define QRFS_PEAK_MFMA_F32 2
#define QRFS_PEAK_VALU_F32 3
#define QRFS_PEAK_VALU_F64 4
#define QRFS_PEAK_HBM_COPY 5

/* *blocks = the number of 256-thread blocks of `kind` the current device
 * keeps resident at once (compute units x resident blocks per unit): one
 * launch of that many blocks fills the device in a single round. */
QRFS_PEAKS_API int qrfs_peak_blocks(int kind, int64_t* blocks);

/* Launches one probe of `kind` with `blocks` blocks of 256 threads
 * (1 <= blocks < 2^24; out holds blocks * 256 floats).  *work receives the launch's nominal work:
 * flops for the MFMA and VALU kinds (2 per multiply-add), bytes moved
 * (read + written) for HBM_COPY. */
QRFS_PEAKS_API int qrfs_peak_launch(int kind, int64_t blocks, int32_t iters, float x, float y,
                                    float* out, const float* src, float* dst, int64_t n,
                                    double* work, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QRFS_PEAKS_H */
