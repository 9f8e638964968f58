// qrfs_temporal.hip -- frozen-flow temporal structure function of the
// differential piston (the statistical test of Sec. 4.4): aperture centres
// moved by the wind, and the time-lag estimator over piston time series.
#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"

namespace qrfs {

// Points 0 .. M-1: c1 - v t_m, points M .. 2M-1: c2 - v t_m, t_m = m dt
// (Taylor: at time t the telescope at c sees the screen at c - v t).
__global__ void k_taylor_points(double c1x, double c1y, double c2x, double c2y, double vx,
                                double vy, double dt, int64_t M, double* __restrict__ px,
                                double* __restrict__ py) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * M) return;
    const bool second = i >= M;
    const double t = (double)(second ? i - M : i) * dt;
    px[i] = (second ? c2x : c1x) - vx * t;
    py[i] = (second ? c2y : c1y) - vy * t;
}

constexpr int TS_THREADS = 256;
constexpr int TS_MAXJ = TEMPORAL_MAX_M / TS_THREADS;  // lags per thread

// Block b: realisations [b RB, (b+1) RB).  For each, the differential
// piston dp[m] = p1[m] - p2[m] goes to LDS; thread t owns lags
// j = t + 256 i and adds the realisation's mean over pairs of
// (dp[m + j] - dp[m])^2 and its square to registers.  Writes
// part[b][j][0..1]; the fixed-order reduction over blocks gives the mean
// over realisations and its standard error.
template <typename T>
__global__ __launch_bounds__(TS_THREADS) void k_temporal_rows(const T* __restrict__ pist,
                                                              int64_t R, int64_t M, int64_t RB,
                                                              double* __restrict__ part) {
    __shared__ double dp[TEMPORAL_MAX_M];
    double s1[TS_MAXJ], s2[TS_MAXJ];
#pragma unroll
    for (int i = 0; i < TS_MAXJ; ++i) s1[i] = s2[i] = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int64_t r1 = r0 + RB < R ? r0 + RB : R;
    for (int64_t r = r0; r < r1; ++r) {
        const T* p1 = pist + r * 2 * M;
        const T* p2 = p1 + M;
        for (int64_t m = threadIdx.x; m < M; m += TS_THREADS)
            dp[m] = (double)p1[m] - (double)p2[m];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TS_MAXJ; ++i) {
            const int64_t j = threadIdx.x + (int64_t)TS_THREADS * i;
            if (j >= 1 && j < M) {
                double acc = 0.0;
                for (int64_t m = 0; m + j < M; ++m) {
                    const double d = dp[m + j] - dp[m];
                    acc += d * d;
                }
                const double v = acc / (double)(M - j);
                s1[i] += v;
                s2[i] += v * v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TS_MAXJ; ++i) {
        const int64_t j = threadIdx.x + (int64_t)TS_THREADS * i;
        if (j < M) {
            part[((int64_t)blockIdx.x * M + j) * 2] = s1[i];
            part[((int64_t)blockIdx.x * M + j) * 2 + 1] = s2[i];
        }
    }
}

static inline int64_t tcdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_taylor_points(const double c1[2], const double c2[2], const double v[2],
                                double dt, int64_t M, double* px, double* py, hipStream_t st) {
    hipLaunchKernelGGL(k_taylor_points, dim3((unsigned)tcdiv(2 * M, 256)), dim3(256), 0, st,
                       c1[0], c1[1], c2[0], c2[1], v[0], v[1], dt, M, px, py);
    return hipGetLastError();
}

int64_t temporal_blocks(int64_t R) { return tcdiv(R, TEMPORAL_ROWS_PER_BLOCK); }

hipError_t launch_temporal_rows(bool fp64, const void* pist, int64_t R, int64_t M, double* part,
                                hipStream_t st) {
    const dim3 g((unsigned)temporal_blocks(R));
    if (fp64)
        hipLaunchKernelGGL((k_temporal_rows<double>), g, dim3(TS_THREADS), 0, st,
                           (const double*)pist, R, M, (int64_t)TEMPORAL_ROWS_PER_BLOCK, part);
    else
        hipLaunchKernelGGL((k_temporal_rows<float>), g, dim3(TS_THREADS), 0, st,
                           (const float*)pist, R, M, (int64_t)TEMPORAL_ROWS_PER_BLOCK, part);
    return hipGetLastError();
}

}  // namespace qrfs
