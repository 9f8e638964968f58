// qrfs_measures.hip -- the noise-free differential-piston structure
// function of each frequency set: its sampling error alone, on which the
// samplers of Sec. 3.1-3.2 are compared.
#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"

namespace qrfs {

// Block s (one set), 256 threads over its frequencies: for each baseline b
// the sum over k of w_k^2 2 (1 - cos 2 pi f_k.B_b), formed as
// w^2 4 sin^2(pi r) with r = f.B reduced to [-1/2, 1/2] in FP64, in
// registers for 8 baselines at a time, then a fixed tree over the threads.
constexpr int SS_THREADS = 256;
constexpr int SS_NB = 8;

__global__ __launch_bounds__(SS_THREADS) void k_set_sf(const double* __restrict__ fx,
                                                       const double* __restrict__ fy,
                                                       const double* __restrict__ w, int64_t K,
                                                       int64_t nB, const double* __restrict__ bx,
                                                       const double* __restrict__ by,
                                                       double* __restrict__ S) {
    __shared__ double red[SS_NB][SS_THREADS];
    const int t = threadIdx.x;
    const int64_t s = blockIdx.x;
    const double* px = fx + s * K;
    const double* py = fy + s * K;
    const double* pw = w + s * K;
    for (int64_t b0 = 0; b0 < nB; b0 += SS_NB) {
        const int nb = nB - b0 < SS_NB ? (int)(nB - b0) : SS_NB;
        double acc[SS_NB];
        double cbx[SS_NB], cby[SS_NB];
#pragma unroll
        for (int q = 0; q < SS_NB; ++q) {
            acc[q] = 0.0;
            cbx[q] = q < nb ? bx[b0 + q] : 0.0;
            cby[q] = q < nb ? by[b0 + q] : 0.0;
        }
        for (int64_t k = t; k < K; k += SS_THREADS) {
            const double f0 = px[k], f1 = py[k], w2 = pw[k] * pw[k];
#pragma unroll
            for (int q = 0; q < SS_NB; ++q) {
                const double r = frac_centered(f0 * cbx[q] + f1 * cby[q]);
                double sh, ch;
                sincos2pi_reduced(0.5 * r, sh, ch);
                acc[q] += w2 * 4.0 * sh * sh;
            }
        }
#pragma unroll
        for (int q = 0; q < SS_NB; ++q) red[q][t] = acc[q];
        __syncthreads();
        for (int h = SS_THREADS / 2; h > 0; h >>= 1) {
            if (t < h) {
#pragma unroll
                for (int q = 0; q < SS_NB; ++q) red[q][t] += red[q][t + h];
            }
            __syncthreads();
        }
        if (t < nb) S[s * nB + b0 + t] = red[t][0];
        __syncthreads();
    }
}


hipError_t launch_set_sf(int64_t n_sets, int64_t K, const double* fx, const double* fy,
                         const double* w, int64_t nB, const double* bx, const double* by,
                         double* S, hipStream_t st) {
    hipLaunchKernelGGL(k_set_sf, dim3((unsigned)n_sets), dim3(SS_THREADS), 0, st, fx, fy, w, K, nB,
                       bx, by, S);
    return hipGetLastError();
}

}  // namespace qrfs
