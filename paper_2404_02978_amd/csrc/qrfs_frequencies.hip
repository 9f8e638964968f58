// qrfs_frequencies.hip -- gfx950 kernels that produce a frequency set: the
// samplers (R2, pseudo-random and jittered placements with their maps and
// cell areas) and the PSD / aperture-filter weights of Eq. 3.
#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"

namespace qrfs {

// ------------------------------------------------------------- sampler ----
// Frequency i of a launch.  Point n = index + 1 + i of the R2 sequence
// (Sec. 3.2, Eq. 6) for schemes 0, 1, 3, of the pseudo-random stream for
// schemes 4-7 (the randomised samplers of Sec. 3.1), mapped by Eq. 5
// (Cartesian: schemes 0, 5), the log-polar map (1, 6), the square-to-disc
// map (3, 7), or placed in its cell of the jittered grid of Eq. 4 (4).
__device__ __forceinline__ void sample_one(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index,
                                           int64_t i, int64_t K, int32_t N, double df, double L,
                                           double fmin, double lr, double acoef, double& fx,
                                           double& fy, double& area) {
    // no fused multiply-adds here or in weight_one: the values then do not
    // depend on the kernel they are inlined into
#pragma clang fp contract(off)
    double ux, uy;
    if (scheme >= 4)
        pseudo_point(s0x, s0y, index + 1u + (uint64_t)i, ux, uy);
    else
        r2_point(s0x, s0y, index + 1u + (uint64_t)i, ux, uy);
    const int map = scheme >= 5 ? (scheme == 7 ? 3 : scheme - 5) : scheme;
    if (map == 0) {
        fx = L * (ux - 0.5);
        fy = L * (uy - 0.5);
        area = acoef;  // L^2 / K
    } else if (map == 4) {
        // Eq. 4: point k = iy N + ix of a set (K = N^2) at its cell's lower
        // corner -N df / 2 + i df plus the jitter u df, as df (i + u - N/2)
        // (no product feeds a sum, so nothing is fused)
        const int64_t k = i % K;
        const double ix = (double)(k % N), iy = (double)(k / N);
        const double h = 0.5 * (double)N;
        fx = df * (ix + ux - h);
        fy = df * (iy + uy - h);
        area = df * df;
    } else if (map == 3) {
        // polar quasi-random frequencies (Sec. 3.2): concentric square-to-
        // disc map of the point, disc radius L, equal cell areas
        const double a = 2.0 * ux - 1.0, b = 2.0 * uy - 1.0;
        double rad = 0.0, ang = 0.0;  // angle in half-turns
        if (fabs(a) > fabs(b)) {
            rad = a;
            ang = 0.25 * (b / a);
        } else if (b != 0.0) {
            rad = b;
            ang = 0.5 - 0.25 * (a / b);
        }
        double s, c;
        sincospi(ang, &s, &c);
        fx = L * rad * c;
        fy = L * rad * s;
        area = acoef;  // pi L^2 / K
    } else {
        // |f| = fmin e^(lr u_x) = fmin 2^(lr log2(e) u_x), angle 2 pi u_y
        // (u_y in [0, 1), reduced exactly)
        double f = fmin * exp2_poly(lr * 1.4426950408889634 * ux);
        double s, c;
        sincos2pi_reduced(uy - rint(uy), s, c);
        fx = f * c;
        fy = f * s;
        area = acoef * f * f;  // 2 pi lr f^2 / K
    }
}

__global__ void k_sample(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n,
                         int64_t K, int32_t N, double df, double L, double fmin, double lr,
                         double acoef, double* __restrict__ fx, double* __restrict__ fy,
                         double* __restrict__ area) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x, y, ar;
    sample_one(scheme, s0x, s0y, index, i, K, N, df, L, fmin, lr, acoef, x, y, ar);
    fx[i] = x;
    fy[i] = y;
    area[i] = ar;
}

// ------------------------------------------------------------- weights ----
// w = sqrt(W(|f|) area) [x F(|f|)], the amplitude of Eq. 3 (Eq. 7 filter),
// with W = c r0^-5/3 q^-11/6, q = |f|^2 (+ L0^-2): evaluated as
// q^-11/12 sqrt(c r0^-5/3 area), the power by pow_m11_12 (no general pow,
// one square root fewer).
// q^(-11/12) for q > 0 (the square root of the PSD's q^(-11/6)): q = 2^(12k) r
// exactly with r in [2^-6, 2^6); a binary32 estimate of r^(-11/12) from the
// hardware log2 / exp2 (relative error ~5e-7); STEPS binary64 Newton steps
// on y^12 r^11 = 1, y <- y (1 + (1 - y^12 r^11) / 12), each squaring the
// relative error (one step: ~2e-12; two: within ~3e-16 of the exact power of
// the rational exponent); rescaled by 2^(-11k).
template <int STEPS>
__device__ __forceinline__ double pow_m11_12(double q) {
    const int e = ilogb(q);
    const int k = (e + 6 + 1200) / 12 - 100;  // floor((e + 6) / 12)
    const double r = ldexp(q, -12 * k);
    const float rf = (float)r;
    double y = (double)__builtin_amdgcn_exp2f(-0.9166666865f * __builtin_amdgcn_logf(rf));
    const double r2 = r * r, r4 = r2 * r2, r11 = (r4 * r4) * (r2 * r);
#pragma unroll
    for (int it = 0; it < STEPS; ++it) {
        const double y2 = y * y, y4 = y2 * y2;
        const double t = ((y4 * y4) * y4) * r11;
        y = fma(y, (1.0 - t) * (1.0 / 12.0), y);
    }
    return ldexp(y, -11 * k);
}

// F32: weights that feed binary32 sums (FP32-class precisions): the PSD
// power to ~2e-12 and the filter by j1x_pi_f32 (absolute error ~1e-8 of the
// unfiltered weight); otherwise every step in binary64.
template <bool F32>
__device__ __forceinline__ double weight_one(int model, double c, double r0_m53, double inv_L02,
                                             int has_ap, double D, double d, double x, double y,
                                             double area) {
#pragma clang fp contract(off)
    const double f2 = x * x + y * y;
    const double q = f2 + (model == 1 ? inv_L02 : 0.0);
    double v = q == 0.0 ? 0.0 : pow_m11_12<F32 ? 1 : 2>(q) * sqrt_nr(c * r0_m53 * area);
    if (has_ap)
        v *= F32 ? (double)aperture_filter_f32(D, d, sqrt_f32_nr(f2))
                 : aperture_filter(D, d, sqrt_nr(f2));
    return v;
}

template <bool F32>
__global__ void k_weights(int model, double c, double r0_m53, double inv_L02, int has_ap,
                          double D, double d, int64_t n, const double* __restrict__ fx,
                          const double* __restrict__ fy, const double* __restrict__ area,
                          double* __restrict__ w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    w[i] = weight_one<F32>(model, c, r0_m53, inv_L02, has_ap, D, d, fx[i], fy[i], area[i]);
}

// Both in one pass, for pipelines that need the weights but not the cell
// areas: the same values as k_sample followed by k_weights, without writing
// and re-reading the areas and the frequencies.
template <bool F32>
__global__ void k_sample_weights(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index,
                                 int64_t n, int64_t K, int32_t N, double df, double L,
                                 double fmin, double lr, double acoef, int model, double c,
                                 double r0_m53,
                                 double inv_L02, int has_ap, double D, double d,
                                 double* __restrict__ fx, double* __restrict__ fy,
                                 double* __restrict__ w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x, y, ar;
    sample_one(scheme, s0x, s0y, index, i, K, N, df, L, fmin, lr, acoef, x, y, ar);
    fx[i] = x;
    fy[i] = y;
    w[i] = weight_one<F32>(model, c, r0_m53, inv_L02, has_ap, D, d, x, y, ar);
}

// ----------------------------------------------------------- launchers ----
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The cell area of a set's points, or its factor: L^2 / K (Cartesian),
// pi L^2 / K (disc), 2 pi ln(fmax/fmin) / K times f^2 (log-polar); the
// jittered grid uses df^2.
static double area_coef(int scheme, int64_t K, double L, double lr) {
    const int map = scheme >= 5 ? (scheme == 7 ? 3 : scheme - 5) : scheme;
    const double pi = 3.141592653589793;
    if (map == 0) return L * L / (double)K;
    if (map == 3) return pi * L * L / (double)K;
    if (map == 1) return 2.0 * pi * lr / (double)K;
    return 0.0;
}

hipError_t launch_sample(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_sets,
                         int64_t K, int32_t N, double df, double fmin, double fmax, double* fx,
                         double* fy, double* area, hipStream_t st) {
    int64_t n = n_sets * K;
    double L = (scheme == 3 || scheme == 7) ? fmax : (double)N * df;
    double lr = (scheme == 1 || scheme == 6) ? log(fmax / fmin) : 0.0;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, scheme, s0x, s0y,
                       index, n, K, N, df, L, fmin, lr, area_coef(scheme, K, L, lr), fx, fy, area);
    return hipGetLastError();
}

hipError_t launch_sample_weights(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index,
                                 int64_t n_sets, int64_t K, int32_t N, double df, double fmin,
                                 double fmax, int model, double c, double r0, double L0,
                                 int has_ap, double D, double d, int f32, double* fx,
                                 double* fy, double* w, hipStream_t st) {
    int64_t n = n_sets * K;
    double L = (scheme == 3 || scheme == 7) ? fmax : (double)N * df;
    double lr = (scheme == 1 || scheme == 6) ? log(fmax / fmin) : 0.0;
    double r0_m53 = pow(r0, -5.0 / 3.0);
    double inv_L02 = model == 1 ? 1.0 / (L0 * L0) : 0.0;
    auto kern = f32 ? k_sample_weights<true> : k_sample_weights<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, scheme, s0x, s0y,
                       index, n, K, N, df, L, fmin, lr, area_coef(scheme, K, L, lr), model, c,
                       r0_m53, inv_L02, has_ap, D, d, fx, fy, w);
    return hipGetLastError();
}

hipError_t launch_weights(int model, double c, double r0, double L0, int has_ap, double D,
                          double d, int f32, int64_t n, const double* fx, const double* fy,
                          const double* area, double* w, hipStream_t st) {
    double r0_m53 = pow(r0, -5.0 / 3.0);
    double inv_L02 = model == 1 ? 1.0 / (L0 * L0) : 0.0;
    auto kern = f32 ? k_weights<true> : k_weights<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, model, c, r0_m53,
                       inv_L02, has_ap, D, d, n, fx, fy, area, w);
    return hipGetLastError();
}

}  // namespace qrfs
