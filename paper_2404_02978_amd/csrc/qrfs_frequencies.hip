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
// The log-polar map of a unit-square point: |f| = fmin e^(lr u_x) =
// fmin 2^(lr log2(e) u_x), angle 2 pi u_y (u_y in [0, 1), reduced exactly),
// cell area 2 pi lr f^2 / K = acoef f^2.
__device__ __forceinline__ void logpolar_map(double ux, double uy, double fmin, double lr,
                                             double acoef, double& fx, double& fy, double& area) {
#pragma clang fp contract(off)
    double f = fmin * exp2_poly(lr * 1.4426950408889634 * ux);
    double s, c;
    sincos2pi_reduced(uy - rint(uy), s, c);
    fx = f * c;
    fy = f * s;
    area = acoef * f * f;
}

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
        logpolar_map(ux, uy, fmin, lr, acoef, fx, fy, area);
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
// hardware log2 / exp2 (relative error ~5e-7); two binary64 Newton steps on
// y^12 r^11 = 1, y <- y (1 + (1 - y^12 r^11) / 12), each squaring the
// relative error (to ~2e-12, then within ~3e-16 of the exact power of the
// rational exponent); rescaled by 2^(-11k).
__device__ __forceinline__ double pow_m11_12(double q) {
    const int e = ilogb(q);
    const int k = (e + 6 + 1200) / 12 - 100;  // floor((e + 6) / 12)
    const double r = ldexp(q, -12 * k);
    const float rf = (float)r;
    double y = (double)__builtin_amdgcn_exp2f(-0.9166666865f * __builtin_amdgcn_logf(rf));
    const double r2 = r * r, r4 = r2 * r2, r11 = (r4 * r4) * (r2 * r);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y2 = y * y, y4 = y2 * y2;
        const double t = ((y4 * y4) * y4) * r11;
        y = fma(y, (1.0 - t) * (1.0 / 12.0), y);
    }
    return ldexp(y, -11 * k);
}

// q^(-11/12) to binary32 accuracy (~1e-7), for weights that feed binary32
// sums: the range reduction of pow_m11_12 (exact), its binary32 estimate,
// and one Newton step carried out in binary32 (r^11 and y^12 with r in
// [2^-6, 2^6) stay inside the binary32 range).
__device__ __forceinline__ double pow_m11_12_f32(double q) {
    const int e = ilogb(q);
    const int k = (e + 6 + 1200) / 12 - 100;  // floor((e + 6) / 12)
    const float r = (float)ldexp(q, -12 * k);
    float y = __builtin_amdgcn_exp2f(-0.9166666865f * __builtin_amdgcn_logf(r));
    const float r2 = r * r, r4 = r2 * r2, r11 = (r4 * r4) * (r2 * r);
    const float y2 = y * y, y4 = y2 * y2;
    const float t = ((y4 * y4) * y4) * r11;
    y = fmaf(y, (1.0f - t) * (1.0f / 12.0f), y);
    return ldexp((double)y, -11 * k);
}

// F32: weights that feed binary32 sums (FP32-class precisions), every
// factor to binary32 accuracy: the PSD power to ~1e-7, the square roots to
// ~1e-14, the filter by j1x_pi_f32 (absolute error ~3e-8 of the unfiltered
// weight); otherwise every step in binary64.
template <bool F32>
__device__ __forceinline__ double weight_one(int model, double c, double r0_m53, double inv_L02,
                                             int has_ap, double D, double d, double x, double y,
                                             double area) {
#pragma clang fp contract(off)
    const double f2 = x * x + y * y;
    const double q = f2 + (model == 1 ? inv_L02 : 0.0);
    const double ca = c * r0_m53 * area;
    double v = 0.0;
    if (q != 0.0) v = F32 ? pow_m11_12_f32(q) * sqrt_f32_nr(ca) : pow_m11_12(q) * sqrt_nr(ca);
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

// Log-polar R2 sets in lane order.  The aperture filter's J1 switches form at
// pi D |f| = 8, and |f| grows with u_x, but consecutive R2 points spread u_x
// over [0, 1), so almost every wave of k_sample_weights runs both forms.
// Points LP_Q = 12096 indices apart differ by 2.5e-4 in u_x (mod 1), so
// here the 64 lanes of a wave take indices LP_Q apart and a wave's u_x span
// 0.016: only the waves at the switch, or where u_x wraps, run both forms.
// A block is 16 waves at 16 consecutive offsets; for every lane they cover
// 16 consecutive indices (one 128-byte line of each output), which go out
// through LDS as whole lines.  Every value is the one k_sample_weights
// gives for the same index (the same device functions).
constexpr int LP_WAVES = 16;
constexpr int64_t LP_Q = 12096;                            // a multiple of LP_WAVES
constexpr int64_t LP_TILE = 64 * LP_Q;                     // indices per tile
constexpr int64_t LP_BLOCKS_PER_TILE = LP_Q / LP_WAVES;   // 756

template <bool F32>
__global__ __launch_bounds__(64 * LP_WAVES) void k_sample_weights_lp(
    uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n, double fmin, double lr, double acoef,
    int model, double c, double r0_m53, double inv_L02, int has_ap, double D, double d,
    double* __restrict__ fx, double* __restrict__ fy, double* __restrict__ w) {
    __shared__ double st[3][LP_WAVES][65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = blockIdx.x / LP_BLOCKS_PER_TILE;
    const int64_t first = tile * LP_TILE + (blockIdx.x % LP_BLOCKS_PER_TILE) * LP_WAVES;
    const uint32_t m = (uint32_t)wave + (uint32_t)lane * (uint32_t)LP_Q;  // index - first
    if (first + (int64_t)m < n) {
        // R2 point index + 1 + first + m: the block's state plus m increments
        const uint64_t nb = index + 1u + (uint64_t)first;
        uint64_t ubx = s0x + nb * kR2IncX, uby = s0y + nb * kR2IncY;
        // kept in scalar registers: the sums below must not be reassociated
        // into a per-lane 64 x 64-bit product
        asm volatile("" : "+s"(ubx), "+s"(uby));
        const double ux = r2_coord(ubx + (uint64_t)m * kR2IncX);
        const double uy = r2_coord(uby + (uint64_t)m * kR2IncY);
        double x, y, ar;
        logpolar_map(ux, uy, fmin, lr, acoef, x, y, ar);
        st[0][wave][lane] = x;
        st[1][wave][lane] = y;
        st[2][wave][lane] = weight_one<F32>(model, c, r0_m53, inv_L02, has_ap, D, d, x, y, ar);
    }
    __syncthreads();
    // thread t writes offset (t mod 16) of lane t / 16's run: each wave
    // stores four whole lines per array
    const int o = tid & (LP_WAVES - 1), l = tid >> 4;
    const int64_t i = first + o + (int64_t)l * LP_Q;
    if (i < n) {
        fx[i] = st[0][o][l];
        fy[i] = st[1][o][l];
        w[i] = st[2][o][l];
    }
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
    if (scheme == 1 && has_ap && !f32 && n >= 32 * LP_TILE) {
        // lane order pays once the partly filled last tile is a small share;
        // it shortens the binary64 filter (about 14 %), but not the
        // FP32-class one, whose two forms are short
        hipLaunchKernelGGL(k_sample_weights_lp<false>, dim3((unsigned)(cdiv(n, LP_TILE) * LP_BLOCKS_PER_TILE)),
                           dim3(64 * LP_WAVES), 0, st, s0x, s0y, index, n, fmin, lr,
                           area_coef(scheme, K, L, lr), model, c, r0_m53, inv_L02, has_ap, D, d,
                           fx, fy, w);
        return hipGetLastError();
    }
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
