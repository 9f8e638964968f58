/*
 * qrfs_oracle.c -- plain FP64 CPU oracle for quasi-random frequency sampling
 * (Berdja, Hadjara, Carbillet, Bernardi, Petrov, "Quasi-Random Frequency
 * Sampling for Optical Turbulence Simulations", arXiv 2404.02978).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP path: every constant below is
 * derived here from its definition.
 *
 * Everything is evaluated in double precision with straightforward loops in
 * the order the paper states the method; OpenMP only splits independent
 * realisations across threads (no reordering inside one result).
 *
 * Readings of the paper that this file encodes (each is also listed in the
 * design notes of the repository):
 *   - R2 sequence (Sec. 3.2, Eq. 6) is kept as an exact 64-bit fixed-point
 *     Weyl sequence U_n = S0 + n*A mod 2^64, A = round(2^64 * alpha); the
 *     state is updated before it is used, so point n = index+1 is the first.
 *   - Cartesian map (Eq. 5): f = delta_f * N * (u - 1/2), i.e. the domain
 *     width N*delta_f equals 2 max(f) (worked example of Sec. 4.4: 0.25/22
 *     and 0.25 give N = 44).
 *   - Coefficients: a_rk, b_rk ~ N(0,1) iid multiply cos and sin of the
 *     harmonic (the two independent normals of Eq. 2); Eq. 3's literal form
 *     (one normal amplitude, one uniform phase, factor 2/sqrt 2) is mode 1.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the
 *     64-bit seed, counter (block, realisation lo, realisation hi, 0);
 *     uniforms ((x >> 9) + 1/2) 2^-23 (exactly representable in binary32
 *     as well as binary64); Box-Muller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* R2 low-discrepancy sequence, Sec. 3.2 Eq. 6                          */
/* ------------------------------------------------------------------ */

/* Plastic number psi: the real root of x^3 = x + 1 (Sec. 3.2), found by
 * Newton's method in binary128 so that 2^64/psi and 2^64/psi^2 can be
 * rounded to integers exactly. */
static __float128 plastic_number_q(void) {
    __float128 x = 1.3Q;
    for (int it = 0; it < 200; ++it) {
        __float128 fx = x * x * x - x - 1.0Q;
        __float128 dfx = 3.0Q * x * x - 1.0Q;
        __float128 nx = x - fx / dfx;
        if (nx == x) break;
        x = nx;
    }
    return x;
}

static uint64_t round_frac_to_u64(__float128 a) {
    /* a in (0,1): returns round(a * 2^64) */
    const __float128 two64 = 18446744073709551616.0Q;
    __float128 v = a * two64 + 0.5Q;
    /* split to avoid relying on a 128-bit -> u64 conversion near 2^64 */
    __float128 hi = (__float128)(uint64_t)(v / 4294967296.0Q);
    __float128 lo = v - hi * 4294967296.0Q;
    return ((uint64_t)hi << 32) + (uint64_t)lo;
}

ORACLE_API void oracle_plastic_number(double* psi) { *psi = (double)plastic_number_q(); }

/* increments A_x = round(2^64 / psi), A_y = round(2^64 / psi^2) */
ORACLE_API void oracle_r2_increments(uint64_t out[2]) {
    __float128 psi = plastic_number_q();
    out[0] = round_frac_to_u64(1.0Q / psi);
    out[1] = round_frac_to_u64(1.0Q / (psi * psi));
}

/* u_n = frac(s0 + n alpha) for n = index+1 .. index+n_pts, returned in [0,1)
 * with 53 significant bits (the top 53 bits of the 64-bit state). */
ORACLE_API void oracle_r2_points(uint64_t s0x, uint64_t s0y, uint64_t index,
                                 int64_t n_pts, double* ux, double* uy) {
    uint64_t inc[2];
    oracle_r2_increments(inc);
    for (int64_t i = 0; i < n_pts; ++i) {
        uint64_t n = index + 1u + (uint64_t)i;
        uint64_t Ux = s0x + n * inc[0];
        uint64_t Uy = s0y + n * inc[1];
        ux[i] = (double)(Ux >> 11) * 0x1p-53;
        uy[i] = (double)(Uy >> 11) * 0x1p-53;
    }
}

/* ------------------------------------------------------------------ */
/* Frequency maps                                                      */
/* ------------------------------------------------------------------ */

/* Maps of unit-square points (ux, uy) to frequencies (map 0: Cartesian,
 * 1: log-polar, 3: disc), K points per set.
 *
 * Cartesian, Eq. 5 with delta_f_x = delta_f_y = df and n_x = n_y = N
 * (Sec. 3.2): f = df*N*(u - 1/2).  Each of the K points of a set stands for
 * an equal share (N df)^2 / K of the square domain (delta_f^2 when
 * K = N^2, Eq. 3).
 *
 * Log-polar: ln|f| uniform on [ln fmin, ln fmax] from the first coordinate,
 * angle 2 pi u from the second.  The (ln f, theta) box has measure
 * 2 pi ln(fmax/fmin); its Jacobian to (fx, fy) is |f|^2, so each of the K
 * points of a set carries area 2 pi ln(fmax/fmin) |f|^2 / K.
 *
 * Disc: polar quasi-random frequencies through the concentric map onto the
 * disc |f| < fmax; every point stands for the same cell area
 * pi fmax^2 / K. */
static void map_points(int32_t map, int64_t n, int64_t K, int32_t N, double df, double fmin,
                       double fmax, const double* ux, const double* uy, double* fx, double* fy,
                       double* area);

ORACLE_API void oracle_sample_cartesian(uint64_t s0x, uint64_t s0y, uint64_t index,
                                        int64_t n_sets, int64_t K, int32_t N, double df,
                                        double* fx, double* fy, double* area) {
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_r2_points(s0x, s0y, index, n, ux, uy);
    map_points(0, n, K, N, df, 0.0, 0.0, ux, uy, fx, fy, area);
    free(ux);
    free(uy);
}

ORACLE_API void oracle_sample_logpolar(uint64_t s0x, uint64_t s0y, uint64_t index,
                                       int64_t n_sets, int64_t K, double fmin, double fmax,
                                       double* fx, double* fy, double* area) {
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_r2_points(s0x, s0y, index, n, ux, uy);
    map_points(1, n, K, 0, 0.0, fmin, fmax, ux, uy, fx, fy, area);
    free(ux);
    free(uy);
}

/* Square-to-disc map for polar quasi-random frequencies (Sec. 3.2 cites
 * Shirley and Chiu's concentric map): (ux, uy) in [0,1)^2 -> (a, b) =
 * (2ux - 1, 2uy - 1); the concentric square max(|a|, |b|) = rho goes to the
 * circle of radius rho, the position along the square's edge to the angle
 * linearly, so the map preserves area (Jacobian pi/4 everywhere). */
ORACLE_API void oracle_concentric_map(double ux, double uy, double* x, double* y) {
    double a = 2.0 * ux - 1.0, b = 2.0 * uy - 1.0;
    double r, phi;
    if (a == 0.0 && b == 0.0) {
        r = 0.0;
        phi = 0.0;
    } else if (fabs(a) > fabs(b)) {
        r = a;
        phi = (M_PI / 4.0) * (b / a);
    } else {
        r = b;
        phi = M_PI / 2.0 - (M_PI / 4.0) * (a / b);
    }
    *x = r * cos(phi);
    *y = r * sin(phi);
}

ORACLE_API void oracle_sample_disc(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_sets,
                                   int64_t K, double fmax, double* fx, double* fy, double* area) {
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_r2_points(s0x, s0y, index, n, ux, uy);
    map_points(3, n, K, 0, 0.0, 0.0, fmax, ux, uy, fx, fy, area);
    free(ux);
    free(uy);
}

static void map_points(int32_t map, int64_t n, int64_t K, int32_t N, double df, double fmin,
                       double fmax, const double* ux, const double* uy, double* fx, double* fy,
                       double* area) {
    if (map == 0) {
        double L = (double)N * df;
        for (int64_t i = 0; i < n; ++i) {
            fx[i] = L * (ux[i] - 0.5);
            fy[i] = L * (uy[i] - 0.5);
            area[i] = L * L / (double)K;
        }
    } else if (map == 1) {
        double lr = log(fmax / fmin);
        for (int64_t i = 0; i < n; ++i) {
            double f = fmin * exp(lr * ux[i]);
            double th = 2.0 * M_PI * uy[i];
            fx[i] = f * cos(th);
            fy[i] = f * sin(th);
            area[i] = 2.0 * M_PI * lr * f * f / (double)K;
        }
    } else {
        for (int64_t i = 0; i < n; ++i) {
            double x, y;
            oracle_concentric_map(ux[i], uy[i], &x, &y);
            fx[i] = fmax * x;
            fy[i] = fmax * y;
            area[i] = M_PI * fmax * fmax / (double)K;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Pseudo-random and jittered frequency sampling (Sec. 3.1, Eq. 4): the  */
/* randomised schemes the quasi-random sampling is set against         */
/* ------------------------------------------------------------------ */

ORACLE_API void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                     uint32_t out[4]);

/* Unit-square point n of the pseudo-random frequency stream: one
 * Philox4x32-10 block keyed by seed_x, counter (n lo, n hi, low word of
 * seed_y, 0x46524551); every coefficient counter ends in a zero word, so
 * the two streams never share a block.  ux is the top 53 bits of words
 * (1:0) times 2^-53, uy the same of words (3:2), the form of the R2 points.
 * Points n = index+1 .. index+n_pts, as for the R2 sequence. */
ORACLE_API void oracle_pseudo_points(uint64_t seed_x, uint64_t seed_y, uint64_t index,
                                     int64_t n_pts, double* ux, double* uy) {
    uint32_t key[2] = {(uint32_t)seed_x, (uint32_t)(seed_x >> 32)};
    for (int64_t i = 0; i < n_pts; ++i) {
        uint64_t n = index + 1u + (uint64_t)i;
        uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), (uint32_t)seed_y, 0x46524551u};
        uint32_t x[4];
        oracle_philox4x32_10(ctr, key, x);
        uint64_t a = ((uint64_t)x[1] << 32) | x[0];
        uint64_t b = ((uint64_t)x[3] << 32) | x[2];
        ux[i] = (double)(a >> 11) * 0x1p-53;
        uy[i] = (double)(b >> 11) * 0x1p-53;
    }
}

/* Fully random frequencies: the pseudo-random points through map 0, 1 or 3
 * (the same maps and cell areas as the quasi-random schemes). */
ORACLE_API void oracle_sample_pseudo(int32_t map, uint64_t seed_x, uint64_t seed_y,
                                     uint64_t index, int64_t n_sets, int64_t K, int32_t N,
                                     double df, double fmin, double fmax, double* fx, double* fy,
                                     double* area) {
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_pseudo_points(seed_x, seed_y, index, n, ux, uy);
    map_points(map, n, K, N, df, fmin, fmax, ux, uy, fx, fy, area);
    free(ux);
    free(uy);
}

/* Randomly jittered grid, Eq. 4: the square of side N df centred on the
 * origin is cut into N x N cells of side df; point k = iy N + ix of a set
 * lies in cell (ix, iy), at its lower corner f' = -N df / 2 + i df plus
 * R_u df, written df (i + R_u - N/2).  One point per cell, so K = N^2 and
 * every point stands for df^2.  R_u: the pseudo-random stream, point
 * n = index + 1 + s K + k for point k of set s. */
ORACLE_API void oracle_sample_jitter(uint64_t seed_x, uint64_t seed_y, uint64_t index,
                                     int64_t n_sets, int32_t N, double df, double* fx,
                                     double* fy, double* area) {
    int64_t K = (int64_t)N * N;
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_pseudo_points(seed_x, seed_y, index, n, ux, uy);
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = i % K;
        double ix = (double)(k % N), iy = (double)(k / N);
        fx[i] = df * (ix + ux[i] - 0.5 * (double)N);
        fy[i] = df * (iy + uy[i] - 0.5 * (double)N);
        area[i] = df * df;
    }
    free(ux);
    free(uy);
}

/* ------------------------------------------------------------------ */
/* Phase PSD and aperture filter, Sec. 4.1 Eq. 7                       */
/* ------------------------------------------------------------------ */

/* Kolmogorov constant of the phase PSD in cycles/m:
 * c = Gamma(11/6)^2 / (2 pi^(11/3)) * (24/5 Gamma(6/5))^(5/6); Eq. 7 prints
 * it rounded to 0.02289. */
ORACLE_API double oracle_psd_constant(void) {
    double g = tgamma(11.0 / 6.0);
    return g * g / (2.0 * pow(M_PI, 11.0 / 3.0)) * pow(24.0 / 5.0 * tgamma(6.0 / 5.0), 5.0 / 6.0);
}

/* model 0: Kolmogorov c r0^(-5/3) f^(-11/3); model 1: von Karman
 * c r0^(-5/3) (f^2 + L0^-2)^(-11/6) (first factor of Eq. 7).  An exact
 * f = 0 has no finite Kolmogorov value and contributes nothing. */
ORACLE_API double oracle_psd(int32_t model, double c, double r0, double L0, double f) {
    double inv_L02 = (model == 1) ? 1.0 / (L0 * L0) : 0.0;
    double q = f * f + inv_L02;
    if (q == 0.0) return 0.0;
    return c * pow(r0, -5.0 / 3.0) * pow(q, -11.0 / 6.0);
}

/* Circular aperture of diameter D with central obstruction d (Eq. 7):
 * F = 2 (D J1(pi D f) - d J1(pi d f)) / (pi (D^2 - d^2) f), F(0) = 1;
 * Eq. 7's factor 4(...)^2 is F^2. */
ORACLE_API double oracle_aperture_filter(double D, double d, double f) {
    if (f == 0.0) return 1.0;
    double num = D * j1(M_PI * D * f);
    if (d > 0.0) num -= d * j1(M_PI * d * f);
    return 2.0 * num / (M_PI * (D * D - d * d) * f);
}

/* w_k = sqrt(W(|f_k|) * area_k) [* F(|f_k|)], the amplitude factor of Eq. 3
 * (sqrt(delta_f_x delta_f_y W)).  has_ap = 0: phase; 1: piston filter. */
ORACLE_API void oracle_weights(int32_t model, double c, double r0, double L0,
                               int32_t has_ap, double D, double d, double wavelength,
                               int64_t n, const double* fx, const double* fy,
                               const double* area, double* w) {
    for (int64_t i = 0; i < n; ++i) {
        double f = sqrt(fx[i] * fx[i] + fy[i] * fy[i]);
        double v = sqrt(oracle_psd(model, c, r0, L0, f) * area[i]);
        if (has_ap) v *= oracle_aperture_filter(D, d, f);
        /* optical path instead of phase: OPD = (lambda / 2 pi) phase, the
         * conversion of the structure function in Sec. 4.4 */
        if (wavelength > 0.0) v *= wavelength / (2.0 * M_PI);
        w[i] = v;
    }
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and Gaussian coefficients                             */
/* ------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each
 * round multiplies words 0 and 2 by the two round multipliers, mixes the
 * high halves with words 1 and 3 and the round key, and bumps the key by
 * the two Weyl constants (the golden ratio and sqrt(3)-1 in 0.32 fixed
 * point). */
ORACLE_API void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                     uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* one 32-bit word -> uniform in (0,1): the top 23 bits plus half a step,
 * (2m + 1) 2^-24 with 2m + 1 < 2^24, so the value is exact in binary32 */
static double word_to_uniform(uint32_t x) { return ((double)(x >> 9) + 0.5) * 0x1p-23; }

static void philox_block(uint64_t seed, uint64_t realisation, uint32_t block, uint32_t out[4]) {
    uint32_t ctr[4] = {block, (uint32_t)realisation, (uint32_t)(realisation >> 32), 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Coefficients of one realisation: c[2k] multiplies cos(2 pi f_k.x),
 * c[2k+1] multiplies sin(2 pi f_k.x).
 * mode 0 (Gaussian cos/sin): Philox block t gives four uniforms; Box-Muller
 *   of (u0,u1) and of (u2,u3) gives c[4t..4t+3].
 * mode 1 (Eq. 3 literal): block t = k gives R_n = sqrt(-2 ln u0) cos(2 pi u1)
 *   and R_u = u2; a = sqrt(2) R_n cos(2 pi R_u), b = -sqrt(2) R_n sin(2 pi R_u),
 *   so a cos + b sin = (2/sqrt 2) R_n cos(2 pi (f.x + R_u)). */
ORACLE_API void oracle_coefficients(uint64_t seed, uint64_t realisation, int64_t K,
                                    int32_t mode, double* c) {
    if (mode == 0) {
        int64_t nblk = (2 * K + 3) / 4;
        for (int64_t t = 0; t < nblk; ++t) {
            uint32_t x[4];
            philox_block(seed, realisation, (uint32_t)t, x);
            double g[4];
            for (int h = 0; h < 2; ++h) {
                double u1 = word_to_uniform(x[2 * h]);
                double u2 = word_to_uniform(x[2 * h + 1]);
                double rho = sqrt(-2.0 * log(u1));
                g[2 * h] = rho * cos(2.0 * M_PI * u2);
                g[2 * h + 1] = rho * sin(2.0 * M_PI * u2);
            }
            for (int i = 0; i < 4; ++i) {
                int64_t j = 4 * t + i;
                if (j < 2 * K) c[j] = g[i];
            }
        }
    } else {
        for (int64_t k = 0; k < K; ++k) {
            uint32_t x[4];
            philox_block(seed, realisation, (uint32_t)k, x);
            double u1 = word_to_uniform(x[0]);
            double u2 = word_to_uniform(x[1]);
            double Rn = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
            double Ru = word_to_uniform(x[2]);
            c[2 * k] = sqrt(2.0) * Rn * cos(2.0 * M_PI * Ru);
            c[2 * k + 1] = -sqrt(2.0) * Rn * sin(2.0 * M_PI * Ru);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Direct harmonic sums, Sec. 3 Eq. 3                                   */
/* ------------------------------------------------------------------ */

/* Realisation r uses frequency set s = r / R_block (fx, fy, w are
 * [n_sets][K]); its coefficients come from coef[r][2K] when coef is
 * non-NULL, else from (seed, counter + r).  filt (nullable) is a per
 * (column, set, frequency) multiplier [n_cols][n_sets][K].
 * out[r][p] = sum_k w_k filt_pk (c_2k cos 2 pi f_k.x_p + c_2k+1 sin 2 pi f_k.x_p) */
static void direct_sum(int64_t K, const double* fx, const double* fy, const double* w,
                       int64_t P, const double* px, const double* py, const double* filt,
                       int64_t n_sets, int64_t R, int64_t R_block, uint64_t seed,
                       uint64_t counter, int32_t mode, const double* coef, double* out) {
#pragma omp parallel
    {
        double* c = (double*)malloc(sizeof(double) * (size_t)(2 * K));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < R; ++r) {
            int64_t s = r / R_block;
            const double* cr = c;
            if (coef) cr = coef + r * 2 * K;
            else oracle_coefficients(seed, counter + (uint64_t)r, K, mode, c);
            for (int64_t p = 0; p < P; ++p) {
                double acc = 0.0;
                for (int64_t k = 0; k < K; ++k) {
                    int64_t i = s * K + k;
                    double arg = 2.0 * M_PI * (fx[i] * px[p] + fy[i] * py[p]);
                    double amp = w[i];
                    if (filt) amp *= filt[(p * n_sets + s) * K + k];
                    acc += amp * (cr[2 * k] * cos(arg) + cr[2 * k + 1] * sin(arg));
                }
                out[r * P + p] = acc;
            }
        }
        free(c);
    }
}

ORACLE_API void oracle_synthesize(int64_t K, const double* fx, const double* fy, const double* w,
                                  int64_t P, const double* px, const double* py, int64_t R,
                                  int64_t R_block, uint64_t seed, uint64_t counter, int32_t mode,
                                  const double* coef, double* phase) {
    int64_t n_sets = (R + R_block - 1) / R_block;
    direct_sum(K, fx, fy, w, P, px, py, NULL, n_sets, R, R_block, seed, counter, mode, coef,
               phase);
}

/* Aperture piston (Sec. 4.1): the phase averaged over the aperture is the
 * harmonic sum with each frequency multiplied by that aperture's filter F
 * (Eq. 7), evaluated at the aperture centre.  w is the unfiltered phase
 * weight. */
ORACLE_API void oracle_piston(int64_t K, const double* fx, const double* fy, const double* w,
                              int64_t n_ap, const double* cx, const double* cy,
                              const double* apD, const double* apd, int64_t R, int64_t R_block,
                              uint64_t seed, uint64_t counter, int32_t mode, const double* coef,
                              double* piston) {
    int64_t n_sets = (R + R_block - 1) / R_block;
    double* filt = (double*)malloc(sizeof(double) * (size_t)(n_ap * n_sets * K));
    for (int64_t p = 0; p < n_ap; ++p)
        for (int64_t i = 0; i < n_sets * K; ++i) {
            double f = sqrt(fx[i] * fx[i] + fy[i] * fy[i]);
            filt[p * n_sets * K + i] = oracle_aperture_filter(apD[p], apd[p], f);
        }
    direct_sum(K, fx, fy, w, n_ap, cx, cy, filt, n_sets, R, R_block, seed, counter, mode, coef,
               piston);
    free(filt);
}

/* Differential-piston structure function over baselines (Sec. 4.4): for
 * each realisation the pistons of two equal apertures at 0 and at B_b are
 * formed (w already carries the aperture filter), their difference squared
 * is averaged over realisations.  sf[b] = mean_r dp^2,
 * sf_stderr[b] = sqrt(sample variance of dp^2 / R). */
ORACLE_API void oracle_diff_piston_sf(int64_t K, const double* fx, const double* fy,
                                      const double* w, int64_t nB, const double* bx,
                                      const double* by, int64_t R, int64_t R_block,
                                      uint64_t seed, uint64_t counter, int32_t mode,
                                      double* sf, double* sf_stderr) {
    int64_t P = nB + 1;
    double* px = (double*)malloc(sizeof(double) * (size_t)P);
    double* py = (double*)malloc(sizeof(double) * (size_t)P);
    px[0] = 0.0;
    py[0] = 0.0;
    for (int64_t b = 0; b < nB; ++b) {
        px[b + 1] = bx[b];
        py[b + 1] = by[b];
    }
    double* pist = (double*)malloc(sizeof(double) * (size_t)(R * P));
    int64_t n_sets = (R + R_block - 1) / R_block;
    direct_sum(K, fx, fy, w, P, px, py, NULL, n_sets, R, R_block, seed, counter, mode, NULL,
               pist);
    for (int64_t b = 0; b < nB; ++b) {
        double s2 = 0.0, s4 = 0.0;
        for (int64_t r = 0; r < R; ++r) {
            double dp = pist[r * P + b + 1] - pist[r * P];
            s2 += dp * dp;
            s4 += dp * dp * dp * dp;
        }
        double mean = s2 / (double)R;
        sf[b] = mean;
        if (sf_stderr) {
            double var = (R > 1) ? (s4 - s2 * s2 / (double)R) / (double)(R - 1) : 0.0;
            sf_stderr[b] = sqrt(var > 0.0 ? var / (double)R : 0.0);
        }
    }
    free(pist);
    free(px);
    free(py);
}

/* ------------------------------------------------------------------ */
/* Angle of arrival (aperture-averaged phase gradient, G-tilt): another  */
/* linear filtering of the phase PSD (Sec. 2 names angle-of-arrival    */
/* fluctuations among the quantities the method simulates)             */
/* ------------------------------------------------------------------ */
/* Gradient along axis (0: x, 1: y) of the piston of aperture j, i.e. the
 * phase gradient averaged over the aperture: differentiating Eq. 3 with the
 * filter F of Eq. 7 with respect to the centre gives
 *   t_r(c) = sum_k w_k F(|f_k|) 2 pi f_axis,k (b_rk cos 2 pi f_k.c
 *                                              - a_rk sin 2 pi f_k.c)
 * in rad/m; the angle of arrival is lambda / (2 pi) times it. */
ORACLE_API void oracle_tilt(int64_t K, const double* fx, const double* fy, const double* w,
                            int64_t n_ap, const double* cx, const double* cy, const double* apD,
                            const double* apd, int64_t R, int64_t R_block, uint64_t seed,
                            uint64_t counter, int32_t mode, const double* coef, int32_t axis,
                            double* tilt) {
#pragma omp parallel
    {
        double* c = (double*)malloc(sizeof(double) * (size_t)(2 * K));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < R; ++r) {
            int64_t s = r / R_block;
            const double* cr = c;
            if (coef) cr = coef + r * 2 * K;
            else oracle_coefficients(seed, counter + (uint64_t)r, K, mode, c);
            for (int64_t j = 0; j < n_ap; ++j) {
                double acc = 0.0;
                for (int64_t k = 0; k < K; ++k) {
                    int64_t i = s * K + k;
                    double f = sqrt(fx[i] * fx[i] + fy[i] * fy[i]);
                    double arg = 2.0 * M_PI * (fx[i] * cx[j] + fy[i] * cy[j]);
                    double g = 2.0 * M_PI * (axis == 0 ? fx[i] : fy[i]);
                    double amp = w[i] * oracle_aperture_filter(apD[j], apd[j], f) * g;
                    acc += amp * (cr[2 * k + 1] * cos(arg) - cr[2 * k] * sin(arg));
                }
                tilt[r * n_ap + j] = acc;
            }
        }
        free(c);
    }
}

/* ------------------------------------------------------------------ */
/* Hyper-parameters of the Cartesian sampling (Sec. 4.3)                */
/* ------------------------------------------------------------------ */
/* g(x) = int_0^x f W(f) F(f)^2 df (the radial integral of the filtered
 * PSD; F = 1 without aperture) and its increments over steps of df,
 * inc(n) = g(n df) - g((n-1) df), by composite Simpson with 64 panels per
 * step.  Stopping rule: the increments must stay below eps g(inf) from
 * the step after n* on (eps relative to the saturated variance, the
 * paper's eps << sigma^2); max f = n* df, so N = 2 n* (N df = 2 max f).
 * g(inf) is the sum of the increments up to x_max = 200/D with an
 * aperture, 2000/L0 without (the integrand decays faster than f^-5 and as
 * f^-8/3: the tails left out are below 1e-7 and 3e-6 of g(inf)).
 * Returns N, or 0 for the Kolmogorov model (g diverges at f = 0), or -1
 * when even the last increment below x_max reaches eps g(inf) (the rule has
 * not settled within the integration range).  With wavelength > 0 the
 * variance is that of the optical path, (lambda / 2 pi)^2 times the phase
 * variance (Sec. 4.4). */
static double filtered_radial(int32_t model, double c, double r0, double L0, int32_t has_ap,
                              double D, double d, double f) {
    if (f <= 0.0) return 0.0;
    double w = oracle_psd(model, c, r0, L0, f);
    double F = has_ap ? oracle_aperture_filter(D, d, f) : 1.0;
    return f * w * F * F;
}

ORACLE_API int64_t oracle_choose_cartesian(int32_t model, double c, double r0, double L0,
                                           int32_t has_ap, double D, double d, double df,
                                           double eps, double wavelength, double* sigma2) {
    if (model != 1) return 0;
    double x_max = has_ap ? 200.0 / D : 2000.0 / L0;
    int64_t n_max = (int64_t)ceil(x_max / df);
    double* inc = (double*)malloc(sizeof(double) * (size_t)n_max);
    double total = 0.0;
    const int panels = 64;
    for (int64_t n = 1; n <= n_max; ++n) {
        double a = (double)(n - 1) * df, h = df / panels, acc = 0.0;
        for (int p = 0; p < panels; ++p) {
            double x0 = a + p * h;
            acc += h / 6.0 *
                   (filtered_radial(model, c, r0, L0, has_ap, D, d, x0) +
                    4.0 * filtered_radial(model, c, r0, L0, has_ap, D, d, x0 + 0.5 * h) +
                    filtered_radial(model, c, r0, L0, has_ap, D, d, x0 + h));
        }
        inc[n - 1] = acc;
        total += acc;
    }
    int64_t nstar = 1;
    for (int64_t n = n_max; n >= 1; --n)
        if (inc[n - 1] >= eps * total) {
            nstar = n;
            break;
        }
    free(inc);
    if (nstar == n_max) return -1;
    double s = wavelength > 0.0 ? wavelength / (2.0 * M_PI) : 1.0;
    if (sigma2) *sigma2 = 2.0 * M_PI * total * s * s;
    return 2 * nstar;
}

/* ------------------------------------------------------------------ */
/* Temporal differential-piston structure function (Sec. 4.4, the      */
/* statistical test of the worked example)                              */
/* ------------------------------------------------------------------ */
/* Frozen flow (Taylor): the turbulence moves with velocity v, so at time
 * t the telescope at c sees the screen at c - v t.  pist[r][0][m] and
 * pist[r][1][m] are the pistons of telescopes 1 and 2 at t_m = m dt.  For
 * each realisation the structure function of the differential piston
 * dp(t) = p1(t) - p2(t) at lag j dt is the average over the M - j
 * available pairs of (dp(t_m + j dt) - dp(t_m))^2; sf[j] averages it over
 * the R realisations and sf_stderr[j] is the standard error of that mean
 * (sample standard deviation over realisations / sqrt R).  sf[0] = 0. */
ORACLE_API void oracle_temporal_sf(const double* pist, int64_t R, int64_t M, double* sf,
                                   double* sf_stderr) {
    for (int64_t j = 0; j < M; ++j) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t r = 0; r < R; ++r) {
            const double* p1 = pist + r * 2 * M;
            const double* p2 = p1 + M;
            double acc = 0.0;
            for (int64_t m = 0; m + j < M; ++m) {
                double d = (p1[m + j] - p2[m + j]) - (p1[m] - p2[m]);
                acc += d * d;
            }
            double v = acc / (double)(M - j);
            s1 += v;
            s2 += v * v;
        }
        sf[j] = s1 / (double)R;
        if (sf_stderr) {
            double var = R > 1 ? (s2 - s1 * s1 / (double)R) / (double)(R - 1) : 0.0;
            sf_stderr[j] = sqrt(var > 0.0 ? var / (double)R : 0.0);
        }
    }
}

/* The whole experiment: aperture centres c - v t_m of both telescopes
 * (t_m = m dt), pistons by Eq. 3 with the aperture-filtered weights w (the
 * filter of equal apertures folds into the weight, Eq. 7), then the
 * temporal structure function above. */
ORACLE_API void oracle_temporal_experiment(int64_t K, const double* fx, const double* fy,
                                           const double* w, const double* c1, const double* c2,
                                           const double* v, double dt, int64_t M, int64_t R,
                                           int64_t R_block, uint64_t seed, uint64_t counter,
                                           int32_t mode, double* sf, double* sf_stderr) {
    int64_t P = 2 * M;
    double* px = (double*)malloc(sizeof(double) * (size_t)P);
    double* py = (double*)malloc(sizeof(double) * (size_t)P);
    for (int64_t m = 0; m < M; ++m) {
        double t = (double)m * dt;
        px[m] = c1[0] - v[0] * t;
        py[m] = c1[1] - v[1] * t;
        px[M + m] = c2[0] - v[0] * t;
        py[M + m] = c2[1] - v[1] * t;
    }
    double* pist = (double*)malloc(sizeof(double) * (size_t)(R * P));
    int64_t n_sets = (R + R_block - 1) / R_block;
    direct_sum(K, fx, fy, w, P, px, py, NULL, n_sets, R, R_block, seed, counter, mode, NULL,
               pist);
    oracle_temporal_sf(pist, R, M, sf, sf_stderr);
    free(pist);
    free(px);
    free(py);
}

/* ------------------------------------------------------------------ */
/* Learned proposal density (the paper suggests systematising the      */
/* sampling with a mapping that knows the PSD, Sec. 5; the model below */
/* is this project's definition of such a mapping)                     */
/* ------------------------------------------------------------------ */
/* Network: x (5 features) -> h1 = tanh(W1 x + b1) (H) -> h2 = tanh(W2 h1 +
 * b2) (H) -> o = W3 h2 + b3 (2).  Flat parameter layout: W1[H][5], b1[H],
 * W2[H][H], b2[H], W3[2][H], b3[2].  Features of (ell = ln|f|, context
 * D, L0, |B|, theta_B) over the band [lmin, lmin + Lw]:
 *   (2 (ell - lmin)/Lw - 1, 2 theta_B/pi - 1, ln(D)/4, ln(L0)/4 - 1, ln|B|/4 - 1/2).
 * Density over (ell, theta): q = p(ell) (1 + alpha cos 2(theta - theta_B)) / (2 pi),
 * p proportional to exp(o0), alpha = 0.9 tanh(o1). */

static void mlp_features(double ell, double lmin, double Lw, const double ctx[4], double x[5]) {
    x[0] = 2.0 * (ell - lmin) / Lw - 1.0;
    x[1] = 2.0 * ctx[3] / M_PI - 1.0;
    x[2] = log(ctx[0]) / 4.0;
    x[3] = log(ctx[1]) / 4.0 - 1.0;
    x[4] = log(ctx[2]) / 4.0 - 0.5;
}

/* forward of one row; h1, h2 (length H) receive the activations */
static void mlp_row(const double* prm, int H, const double x[5], double* h1, double* h2,
                    double o[2]) {
    const double* W1 = prm;
    const double* b1 = W1 + 5 * H;
    const double* W2 = b1 + H;
    const double* b2 = W2 + H * H;
    const double* W3 = b2 + H;
    const double* b3 = W3 + 2 * H;
    for (int i = 0; i < H; ++i) {
        double s = b1[i];
        for (int j = 0; j < 5; ++j) s += W1[i * 5 + j] * x[j];
        h1[i] = tanh(s);
    }
    for (int i = 0; i < H; ++i) {
        double s = b2[i];
        for (int j = 0; j < H; ++j) s += W2[i * H + j] * h1[j];
        h2[i] = tanh(s);
    }
    for (int k = 0; k < 2; ++k) {
        double s = b3[k];
        for (int j = 0; j < H; ++j) s += W3[k * H + j] * h2[j];
        o[k] = s;
    }
}

ORACLE_API int64_t oracle_mlp_param_count(int H) { return 5 * H + H + H * H + H + 2 * H + 2; }

/* o[N][2] for rows (ell[i], ctx[i][4]) */
ORACLE_API void oracle_mlp_forward(const double* prm, int H, double lmin, double Lw, int64_t N,
                                   const double* ell, const double* ctx, double* out) {
#pragma omp parallel
    {
        double* h1 = (double*)malloc(sizeof(double) * (size_t)H);
        double* h2 = (double*)malloc(sizeof(double) * (size_t)H);
#pragma omp for
        for (int64_t i = 0; i < N; ++i) {
            double x[5];
            mlp_features(ell[i], lmin, Lw, ctx + 4 * i, x);
            mlp_row(prm, H, x, h1, h2, out + 2 * i);
        }
        free(h1);
        free(h2);
    }
}

/* backward of one row: adds dL/dprm given dL/do (do[2]) */
static void mlp_row_backward(const double* prm, int H, const double x[5], const double* h1,
                             const double* h2, const double dout[2], double* grad) {
    const double* W2 = prm + 5 * H + H;
    const double* W3 = W2 + H * H + H;
    double* gW1 = grad;
    double* gb1 = gW1 + 5 * H;
    double* gW2 = gb1 + H;
    double* gb2 = gW2 + H * H;
    double* gW3 = gb2 + H;
    double* gb3 = gW3 + 2 * H;
    double* d2 = (double*)malloc(sizeof(double) * (size_t)H);
    double* d1 = (double*)malloc(sizeof(double) * (size_t)H);
    for (int k = 0; k < 2; ++k) {
        gb3[k] += dout[k];
        for (int j = 0; j < H; ++j) gW3[k * H + j] += dout[k] * h2[j];
    }
    for (int j = 0; j < H; ++j) {
        double s = dout[0] * W3[j] + dout[1] * W3[H + j];
        d2[j] = s * (1.0 - h2[j] * h2[j]);
    }
    for (int i = 0; i < H; ++i) {
        gb2[i] += d2[i];
        for (int j = 0; j < H; ++j) gW2[i * H + j] += d2[i] * h1[j];
    }
    for (int j = 0; j < H; ++j) {
        double s = 0.0;
        for (int i = 0; i < H; ++i) s += W2[i * H + j] * d2[i];
        d1[j] = s * (1.0 - h1[j] * h1[j]);
    }
    for (int i = 0; i < H; ++i) {
        gb1[i] += d1[i];
        for (int j = 0; j < 5; ++j) gW1[i * 5 + j] += d1[i] * x[j];
    }
    free(d1);
    free(d2);
}

/* Loss and gradient of one mini-batch.  Contexts c < n_ctx (ctx[c][4]);
 * each owns m sample rows (ell, theta, h) at rows c*m .. c*m+m-1 and the
 * G-point midpoint grid of [lmin, lmin+Lw] that normalises p:
 *   logZ_c = log( sum_j exp(o0(grid_j, c)) Lw/G )
 *   L = -(1/H) sum_i h_i [ o0_i - logZ_c(i) + log(1 + alpha_i cos 2(theta_i - theta_B)) ]
 * with H = sum_i h_i, alpha = 0.9 tanh(o1).  grad receives dL/dprm. */
ORACLE_API double oracle_mlp_loss_grad(const double* prm, int Hd, double lmin, double Lw,
                                       int64_t n_ctx, int64_t m, const double* ctx,
                                       const double* ell, const double* theta, const double* h,
                                       int G, double* grad) {
    int64_t np = oracle_mlp_param_count(Hd);
    for (int64_t i = 0; i < np; ++i) grad[i] = 0.0;
    double* h1 = (double*)malloc(sizeof(double) * (size_t)Hd);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)Hd);
    double* og = (double*)malloc(sizeof(double) * (size_t)G);
    double Htot = 0.0;
    for (int64_t i = 0; i < n_ctx * m; ++i) Htot += h[i];
    double loss = 0.0;
    for (int64_t c = 0; c < n_ctx; ++c) {
        const double* cc = ctx + 4 * c;
        /* grid forward and log-normaliser */
        double mx = -1e300;
        for (int j = 0; j < G; ++j) {
            double x[5], o[2];
            mlp_features(lmin + (j + 0.5) * Lw / G, lmin, Lw, cc, x);
            mlp_row(prm, Hd, x, h1, h2, o);
            og[j] = o[0];
            if (o[0] > mx) mx = o[0];
        }
        double se = 0.0;
        for (int j = 0; j < G; ++j) se += exp(og[j] - mx);
        double logZ = mx + log(se * Lw / G);
        double Hc = 0.0;
        /* sample rows */
        for (int64_t r = 0; r < m; ++r) {
            int64_t i = c * m + r;
            double x[5], o[2];
            mlp_features(ell[i], lmin, Lw, cc, x);
            mlp_row(prm, Hd, x, h1, h2, o);
            double ta = tanh(o[1]);
            double alpha = 0.9 * ta;
            double C = cos(2.0 * (theta[i] - cc[3]));
            double wi = h[i] / Htot;
            loss -= wi * (o[0] - logZ + log(1.0 + alpha * C));
            double dout[2] = {-wi, -wi * C / (1.0 + alpha * C) * 0.9 * (1.0 - ta * ta)};
            mlp_row_backward(prm, Hd, x, h1, h2, dout, grad);
            Hc += h[i];
        }
        /* grid rows: d logZ / d o0_j = softmax_j */
        for (int j = 0; j < G; ++j) {
            double x[5], o[2];
            mlp_features(lmin + (j + 0.5) * Lw / G, lmin, Lw, cc, x);
            mlp_row(prm, Hd, x, h1, h2, o);
            double dout[2] = {(Hc / Htot) * exp(og[j] - mx) / se, 0.0};
            mlp_row_backward(prm, Hd, x, h1, h2, dout, grad);
        }
    }
    free(og);
    free(h1);
    free(h2);
    return loss;
}

/* Training rows from the plain log-polar sampler: row i of context c uses
 * R2 point index+1+c*m+r; h = f^2 W(f) F_D(f)^2 2 (1 - cos 2 pi f |B| cos(theta - theta_B)),
 * the variance contribution per unit (ln f, theta) of the differential
 * piston over B (Eq. 7 and the structure function of Sec. 4.4). */
ORACLE_API void oracle_proposal_rows(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_ctx,
                                     int64_t m, const double* ctx, double r0, double c_psd,
                                     double fmin, double fmax, double* ell, double* theta,
                                     double* h) {
    int64_t n = n_ctx * m;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_r2_points(s0x, s0y, index, n, ux, uy);
    double lmin = log(fmin), Lw = log(fmax / fmin);
    for (int64_t i = 0; i < n; ++i) {
        const double* cc = ctx + 4 * (i / m);
        double l = lmin + Lw * ux[i];
        double th = 2.0 * M_PI * uy[i];
        double f = exp(l);
        double W = oracle_psd(1, c_psd, r0, cc[1], f);
        double F = oracle_aperture_filter(cc[0], 0.0, f);
        double proj = f * cc[2] * cos(th - cc[3]);
        ell[i] = l;
        theta[i] = th;
        h[i] = f * f * W * F * F * 2.0 * (1.0 - cos(2.0 * M_PI * proj));
    }
    free(ux);
    free(uy);
}

/* Sampling table of the proposal for aperture D, outer scale L0 and nB
 * baselines (length bl[b], direction bth[b]): on n_cells equal cells of
 * [lmin, lmin+Lw] (midpoints ell_j), per baseline p_b(j) = exp(o0)/Z_b with
 * Z_b = sum_j exp(o0) dl, alpha_b(j) = 0.9 tanh(o1); the mixture over
 * baselines has angular part sum_b p_b alpha_b cos 2(theta - theta_b) / nB
 * = pbar (abar cos 2(theta - phi)); the defensive mixture adds beta of the
 * plain density 1/Lw:  p = (1-beta) pbar + beta/Lw,
 * alpha = (1-beta) pbar abar / p.  cdf[j] = sum_{i<j} p_i dl / sum_i p_i dl. */
ORACLE_API void oracle_proposal_table(const double* prm, int H, double lmin, double Lw,
                                      int n_cells, double D, double L0, int64_t nB,
                                      const double* bl, const double* bth, double beta,
                                      double* p, double* alpha, double* phi, double* cdf) {
    double dl = Lw / n_cells;
    double* pb = (double*)calloc((size_t)n_cells, sizeof(double));
    double* A = (double*)calloc((size_t)n_cells, sizeof(double));
    double* B = (double*)calloc((size_t)n_cells, sizeof(double));
    double* o0 = (double*)malloc(sizeof(double) * (size_t)n_cells);
    double* o1 = (double*)malloc(sizeof(double) * (size_t)n_cells);
    double* h1 = (double*)malloc(sizeof(double) * (size_t)H);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)H);
    for (int64_t b = 0; b < nB; ++b) {
        double cc[4] = {D, L0, bl[b], bth[b]};
        double mx = -1e300;
        for (int j = 0; j < n_cells; ++j) {
            double x[5], o[2];
            mlp_features(lmin + (j + 0.5) * dl, lmin, Lw, cc, x);
            mlp_row(prm, H, x, h1, h2, o);
            o0[j] = o[0];
            o1[j] = o[1];
            if (o[0] > mx) mx = o[0];
        }
        double Z = 0.0;
        for (int j = 0; j < n_cells; ++j) Z += exp(o0[j] - mx) * dl;
        for (int j = 0; j < n_cells; ++j) {
            double pj = exp(o0[j] - mx) / Z;
            double al = 0.9 * tanh(o1[j]);
            pb[j] += pj / (double)nB;
            A[j] += pj * al * cos(2.0 * bth[b]) / (double)nB;
            B[j] += pj * al * sin(2.0 * bth[b]) / (double)nB;
        }
    }
    double tot = 0.0;
    for (int j = 0; j < n_cells; ++j) {
        double amp = sqrt(A[j] * A[j] + B[j] * B[j]);
        p[j] = (1.0 - beta) * pb[j] + beta / Lw;
        alpha[j] = (1.0 - beta) * amp / p[j];
        phi[j] = 0.5 * atan2(B[j], A[j]);
        tot += p[j] * dl;
    }
    double run = 0.0;
    for (int j = 0; j < n_cells; ++j) {
        p[j] /= tot;
        cdf[j] = run;
        run += p[j] * dl;
    }
    free(pb); free(A); free(B); free(o0); free(o1); free(h1); free(h2);
}

/* Learned frequency sampler: R2 point (u1, u2) -> cell j with
 * cdf[j] <= u1 < cdf[j+1]; ell = lmin + j dl + (u1 - cdf[j]) / p[j]; the
 * angle solves t + (alpha/2) sin 2t = 2 pi u2 (12 Newton steps from
 * t = 2 pi u2), theta = t + phi[j]; area = f^2 / (K q) with
 * q = p[j] (1 + alpha cos 2t) / (2 pi), the inverse density of the draw. */
ORACLE_API void oracle_sample_learned(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_sets,
                                      int64_t K, double lmin, double Lw, int n_cells,
                                      const double* p, const double* alpha, const double* phi,
                                      const double* cdf, double* fx, double* fy, double* area) {
    int64_t n = n_sets * K;
    double* ux = (double*)malloc(sizeof(double) * (size_t)n);
    double* uy = (double*)malloc(sizeof(double) * (size_t)n);
    oracle_r2_points(s0x, s0y, index, n, ux, uy);
    double dl = Lw / n_cells;
    for (int64_t i = 0; i < n; ++i) {
        int j = n_cells - 1;
        for (int c = 1; c < n_cells; ++c)
            if (cdf[c] > ux[i]) { j = c - 1; break; }
        double ell = lmin + j * dl + (ux[i] - cdf[j]) / p[j];
        double target = 2.0 * M_PI * uy[i];
        double t = target;
        for (int it = 0; it < 12; ++it)
            t -= (t + 0.5 * alpha[j] * sin(2.0 * t) - target) / (1.0 + alpha[j] * cos(2.0 * t));
        double th = t + phi[j];
        double f = exp(ell);
        double q = p[j] * (1.0 + alpha[j] * cos(2.0 * t)) / (2.0 * M_PI);
        fx[i] = f * cos(th);
        fy[i] = f * sin(th);
        area[i] = f * f / ((double)K * q);
    }
    free(ux);
    free(uy);
}

/* ------------------------------------------------------------------ */
/* Point-set measures of frequency sets (Sec. 3.1-3.2: clashes, gaps,   */
/* discrepancy) and the per-set sampling error                          */
/* ------------------------------------------------------------------ */
/* For each set s of K points, mapped to the unit square by
 * u = ((fx - x0)/Lx, (fy - y0)/Ly):
 *   min_dist[s]  the smallest distance between two of its points;
 *   n_clash[s]   the number of pairs closer than r_clash (the frequency
 *                "clashes" of Sec. 3.1);
 *   l2_star[s]   the L2 star discrepancy T, from Warnock's closed form
 *     T^2 = 1/9 - (1/(2K)) sum_i (1 - x_i^2)(1 - y_i^2)
 *           + (1/K^2) sum_i sum_j (1 - max(x_i, x_j)) (1 - max(y_i, y_j)). */
ORACLE_API void oracle_point_set_measures(int64_t n_sets, int64_t K, const double* fx,
                                          const double* fy, double x0, double y0, double Lx,
                                          double Ly, double r_clash, double* min_dist,
                                          int64_t* n_clash, double* l2_star) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sets; ++s) {
        const double* px = fx + s * K;
        const double* py = fy + s * K;
        double dmin2 = INFINITY, s1 = 0.0, s2 = 0.0;
        int64_t clash = 0;
        for (int64_t i = 0; i < K; ++i) {
            double xi = (px[i] - x0) / Lx, yi = (py[i] - y0) / Ly;
            s1 += (1.0 - xi * xi) * (1.0 - yi * yi);
            for (int64_t j = 0; j < K; ++j) {
                double xj = (px[j] - x0) / Lx, yj = (py[j] - y0) / Ly;
                s2 += (1.0 - fmax(xi, xj)) * (1.0 - fmax(yi, yj));
                if (j > i) {
                    double d2 = (xi - xj) * (xi - xj) + (yi - yj) * (yi - yj);
                    if (d2 < dmin2) dmin2 = d2;
                    if (d2 < r_clash * r_clash) ++clash;
                }
            }
        }
        double Kd = (double)K;
        double T2 = 1.0 / 9.0 - s1 / (2.0 * Kd) + s2 / (Kd * Kd);
        min_dist[s] = sqrt(dmin2);
        n_clash[s] = clash;
        l2_star[s] = sqrt(T2 > 0.0 ? T2 : 0.0);
    }
}

/* Conditional expectation of the differential-piston structure function
 * given one frequency set (its noise-free value): the coefficients are iid
 * N(0,1), so p(B) - p(0) is N(0, S) with
 *   S[s][b] = sum_k w_k^2 2 (1 - cos 2 pi f_k.B_b),
 * w carrying the aperture filter of Eq. 7.  Its relative error against the
 * analytic curve is the sampling error of the set alone. */
ORACLE_API void oracle_set_sf_expectation(int64_t K, const double* fx, const double* fy,
                                          const double* w, int64_t n_sets, int64_t nB,
                                          const double* bx, const double* by, double* S) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sets; ++s) {
        for (int64_t b = 0; b < nB; ++b) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                int64_t i = s * K + k;
                double arg = 2.0 * M_PI * (fx[i] * bx[b] + fy[i] * by[b]);
                acc += w[i] * w[i] * 2.0 * (1.0 - cos(arg));
            }
            S[s * nB + b] = acc;
        }
    }
}
