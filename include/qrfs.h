/*
 * qrfs.h -- C ABI of libqrfs, quasi-random frequency sampling for optical
 * turbulence on AMD Instinct MI355X (gfx950).
 *
 * Method: Berdja et al., "Quasi-Random Frequency Sampling for Optical
 * Turbulence Simulations" (arXiv 2404.02978).  A turbulent quantity is the
 * direct harmonic sum of Sec. 3, Eq. 3 over K spatial frequencies f_k placed
 * by the R2 low-discrepancy sequence (Sec. 3.2, Eqs. 5-6), each weighted by
 * sqrt(PSD x cell area) (Eq. 3) and, for aperture piston, by the circular
 * aperture filter of Sec. 4.1, Eq. 7.  Each frequency carries two random
 * coefficients:
 *     phi_r(x) = sum_k w_k [ a_rk cos(2 pi f_k.x) + b_rk sin(2 pi f_k.x) ].
 *
 * Conventions for every entry point
 *   - Units: frequencies in cycles/m, positions in m, phase in rad at the
 *     wavelength r0 refers to (Sec. 4.1), structure functions in rad^2;
 *     with qrfs_psd.wavelength > 0 every output of the PSD-weighted sums is
 *     optical path instead (m, m^2 for structure functions, Sec. 4.4).
 *   - Array arguments are DEVICE pointers (memory of the context's device),
 *     contiguous, naturally aligned, owned by the caller, unless the comment
 *     says "host".  Struct arguments are host pointers.  Outputs must be
 *     ordinary (coarse-grained) device memory, as hipMalloc returns: the
 *     kernels for wide point sets add partial sums into them with device
 *     float atomics, which host-mapped or fine-grained memory does not
 *     support.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL =
 *     the null stream) and the call returns after enqueueing; results are
 *     ready when the stream is synchronised.  Calls on one context must not
 *     overlap in time (the context's workspace is shared).
 *   - Every argument is checked before anything is enqueued.  On error the
 *     call returns a negative status, enqueues nothing and leaves a
 *     thread-local detail message (qrfs_last_error_detail).  No C++
 *     exception crosses this boundary.
 *   - Realisations are grouped in frequency sets (R_block realisations per
 *     set, n_sets = ceil(R / R_block)): realisation r uses set r / R_block.
 *     R_block = 1 gives every realisation fresh frequencies, as the paper
 *     does (Sec. 3.2: the sequence is never reinitialised); R_block = R
 *     shares one set (the static sampling Sec. 2.3 warns about).
 *   - Random coefficients: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed lo32, seed hi32) = rng.seed and counter (block t, realisation
 *     lo32, realisation hi32, 0), realisation = rng.counter + r, gives the
 *     words x0..x3 of block t; each word gives the uniform
 *     u = ((x >> 9) + 1/2) 2^-23 = (2m + 1) 2^-24, m = x >> 9 (exact in
 *     binary32, never 0 or 1); Box-Muller of (u0,u1) gives
 *     c[4t] = sqrt(-2 ln u0) cos(2 pi u1), c[4t+1] = sqrt(-2 ln u0) sin(2 pi u1),
 *     and of (u2,u3) likewise c[4t+2], c[4t+3], with c[2k] = a_k,
 *     c[2k+1] = b_k (QRFS_COEF_GAUSS_CS).  QRFS_COEF_EQ3 uses
 *     block t = k: R_n = sqrt(-2 ln u0) cos(2 pi u1), R_u = u2,
 *     a = sqrt2 R_n cos(2 pi R_u), b = -sqrt2 R_n sin(2 pi R_u), which is the
 *     literal (2/sqrt2) R_n cos(2 pi (f.x + R_u)) term of Eq. 3.
 */
#ifndef QRFS_H
#define QRFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define QRFS_API __attribute__((visibility("default")))
#else
#define QRFS_API
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t qrfs_status;
#define QRFS_OK 0
#define QRFS_ERR_INVALID_ARG (-1)   /* bad size, pointer, parameter          */
#define QRFS_ERR_OUT_OF_MEMORY (-2) /* workspace allocation failed            */
#define QRFS_ERR_DEVICE (-3)        /* HIP runtime error (launch, fault)      */
#define QRFS_ERR_UNSUPPORTED (-4)   /* valid but not implemented combination  */
#define QRFS_ERR_NOT_CONVERGED (-5) /* an iterative rule did not settle       */

#define QRFS_ABI_VERSION 5

/* Static string for a status code. */
QRFS_API const char* qrfs_error_string(qrfs_status s);
/* Thread-local detail of the last failing call on this thread ("" if none);
 * valid until the next library call on the same thread. */
QRFS_API const char* qrfs_last_error_detail(void);
/* QRFS_ABI_VERSION of the built library. */
QRFS_API int32_t qrfs_abi_version(void);

/* --------------------------------------------------------------- context */
/* Opaque: device ordinal, device workspace (grown on demand, freed by
 * destroy), tuned launch shapes. */
typedef struct qrfs_context qrfs_context;

/* Creates a context on HIP device `device`.  *out receives the handle.
 * workspace_cap_bytes bounds the device workspace the context may hold
 * (0: no bound).  A call whose workspace would exceed it fails with
 * QRFS_ERR_OUT_OF_MEMORY before enqueueing anything; the two-phase kernel
 * cuts its coefficient tiles into pieces that fit the cap when it can (at
 * least one 256-row block of one set).  Batches allocate their own buffers
 * (qrfs_batch_create) and are not bounded by it.
 * Errors: out NULL; device out of range; no HIP device (QRFS_ERR_DEVICE). */
QRFS_API qrfs_status qrfs_context_create(qrfs_context** out, int32_t device,
                                         size_t workspace_cap_bytes);
/* Synchronises the device and frees the workspace.  NULL is accepted. */
QRFS_API qrfs_status qrfs_context_destroy(qrfs_context* ctx);

/* Launch policy of a context (no paper passage: an implementation knob).
 * QRFS_TUNE_WIDE_PATH selects how FP32 / split-BF16 / BF16x6 phase fields
 * and pistons (qrfs_synthesize_phase, qrfs_piston, qrfs_diff_piston) are
 * contracted: 0 (default) lets the library choose, 1 always uses the fused
 * kernel (coefficients drawn in registers per column tile), 2 uses the
 * two-phase kernel (coefficients drawn once into workspace tiles of at most
 * 2 GiB, then 256 x 256 MFMA tiles) whenever the output fits it.
 * QRFS_TUNE_RANGE_FREQS sets how many frequencies the two-phase kernel
 * sums in FP32 before adding them into the output in FP32-class precisions
 * (default 2048, rounded to whole chunks; 0 restores the default).
 * QRFS_TUNE_TILE_BYTES caps the workspace the two-phase kernel stages its
 * coefficient tiles in (default 2 GiB, 0 restores it); larger problems are
 * cut into pieces of whole sets, or of 256-row blocks of one set.
 * Errors: NULL context, unknown key, value out of range. */
#define QRFS_TUNE_WIDE_PATH 1
#define QRFS_TUNE_RANGE_FREQS 2
#define QRFS_TUNE_TILE_BYTES 3
QRFS_API qrfs_status qrfs_context_set_tuning(qrfs_context* ctx, int32_t key, int64_t value);

/* ------------------------------------------------------------ parameters */
/* Phase PSD (Sec. 4.1, Eq. 7 first factor), cycles/m:
 *   von Karman  W(f) = c r0^(-5/3) (f^2 + L0^-2)^(-11/6)
 *   Kolmogorov  W(f) = c r0^(-5/3) f^(-11/3)     (L0 ignored; W(0) := 0)
 * c <= 0 selects Gamma(11/6)^2/(2 pi^(11/3)) (24/5 Gamma(6/5))^(5/6)
 * = 0.0228955871..., the value Eq. 7 prints as 0.02289.
 * r0 is the Fried parameter at the wavelength lambda of the light
 * (Sec. 4.1: r0 = r0(lambda); it scales as lambda^(6/5), so a caller with
 * r0 given at another wavelength converts it first).  wavelength = 0: phases
 * in rad at that wavelength.  wavelength = lambda > 0 (m): optical path
 * instead, phase times lambda / (2 pi), so every weight carries that factor
 * and structure functions come out as D_OPD = (lambda / 2 pi)^2 D_phase in
 * m^2 (Sec. 4.4).  Entry points that take a qrfs_psd apply it
 * (qrfs_weights, qrfs_sample_weights, qrfs_diff_piston_structure,
 * qrfs_temporal_piston_structure, batch instances, and the variance of
 * qrfs_choose_cartesian). */
#define QRFS_PSD_KOLMOGOROV 0
#define QRFS_PSD_VON_KARMAN 1
typedef struct {
    int32_t model;
    double c;
    double r0;         /* Fried parameter at `wavelength`, m (> 0)      */
    double L0;         /* outer scale, m (> 0 for von Karman)            */
    double wavelength; /* m; 0: outputs in rad, > 0: optical path in m  */
} qrfs_psd;

/* Circular aperture of diameter D with central obstruction d (Eq. 7):
 * F(f) = 2 (D J1(pi D f) - d J1(pi d f)) / (pi (D^2 - d^2) f), F(0) = 1,
 * applied signed (Eq. 7's 4(...)^2 is F^2).  0 <= d < D. */
typedef struct {
    double D;
    double d;
} qrfs_aperture;

/* Frequency sampler (Sec. 3.2).  The 2-D R2 sequence is kept as the exact
 * 64-bit Weyl sequence U_n = S0 + n A mod 2^64 with A = round(2^64/psi^j),
 * psi the plastic number (Eq. 6); u = (U >> 11) 2^-53.  The state is
 * updated before use, so a call starting at `index` uses n = index+1 ...
 *   R2_CARTESIAN (Eq. 5, delta_f_x = delta_f_y = df, n_x = n_y = N):
 *       f = N df (u - 1/2), cell area (N df)^2 / K   (= df^2 for K = N^2);
 *       N df = 2 max|f|, as the worked example of Sec. 4.4 fixes.
 *   R2_LOGPOLAR: |f| = fmin (fmax/fmin)^(u_x), angle = 2 pi u_y,
 *       cell area = 2 pi ln(fmax/fmin) |f|^2 / K.
 *   R2_DISC: polar quasi-random frequencies (Sec. 3.2's square-to-disc
 *       mapping): the concentric map of Shirley and Chiu sends
 *       (a, b) = (2u_x - 1, 2u_y - 1) to radius max(|a|, |b|) fmax and an
 *       angle linear along the concentric square's edge; it preserves area,
 *       so every point stands for pi fmax^2 / K.  Uses fmax only.
 *   LEARNED: the points are drawn from the sampling table of `proposal`
 *       (built by qrfs_proposal_tabulate): u_x through the inverse CDF of
 *       its piecewise-constant density in ln|f| over [fmin, fmax] of the
 *       proposal, u_y through the inverse CDF of its angular factor, and
 *       each point gets the area f^2 / (K q), q the density of the draw, so
 *       the weighted sums stay unbiased.
 * The randomised schemes that Sec. 3.1 sets the quasi-random sampling
 * against draw their unit-square points u from a pseudo-random stream
 * instead: Philox4x32-10 keyed by seed_x, counter (n lo, n hi, low word of
 * seed_y, 0x46524551) for point n (disjoint from every coefficient
 * counter, whose last word is 0); u_x = top 53 bits of words (1:0) times
 * 2^-53, u_y the same of words (3:2).
 *   RANDOM_CARTESIAN, RANDOM_LOGPOLAR, RANDOM_DISC: fully random
 *       frequencies through the Cartesian, log-polar and disc maps above
 *       (same parameters and cell areas).
 *   JITTER (Eq. 4): the square of side N df centred on the origin is cut
 *       into N x N cells of side df; point k = iy N + ix of a set lies in
 *       cell (ix, iy) at df (i + u - N/2) per axis, area df^2.  K must
 *       equal N^2.
 * seed_x, seed_y: R2 schemes: S0 in 0.64 fixed point (2^63 = 1/2,
 * Sec. 3.2's (0.5, 0.5)); randomised schemes: key and stream id as above.
 * index (IN/OUT): position in the sequence; every call advances it by the
 * number of points drawn, so consecutive calls continue the sequence. */
#define QRFS_SAMPLER_R2_CARTESIAN 0
#define QRFS_SAMPLER_R2_LOGPOLAR 1
#define QRFS_SAMPLER_LEARNED 2
#define QRFS_SAMPLER_R2_DISC 3
#define QRFS_SAMPLER_JITTER 4
#define QRFS_SAMPLER_RANDOM_CARTESIAN 5
#define QRFS_SAMPLER_RANDOM_LOGPOLAR 6
#define QRFS_SAMPLER_RANDOM_DISC 7
typedef struct {
    int32_t scheme;
    int32_t N;   /* Cartesian, jitter: points per axis (> 0)        */
    double df;   /* Cartesian, jitter: frequency pitch (> 0)         */
    double fmin; /* log-polar: band, 0 < fmin < fmax                 */
    double fmax; /* log-polar: upper band edge; disc: radius (> 0)   */
    uint64_t seed_x;
    uint64_t seed_y;
    uint64_t index;
    const struct qrfs_proposal* proposal; /* LEARNED only, else ignored */
} qrfs_sampler;

#define QRFS_COEF_GAUSS_CS 0
#define QRFS_COEF_EQ3 1
typedef struct {
    uint64_t seed;    /* Philox key                                   */
    uint64_t counter; /* global index of realisation 0 of this call   */
    int32_t mode;     /* QRFS_COEF_GAUSS_CS or QRFS_COEF_EQ3          */
} qrfs_rng;

/* Arithmetic of the sums:
 *   FP64        FP64 range reduction, FP64 sincos, FP64 Box-Muller and
 *               FP64 accumulation (vector ALU); output double.
 *   FP32        FP64 range reduction of 2 pi f.x, FP32 sincos and
 *               Box-Muller, FP32 matrix-core (MFMA) contraction with FP32
 *               accumulation, folded into a second FP32 accumulator every
 *               32 frequencies (the two-phase kernel for wide point sets
 *               adds into the output every 2048); output float.
 *   (All FP32-class precisions sum sets of at most 8 realisations on the
 *   vector ALU with this FP32 arithmetic: a matrix-core tile needs 32 rows.
 *   The split-BF16 and BF16x6 results are then those FP32 sums.  Their
 *   per-aperture filter of Eq. 7 (qrfs_piston, qrfs_tilt) is evaluated to
 *   binary32 accuracy like the basis it scales (the J1 of qrfs_weights'
 *   FP32-class weights); FP64 evaluates it in binary64.)
 *   SPLIT_BF16  as FP32 but each operand is split into bf16 hi + lo and the
 *               contraction is hi.hi + hi.lo + lo.hi on bf16 MFMA with FP32
 *               accumulation (~16 significant bits); output float.
 *   BF16X6      each operand split three ways into bf16 hi + mid + lo (24
 *               significant bits) and six products (hi.hi, hi.mid, mid.hi,
 *               hi.lo, mid.mid, lo.hi) on bf16 MFMA: FP32-class accuracy on
 *               the matrix cores, which run concurrently with the vector ALU
 *               that draws the coefficients (FP32 MFMA shares the vector
 *               datapath and does not); output float.
 *   FP16X3      each operand split into fp16 hi (rounded to nearest, 11
 *               significant bits) + lo (the rounded remainder): 22
 *               significant bits, three products (lo.hi, hi.lo, hi.hi) on
 *               fp16 MFMA with FP32 accumulation; the basis amplitudes of
 *               each block's frequency range are scaled by a power of two
 *               into the fp16 range and the sums scaled back exactly.
 *               FP32-class accuracy (per-product error <= 2^-19 relative, an
 *               absolute floor of 2^-25 times the range's scale) with half
 *               the operand-split work and half the products of BF16X6.
 *               qrfs_synthesize_phase, qrfs_piston, qrfs_tilt,
 *               qrfs_diff_piston and the structure functions; the two-phase
 *               kernel for wide point sets scales each set's coefficient
 *               tiles by one power of two (from its largest weight and the
 *               largest coefficient the generators draw), so with
 *               caller-given coefficients it contracts in the fused kernel;
 *               batches take it on every launch shape; output float. */
#define QRFS_PREC_FP64 0
#define QRFS_PREC_FP32 1
#define QRFS_PREC_SPLIT_BF16 2
#define QRFS_PREC_BF16X6 3
#define QRFS_PREC_FP16X3 4

/* ---------------------------------------------------------- entry points */

/* Largest number of frequencies one sampling or weight call handles (one
 * launch: 2^32 - 2^20, about 4.3e9, i.e. 103 GB of fx, fy and weights). */
#define QRFS_MAX_POINTS_PER_CALL ((int64_t)4293918720)

/* R2 frequency sampling (Sec. 3.2, Eqs. 5-6).  Writes n_sets*K points
 * (set-major: set s occupies [s*K, (s+1)*K)) to fx, fy (cycles/m) and the
 * cell area each point stands for to area (m^-2), all double[n_sets*K].
 * Cell areas are per set of K points.  s->index += n_sets*K on success.
 * One call draws at most QRFS_MAX_POINTS_PER_CALL points (one launch);
 * larger sets of points are drawn in several calls, which continue the
 * sequence from s->index.
 * Errors: K, n_sets <= 0; n_sets*K > QRFS_MAX_POINTS_PER_CALL; NULL
 * pointers; Cartesian N <= 0 or df <= 0; log-polar fmin <= 0 or
 * fmax <= fmin; LEARNED without a proposal or before its table was built. */
QRFS_API qrfs_status qrfs_sample_frequencies(qrfs_context* ctx, qrfs_sampler* s, int64_t n_sets,
                                    int64_t K, double* fx, double* fy, double* area,
                                    void* stream);

/* Amplitude weights of Eq. 3: w = sqrt(W(|f|) area) (phase), multiplied by
 * the signed aperture filter F(|f|) when ap != NULL (piston of equal
 * apertures, Eq. 7).  All arrays double[n].  An exact f = 0 with the
 * Kolmogorov model contributes w = 0.
 * precision: the precision of the sums the weights will feed.
 *   QRFS_PREC_FP64: every step in binary64 (the PSD power within ~3e-16,
 *   the filter's J1 within ~2e-15).
 *   QRFS_PREC_FP32, _SPLIT_BF16, _BF16X6, _FP16X3: weights for FP32-class
 *   sums, which round them to binary32 anyway, with every factor to
 *   binary32 accuracy: the PSD power within ~1e-7 (binary32 Newton step),
 *   the square roots within ~1e-14, the filter from a shorter J1 with a
 *   binary32 Hankel branch (absolute error ~3e-8 of the unfiltered
 *   weight); cheaper to evaluate (mostly binary32 work instead of binary64).
 *   The frequencies are the same in both modes.
 * Errors: n <= 0 or n > QRFS_MAX_POINTS_PER_CALL; NULL arrays; r0 <= 0;
 * von Karman L0 <= 0; unknown model; ap with D <= 0, d < 0 or d >= D;
 * unknown precision. */
QRFS_API qrfs_status qrfs_weights(qrfs_context* ctx, const qrfs_psd* psd, const qrfs_aperture* ap,
                         int64_t n, const double* fx, const double* fy, const double* area,
                         int32_t precision, double* w, void* stream);

/* qrfs_sample_frequencies followed by qrfs_weights in one pass, for callers
 * that need the frequencies and their weights but not the cell areas
 * (Sec. 3.2, Eqs. 5-7): writes fx, fy (cycles/m) and w, all
 * double[n_sets*K], set-major, with the same values the two calls give
 * (the same precision argument).  ap == NULL: phase weights; else the filter
 * of equal apertures is folded in.  The learned sampler keeps its cell areas
 * in the context's workspace (grown to n_sets*K doubles if needed).
 * s->index += n_sets*K on success.
 * Errors: as qrfs_sample_frequencies and qrfs_weights. */
QRFS_API qrfs_status qrfs_sample_weights(qrfs_context* ctx, qrfs_sampler* s, int64_t n_sets,
                                         int64_t K, const qrfs_psd* psd, const qrfs_aperture* ap,
                                         int32_t precision, double* fx, double* fy, double* w,
                                         void* stream);

/* Hyper-parameters of the Cartesian sampler (Sec. 4.3), host-only (no
 * device work, no context): with g(x) = int_0^x f W(f) F(f)^2 df (F the
 * filter of ap, 1 when ap is NULL), the smallest max|f| = n* df beyond which
 * every increment g(n df) - g((n-1) df) stays below eps g(inf) (eps
 * relative to the saturated variance, the paper's eps << sigma^2); returns
 * *N = 2 n* (N df = 2 max|f|), *df_out the pitch used (df <= 0 selects the
 * paper's 0.25 / L0) and, when sigma2 is not NULL, the variance
 * 2 pi g(inf) (rad^2, of the piston when ap is given).
 * Errors: Kolmogorov model (g diverges at f = 0: QRFS_ERR_UNSUPPORTED);
 * r0, L0 <= 0; eps outside (0, 1); bad aperture; NULL N or df_out;
 * more than 2^31 steps; QRFS_ERR_NOT_CONVERGED when the increments are
 * still at or above eps g(inf) at the integration limit (200/D, or
 * 2000/L0 without an aperture), i.e. eps is below what the rule can
 * resolve there (*N, *df_out and *sigma2 are then left unchanged). */
QRFS_API qrfs_status qrfs_choose_cartesian(const qrfs_psd* psd, const qrfs_aperture* ap,
                                           double df, double eps, int32_t* N, double* df_out,
                                           double* sigma2);

/* Phase field, Eq. 3: phase[r][p] = phi_r(px[p], py[p]) for r < R, p < P.
 * fx, fy, w: double[n_sets][K] (n_sets = ceil(R/R_block)); px, py:
 * double[P]; coef: NULL to draw the coefficients with rng (rng then
 * required), or double[R][2K] (c[2k] = a, c[2k+1] = b) supplied by the
 * caller (rng ignored).  phase: double[R][P] for QRFS_PREC_FP64, float[R][P]
 * otherwise (row-major).
 * Errors: K, P, R <= 0; R_block outside [1, R]; NULL arrays; unknown
 * precision; rng NULL with coef NULL; unknown coefficient mode. */
QRFS_API qrfs_status qrfs_synthesize_phase(qrfs_context* ctx, int64_t K, const double* fx,
                                  const double* fy, const double* w, int64_t P,
                                  const double* px, const double* py, int64_t R,
                                  int64_t R_block, const qrfs_rng* rng, const double* coef,
                                  int32_t precision, void* phase, void* stream);

/* Aperture pistons (Sec. 4.1): the phase averaged over aperture j (centre
 * cx[j], cy[j], diameters apD[j] > apd[j] >= 0) equals the harmonic sum with
 * each frequency multiplied by that aperture's filter F (Eq. 7), evaluated
 * at the centre.  w is the UNFILTERED phase weight.  piston: [R][n_ap],
 * double for FP64, float otherwise.  Other arguments as
 * qrfs_synthesize_phase.  Extra errors: n_ap <= 0; NULL apD/apd. */
QRFS_API qrfs_status qrfs_piston(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                        const double* w, int64_t n_ap, const double* cx, const double* cy,
                        const double* apD, const double* apd, int64_t R, int64_t R_block,
                        const qrfs_rng* rng, const double* coef, int32_t precision,
                        void* piston, void* stream);

/* Angle of arrival (G-tilt): the phase gradient averaged over each aperture,
 * along the direction (ux, uy), in rad/m (times lambda / (2 pi) for the
 * angle in radians).  Sec. 2 counts angle-of-arrival fluctuations among the
 * linear functionals of the phase the method simulates; the average of the
 * gradient over the aperture is the gradient of the piston with respect to
 * the centre, so differentiating Eq. 3 with the filter of Eq. 7 gives
 *   tilt[r][j] = sum_k w_k F_j(|f_k|) 2 pi (u.f_k)
 *                (b_rk cos 2 pi f_k.c_j - a_rk sin 2 pi f_k.c_j).
 * (ux, uy) need not be a unit vector (the result scales with it).  Arguments,
 * layouts and errors as qrfs_piston; extra error: (ux, uy) zero or not
 * finite. */
QRFS_API qrfs_status qrfs_tilt(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                      const double* w, int64_t n_ap, const double* cx, const double* cy,
                      const double* apD, const double* apd, double ux, double uy, int64_t R,
                      int64_t R_block, const qrfs_rng* rng, const double* coef,
                      int32_t precision, void* tilt, void* stream);

/* Differential pistons between two equal apertures, one at the origin and
 * one at baseline b (Sec. 4.4): dp[r][b] = p_r(bx[b], by[b]) - p_r(0, 0),
 * evaluated directly as sum_k w_k [a (cos 2 pi f.B - 1) + b sin 2 pi f.B].
 * w must already carry the aperture filter (qrfs_weights with ap).
 * dp: [R][nB], double for FP64, float otherwise.  Other arguments and
 * errors as qrfs_synthesize_phase, with bx, by: double[nB] (device). */
QRFS_API qrfs_status qrfs_diff_piston(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                             const double* w, int64_t nB, const double* bx, const double* by,
                             int64_t R, int64_t R_block, const qrfs_rng* rng, const double* coef,
                             int32_t precision, void* dp, void* stream);

/* Differential-piston structure function (Sec. 4.4), end to end: draws
 * ceil(R/R_block) frequency sets of K points with the sampler (advancing
 * s->index by n_sets*K), weights them with the PSD and the aperture filter,
 * draws the coefficients with rng and returns, per baseline b,
 *   sf[b]        = (1/R) sum_r dp_rb^2                       (rad^2)
 *   sf_stderr[b] = sqrt( (sum dp^4 - (sum dp^2)^2 / R) / ((R-1) R) )
 * (the standard error of sf, NULL to skip).  dp never reaches memory; the
 * sums are accumulated in FP64 and reduced in a fixed order, so results are
 * bit-reproducible.  sf, sf_stderr: double[nB] (device).  bx, by: double[nB]
 * (device).  Errors: as qrfs_sample_frequencies, qrfs_weights (ap required)
 * and qrfs_synthesize_phase. */
QRFS_API qrfs_status qrfs_diff_piston_structure(qrfs_context* ctx, const qrfs_psd* psd,
                                       const qrfs_aperture* ap, int64_t nB, const double* bx,
                                       const double* by, qrfs_sampler* s, int64_t K, int64_t R,
                                       int64_t R_block, const qrfs_rng* rng, int32_t precision,
                                       double* sf, double* sf_stderr, void* stream);

/* Differential-piston structure function for caller-supplied frequency
 * sets: the same sums as qrfs_diff_piston_structure without the sampling and
 * weighting steps.  fx, fy, w: double[n_sets][K] (n_sets = ceil(R/R_block)),
 * w carrying the aperture filter; bx, by: double[nB]; sf, sf_stderr:
 * double[nB] (sf_stderr may be NULL); all device.  Errors as
 * qrfs_synthesize_phase. */
QRFS_API qrfs_status qrfs_diff_piston_structure_sets(qrfs_context* ctx, int64_t K,
                                                     const double* fx, const double* fy,
                                                     const double* w, int64_t nB,
                                                     const double* bx, const double* by,
                                                     int64_t R, int64_t R_block,
                                                     const qrfs_rng* rng, int32_t precision,
                                                     double* sf, double* sf_stderr,
                                                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as qrfs_diff_piston_structure_sets, with arguments, layouts and
 * errors as there, computed without any allocation.  Its scratch (per-tile
 * partial sums and split-K partials) is a static device array of 64 MiB
 * that each GPU the library runs on holds until the process ends; its
 * address on the context's device is looked up once, when the first
 * context on that device is created.  To fit, the sums may take fewer
 * frequency ranges (split-K) than qrfs_diff_piston_structure_sets would,
 * so results agree to rounding (bit-equal when the plan is the same).
 * Every call on one GPU shares that array: calls that overlap in time on
 * one GPU (other streams, threads or contexts) race; nothing in it needs
 * clearing between calls.  Extra error: a problem whose scratch exceeds
 * 64 MiB even with one range (QRFS_ERR_INVALID_ARG).  With one range the
 * scratch is 16 nB bytes per row tile of a set (tiles of at most 128 rows;
 * one tile per set when R_block = 1), e.g. up to 131072 realisations of
 * 32 baselines at R_block = 1; larger problems are split over calls. */
QRFS_API qrfs_status qrfs_diff_piston_structure_sets_noalloc(
    qrfs_context* ctx, int64_t K, const double* fx, const double* fy, const double* w,
    int64_t nB, const double* bx, const double* by, int64_t R, int64_t R_block,
    const qrfs_rng* rng, int32_t precision, double* sf, double* sf_stderr, void* stream);

/* ----------------------------------------------- frozen-flow time series */
/* Temporal structure function of the differential piston (the statistical
 * test of Sec. 4.4): pistons [R][2][M] hold, per realisation, the pistons of
 * telescopes 1 and 2 at times t_m = m dt (double for QRFS_PREC_FP64, float
 * otherwise; device).  For lag j, each realisation contributes the mean over
 * its M - j pairs of (dp(t_m + j dt) - dp(t_m))^2, dp = p1 - p2; sf[j] is
 * the mean over realisations, sf_stderr[j] its standard error (sample
 * standard deviation / sqrt R; NULL to skip), both double[M] (device,
 * rad^2; sf[0] = 0).  Accumulated in FP64, reduced in a fixed order.
 * Errors: R < 1; M outside [1, 4096]; NULL or misaligned arrays; unknown
 * precision. */
QRFS_API qrfs_status qrfs_temporal_sf(qrfs_context* ctx, int64_t R, int64_t M, int32_t precision,
                                      const void* pistons, double* sf, double* sf_stderr,
                                      void* stream);

/* The experiment of Sec. 4.4 end to end under frozen flow (Taylor): the
 * turbulence moves with velocity v (m/s), so at time t the telescope at c
 * sees the screen at c - v t.  Draws ceil(R/R_block) frequency sets of K
 * points with the sampler (advancing s->index by n_sets*K), weights them
 * with the PSD and the filter of the equal apertures ap (Eq. 7), evaluates
 * the pistons of Eq. 3 at c1 - v t_m and c2 - v t_m (t_m = m dt, m < M) for
 * R realisations (coefficients from rng) and returns the temporal structure
 * function of qrfs_temporal_sf.  c1, c2, v: host double[2] (m, m/s).
 * The pistons equal qrfs_synthesize_phase with the filtered weights at
 * those 2M points.  Errors: as qrfs_diff_piston_structure (ap required),
 * M outside [1, 4096], dt negative or not finite, NULL c1/c2/v. */
QRFS_API qrfs_status qrfs_temporal_piston_structure(
    qrfs_context* ctx, const qrfs_psd* psd, const qrfs_aperture* ap, const double* c1,
    const double* c2, const double* v, double dt, int64_t M, qrfs_sampler* s, int64_t K,
    int64_t R, int64_t R_block, const qrfs_rng* rng, int32_t precision, double* sf,
    double* sf_stderr, void* stream);

/* --------------------------------------------------- sampler comparison */
/* Point-set measures of frequency sets, the properties Sec. 3.1-3.2 weigh
 * the samplers by: frequencies that "clash" (fall almost on top of each
 * other), gaps, and even coverage.  Set s is fx, fy [s*K, (s+1)*K), mapped
 * to the unit square by u = ((fx - x0)/Lx, (fy - y0)/Ly) (for the Cartesian
 * and jittered schemes x0 = y0 = -N df/2, Lx = Ly = N df).  Per set:
 *   min_dist[s]  smallest distance |u_i - u_j| over its pairs (+inf for K=1),
 *   n_clash[s]   number of pairs with |u_i - u_j| < r_clash,
 *   l2_star[s]   L2 star discrepancy T of the points in [0,1]^2 (Warnock):
 *     T^2 = 1/9 - (1/(2K)) sum_i (1 - x_i^2)(1 - y_i^2)
 *           + (1/K^2) sum_{i,j} (1 - max(x_i, x_j)) (1 - max(y_i, y_j)).
 * Distances are formed in FP64 without fused multiply-adds, so min_dist and
 * n_clash are those of the plain definition exactly; the sums run in FP64
 * in a fixed order (bit-reproducible).  O(K^2) work per set.
 * fx, fy: device double[n_sets*K]; min_dist, l2_star: device double[n_sets];
 * n_clash: device int64[n_sets].  Uses the context's workspace.
 * Errors: n_sets, K < 1; K > 2^24; n_sets * ceil(K/256) >= 2^24; Lx, Ly not
 * > 0 or x0, y0 not finite; r_clash < 0; NULL or misaligned arrays. */
QRFS_API qrfs_status qrfs_point_set_measures(qrfs_context* ctx, int64_t n_sets, int64_t K,
                                             const double* fx, const double* fy, double x0,
                                             double y0, double Lx, double Ly, double r_clash,
                                             double* min_dist, int64_t* n_clash, double* l2_star,
                                             void* stream);

/* Noise-free differential-piston structure function of each frequency set:
 * given the set, the coefficients are iid N(0, 1), so p(B) - p(0) is
 * N(0, S) with
 *   S[s][b] = sum_k w_k^2 2 (1 - cos 2 pi f_k.B_b)
 * (w carrying the aperture filter of Eq. 7, as qrfs_weights gives it with
 * an aperture).  Its relative error against the analytic curve is the
 * sampling error of the set alone (no coefficient noise), the quantity the
 * samplers are compared on.  Formed as w^2 4 sin^2(pi r), r = f.B reduced
 * to [-1/2, 1/2] in FP64; FP64 sums in a fixed order.
 * fx, fy, w: device double[n_sets*K]; bx, by: device double[nB];
 * S: device double[n_sets][nB].
 * Errors: K, n_sets, nB < 1; n_sets >= 2^24; NULL or misaligned arrays. */
QRFS_API qrfs_status qrfs_set_sf_expectation(qrfs_context* ctx, int64_t K, const double* fx,
                                             const double* fy, const double* w, int64_t n_sets,
                                             int64_t nB, const double* bx, const double* by,
                                             double* S, void* stream);

/* ------------------------------------------------------ learned proposal */
/* A proposal density for the frequency sampler, learned from the variance
 * contributions the plain method generates (the paper leaves the choice of
 * the sampling to the user and suggests a PSD-aware mapping, Sec. 5):
 *   q(ell, theta) = p(ell) (1 + alpha(ell) cos 2(theta - theta_B)) / (2 pi),
 * ell = ln|f| in [ln fmin, ln fmax], p proportional to exp(o0),
 * alpha = 0.9 tanh(o1), o = network(2 (ell - ln fmin)/Lw - 1,
 * 2 theta_B/pi - 1, ln D / 4, ln L0 / 4 - 1, ln|B| / 4 - 1/2),
 * Lw = ln(fmax/fmin), network 5 -> 128 (tanh) -> 128 (tanh) -> 2 with flat
 * FP32 parameters W1[128][5], b1[128], W2[128][128], b2[128], W3[2][128],
 * b3[2] (QRFS_PROPOSAL_NPARAM floats).  Training minimises the
 * cross-entropy -sum h log q / sum h toward the contributions h of plain
 * samples, with p normalised on a G-point midpoint grid; Adam (Kingma & Ba).
 * The sampling table is piecewise constant on n_cells cells: the mixture of
 * the per-baseline densities of a target geometry plus a defensive share
 * beta of the plain density, so q > 0 everywhere. */
#define QRFS_PROPOSAL_NPARAM 17538
#define QRFS_PROPOSAL_MAX_CELLS 1024
typedef struct qrfs_proposal qrfs_proposal;

/* Creates a proposal over [fmin, fmax] with the given initial parameters
 * (device float[QRFS_PROPOSAL_NPARAM], copied); Adam moments start at 0. */
QRFS_API qrfs_status qrfs_proposal_create(qrfs_context* ctx, double fmin, double fmax,
                                          const float* init_params, qrfs_proposal** out);
QRFS_API qrfs_status qrfs_proposal_destroy(qrfs_proposal* p);
/* Device-to-device copies of the parameters (float[QRFS_PROPOSAL_NPARAM]). */
QRFS_API qrfs_status qrfs_proposal_get_params(const qrfs_proposal* p, float* dst, void* stream);
QRFS_API qrfs_status qrfs_proposal_set_params(qrfs_proposal* p, const float* src, void* stream);
/* Network outputs out[n][2] (o0, o1) for rows ell[n] with contexts
 * ctx4[n][4] = (D, L0, |B|, theta_B); all device.  1 <= n <= 2^30 - 2^16. */
QRFS_API qrfs_status qrfs_proposal_forward(qrfs_proposal* p, int64_t n, const double* ell,
                                           const double* ctx4, float* out, void* stream);
/* Training rows from the plain log-polar sampler `plain` (advanced by
 * n_ctx*m): context c (ctx4[c], device [n_ctx][4]) owns rows c*m .. c*m+m-1
 * with ell, theta and the contribution
 * h = f^2 W(f) F_D(f)^2 2 (1 - cos(2 pi f |B| cos(theta - theta_B)))
 * of a von Karman PSD with Fried parameter r0 (c_psd <= 0: exact constant)
 * and outer scale L0 of the context.  Outputs device double[n_ctx*m];
 * n_ctx * m <= QRFS_MAX_POINTS_PER_CALL. */
QRFS_API qrfs_status qrfs_proposal_rows(qrfs_proposal* p, qrfs_sampler* plain, int64_t n_ctx,
                                        int64_t m, const double* ctx4, double r0, double c_psd,
                                        double* ell, double* theta, double* h, void* stream);
/* Loss and its gradient for all n_ctx contexts of a training set (the
 * training step's computation, exposed for checking): grad device
 * float[QRFS_PROPOSAL_NPARAM], loss device double[1].  G: normaliser grid
 * points (1..4096).  n_ctx <= 1024, n_ctx * m <= 2^29. */
QRFS_API qrfs_status qrfs_proposal_loss_grad(qrfs_proposal* p, int64_t n_ctx, int64_t m,
                                             const double* ctx4, const double* ell,
                                             const double* theta, const double* h, int32_t G,
                                             float* grad, double* loss, void* stream);
/* `steps` Adam steps (learning rate lr) on mini-batches of ctx_per_step
 * contexts (<= 1024, ctx_per_step * m <= 2^29) taken in an order
 * reshuffled every epoch from shuffle_seed; loss_log: device double[steps]
 * or NULL. */
QRFS_API qrfs_status qrfs_proposal_train(qrfs_proposal* p, int64_t n_ctx, int64_t m,
                                         const double* ctx4, const double* ell,
                                         const double* theta, const double* h,
                                         int64_t ctx_per_step, int64_t steps, int32_t G,
                                         double lr, uint64_t shuffle_seed, double* loss_log,
                                         void* stream);
/* Builds the sampling table for aperture D, outer scale L0 and nB
 * baselines of length blen[b] and direction bth[b] (host arrays), with
 * n_cells (1..QRFS_PROPOSAL_MAX_CELLS) cells and defensive share beta in
 * (0, 1]. */
QRFS_API qrfs_status qrfs_proposal_tabulate(qrfs_proposal* p, double D, double L0, int64_t nB,
                                            const double* blen, const double* bth,
                                            int32_t n_cells, double beta, void* stream);
/* Table access (device double[n_cells] each): density p of ln|f| per cell,
 * alpha, phi (angular factor 1 + alpha cos 2(theta - phi)), cdf at the
 * cell's left edge.  set_table replaces the table (cdf[0] = 0, increasing,
 * p > 0, |alpha| < 1 are the caller's responsibility). */
QRFS_API qrfs_status qrfs_proposal_get_table(const qrfs_proposal* p, int32_t* n_cells,
                                             double* tp, double* talpha, double* tphi,
                                             double* tcdf, void* stream);
QRFS_API qrfs_status qrfs_proposal_set_table(qrfs_proposal* p, int32_t n_cells, const double* tp,
                                             const double* talpha, const double* tphi,
                                             const double* tcdf, void* stream);
/* Parameters to / from a file: 8-byte magic "QRFSPRP1", fmin, fmax (double),
 * QRFS_PROPOSAL_NPARAM floats (little-endian).  Synchronises the device. */
QRFS_API qrfs_status qrfs_proposal_save(const qrfs_proposal* p, const char* path);
QRFS_API qrfs_status qrfs_proposal_load(qrfs_proposal* p, const char* path);

/* ------------------------------------------------------ batched launches */
/* Many uneven instances in one persistent launch: the phase of Eq. 3 at
 * each instance's points, as qrfs_synthesize_phase computes it, or, for an
 * instance that brings aperture diameters, the pistons of apertures
 * (filled or annular) centred at the points, as qrfs_piston computes them,
 * or their G-tilts along (ux, uy), as qrfs_tilt computes them.
 * Each instance brings its own PSD, sampler (the instance draws
 * ceil(R/R_block) sets of K frequencies starting at sampler.index), points,
 * realisations and output.  The batch owns the frequency buffers; executing
 * it runs, on one stream: per instance the sampler and the weights, then one
 * persistent kernel whose blocks pull (instance, set, row tile, column tile)
 * work items, longest first, from a device counter.  Executions replay the
 * same draws (sampler indices and rng counters are not advanced).
 * Pointers inside an instance must stay valid until qrfs_batch_destroy. */
typedef struct {
    qrfs_psd psd;         /* phase PSD of the instance                  */
    qrfs_sampler sampler; /* R2 placement; LEARNED is not accepted      */
    int64_t K;            /* frequencies per set                        */
    int64_t P;            /* points                                     */
    const double* px;     /* device double[P]                           */
    const double* py;     /* device double[P]                           */
    int64_t R;            /* realisations                               */
    int64_t R_block;      /* realisations per frequency set, in [1, R]  */
    qrfs_rng rng;         /* coefficient stream (GAUSS_CS or EQ3)       */
    float* phase;         /* device float[R][P] output (phase, pistons
                             or tilts)                                  */
    const double* apD;    /* NULL: phase at the points; else device
                             double[P] outer diameters D > 0 of the
                             apertures centred at the points            */
    const double* apd;    /* with apD: device double[P] inner diameters
                             0 <= d < D (0: filled); NULL otherwise     */
    double ux, uy;        /* with apD: (0, 0) for pistons, else the
                             direction of the G-tilt; 0 without apD     */
} qrfs_batch_instance;

typedef struct qrfs_batch qrfs_batch;

/* Builds the work list of n instances (host array, copied).  precision:
 * QRFS_PREC_FP32, QRFS_PREC_SPLIT_BF16, QRFS_PREC_BF16X6 or QRFS_PREC_FP16X3
 * (FP64 -> QRFS_ERR_UNSUPPORTED).  Allocates the batch's device buffers.
 * Errors: n <= 0 or > 65535, any instance invalid as for
 * qrfs_synthesize_phase / qrfs_sample_frequencies / qrfs_weights /
 * qrfs_piston / qrfs_tilt; apD and apd not both NULL or both set; a
 * direction without apertures; a direction not finite. */
QRFS_API qrfs_status qrfs_batch_create(qrfs_context* ctx, int64_t n,
                                       const qrfs_batch_instance* inst, int32_t precision,
                                       qrfs_batch** out);
/* Launch shapes: 0-3 fused (each block draws its coefficients in registers;
 * rows and columns per block, resident blocks per CU), 4 two-phase (each
 * instance's coefficients drawn once into tiles the batch allocates on first
 * use, at most 16 GiB in all, then 256 x 256 items on one block per CU).
 * A new batch starts on shape 4 when its tiles fit, else on shape 0. */
#define QRFS_BATCH_SHAPES 5
/* Times every candidate launch shape on this batch and keeps the fastest;
 * synchronises the stream.  best_ms (host, may be NULL) receives its time
 * in ms.  cache_path (host string, may be NULL): a text file of earlier
 * choices, one line "qrfs-autotune-1 <key> <shape> <ms>" per tuned batch,
 * the key a 64-bit hash (hex) of the device's architecture name and compute
 * unit count, the precision and every instance's K, P, R, R_block and
 * aperture/tilt flags.  When the file holds the key, its (last) shape is
 * selected without timing and its ms returned; otherwise the batch is timed
 * and a line appended.  A missing file is an empty cache.
 * Errors: NULL batch; the cache file cannot be appended to
 * (QRFS_ERR_INVALID_ARG, after the tuned shape was selected); HIP errors. */
QRFS_API qrfs_status qrfs_batch_autotune(qrfs_batch* b, void* stream, const char* cache_path,
                                         double* best_ms);
/* Selects launch shape `shape` (an implementation knob, for callers that
 * tune offline).  Errors: shape outside [0, QRFS_BATCH_SHAPES); the
 * two-phase shape when its tiles exceed the cap (QRFS_ERR_UNSUPPORTED);
 * allocation failure of the tiles (QRFS_ERR_OUT_OF_MEMORY). */
QRFS_API qrfs_status qrfs_batch_set_shape(qrfs_batch* b, int32_t shape);
/* Enqueues one execution on `stream`.  use_graph != 0: the first call
 * captures the whole sequence in a HIP graph (re-captured after an autotune
 * changes the shape), later calls replay it. */
QRFS_API qrfs_status qrfs_batch_execute(qrfs_batch* b, int32_t use_graph, void* stream);
/* Host outputs (each may be NULL): number of work items, chosen shape
 * index, total terms R*K*P of one execution. */
QRFS_API qrfs_status qrfs_batch_info(const qrfs_batch* b, int64_t* n_items, int32_t* shape,
                                     double* terms);
/* Synchronises the device and frees the batch.  NULL is accepted. */
QRFS_API qrfs_status qrfs_batch_destroy(qrfs_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* QRFS_H */
