// qrfs_device.hpp -- device-side building blocks of the quasi-random
// frequency sampling path (arXiv 2404.02978) for gfx950.
//
// Everything here is written for CDNA4 directly: 64-lane wavefronts, the
// revolution-domain hardware sine/cosine (v_sin_f32 / v_cos_f32 take x and
// return sin(2 pi x)), FP64 vector arithmetic at full rate, and the
// 32x32 MFMA operand layouts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrfs {

// a * b + c in binary64 with the constant c taken from a scalar register
// pair.  Polynomial steps written as fma() compile to v_fmac_f64, whose
// addend is the destination: every constant coefficient then costs two
// v_mov_b32 on the vector ALU before its FMA.  A v_fma_f64 reads the
// coefficient from scalar registers that s_mov loads (scalar ALU, beside
// the vector work): one vector instruction per step.
__device__ __forceinline__ double fma_s(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// ---------------------------------------------------------------- R2 ----
// Weyl increments of the 2-D R2 sequence (Sec. 3.2, Eq. 6):
// round(2^64 / psi) and round(2^64 / psi^2), psi = 1.3247179572447460...
// the real root of x^3 = x + 1.
constexpr uint64_t kR2IncX = 0xC13FA9A902A6328FULL;
constexpr uint64_t kR2IncY = 0x91E10DA5C79E7B1DULL;

// A 0.64 fixed-point coordinate as the double (U >> 11) 2^-53 in [0, 1):
// the high word times 2^-32 plus the low word without its 11 low bits times
// 2^-64, both exact, and their sum has 53 significant bits, so the one
// rounding of the fma is exact.
__device__ __forceinline__ double r2_coord(uint64_t U) {
    uint32_t hw = (uint32_t)(U >> 32);
    // a plain 32-bit word to the conversion (seen as the top half of a
    // 64-bit value, it is converted as one, with an extra add of zero)
    asm("" : "+v"(hw));
    const double hi = (double)hw;
    const double lo = (double)((uint32_t)U & 0xfffff800u);
    return fma(hi, 0x1p-32, lo * 0x1p-64);
}

// Point n (n >= 1) of the sequence started at (s0x, s0y) in 0.64 fixed
// point, as doubles in [0,1) carrying the top 53 bits.
__device__ __forceinline__ void r2_point(uint64_t s0x, uint64_t s0y, uint64_t n, double& ux,
                                         double& uy) {
    ux = r2_coord(s0x + n * kR2IncX);
    uy = r2_coord(s0y + n * kR2IncY);
}

// --------------------------------------------------------------- Philox ----
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The 32x32->64 products
// map onto v_mad_u64_u32; the key schedule is wave-uniform and stays scalar;
// each round's two three-way xors are one v_bitop3_b32 each (truth table
// 0x96 is the parity of the three inputs), not two v_xor_b32.
struct U32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U32x4{c0, c1, c2, c3};
}

// Block t of realisation `real` under key `seed`: counter (t, real lo, real hi, 0).
__device__ __forceinline__ U32x4 coef_block(uint64_t seed, uint64_t real, uint32_t t) {
    return philox4x32_10(t, (uint32_t)real, (uint32_t)(real >> 32), 0u, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// Unit-square point n of the pseudo-random frequency stream (the randomised
// samplers of Sec. 3.1): one block keyed by seed_x with counter
// (n lo, n hi, low word of seed_y, 0x46524551).  Coefficient counters end
// in a zero word, so the two streams never share a block.  Each coordinate
// is the top 53 bits of a word pair ((y:x) and (w:z)) times 2^-53.
__device__ __forceinline__ void pseudo_point(uint64_t seed_x, uint64_t seed_y, uint64_t n,
                                             double& ux, double& uy) {
    const U32x4 r = philox4x32_10((uint32_t)n, (uint32_t)(n >> 32), (uint32_t)seed_y,
                                  0x46524551u, (uint32_t)seed_x, (uint32_t)(seed_x >> 32));
    const uint64_t a = ((uint64_t)r.y << 32) | r.x;
    const uint64_t b = ((uint64_t)r.w << 32) | r.z;
    ux = (double)(a >> 11) * 0x1p-53;
    uy = (double)(b >> 11) * 0x1p-53;
}

// 32-bit word -> (2m+1) 2^-24 with m = x >> 9: exact in binary32, in (0,1).
// One funnel shift places m under the exponent of 1.0 (the bit pattern of
// 1 + m 2^-23), and subtracting 1 - 2^-24 is exact (the difference has at
// most 24 significant bits).
__device__ __forceinline__ float word_uniform_f32(uint32_t x) {
    const uint32_t one_m = __builtin_amdgcn_alignbit(0x7fu, x, 9u);  // (x >> 9) | 0x3f800000
    return __uint_as_float(one_m) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double word_uniform_f64(uint32_t x) {
    return ((double)(x >> 9) + 0.5) * 0x1p-23;
}

// sin and cos of 2 pi u for u = (2m + 1) 2^-24 in (0,1), exact in binary32:
// the hardware revolution-domain sine/cosine take u as it is; over all 2^23
// such u their largest error against sin and cos of 2 pi u in binary64 is
// 1.25e-7 absolute on MI355X, the same as for the shifted u - 1/2.
__device__ __forceinline__ void sincos2pi_unit_f32(float u, float& s, float& c) {
    s = __builtin_amdgcn_sinf(u);
    c = __builtin_amdgcn_cosf(u);
}

// Box-Muller on binary32: (u1, u2) -> rho (cos 2 pi u2, sin 2 pi u2),
// rho = sqrt(-2 ln u1) = sqrt(-2 ln2 log2 u1).
__device__ __forceinline__ void box_muller_f32(float u1, float u2, float& g0, float& g1) {
    // the argument lies in [1.2e-7, 33.3] (normal), where the raw
    // v_sqrt_f32 is within 1 ulp
    float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    float s, c;
    sincos2pi_unit_f32(u2, s, c);
    g0 = rho * c;
    g1 = rho * s;
}

// The same coefficients divided by sqrt(2 ln 2): rho / sqrt(2 ln 2) =
// sqrt(-log2 u1) needs no product (the negation is a free input modifier);
// kernels that multiply every coefficient by an amplitude fold the factor
// kBoxMullerLog2 into it.
constexpr double kBoxMullerLog2 = 1.1774100225154747;  // sqrt(2 ln 2)
__device__ __forceinline__ void gauss4_f32_log2(uint64_t seed, uint64_t real, uint32_t t,
                                                float g[4]) {
    U32x4 x = coef_block(seed, real, t);
    float s, c;
    float rho = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(word_uniform_f32(x.x)));
    sincos2pi_unit_f32(word_uniform_f32(x.y), s, c);
    g[0] = rho * c;
    g[1] = rho * s;
    rho = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(word_uniform_f32(x.z)));
    sincos2pi_unit_f32(word_uniform_f32(x.w), s, c);
    g[2] = rho * c;
    g[3] = rho * s;
}

// Four consecutive coefficients c[4t .. 4t+3] of one realisation
// (Gaussian cos/sin mode), binary32.
__device__ __forceinline__ void gauss4_f32(uint64_t seed, uint64_t real, uint32_t t, float g[4]) {
    U32x4 x = coef_block(seed, real, t);
    box_muller_f32(word_uniform_f32(x.x), word_uniform_f32(x.y), g[0], g[1]);
    box_muller_f32(word_uniform_f32(x.z), word_uniform_f32(x.w), g[2], g[3]);
}

// Eq. 3 mode for frequency k: (a, b) = sqrt2 R_n (cos 2 pi R_u, -sin 2 pi R_u).
__device__ __forceinline__ void eq3_pair_f32(uint64_t seed, uint64_t real, uint32_t k, float& a,
                                             float& b) {
    U32x4 x = coef_block(seed, real, k);
    float rn, unused;
    box_muller_f32(word_uniform_f32(x.x), word_uniform_f32(x.y), rn, unused);
    float s, c;
    sincos2pi_unit_f32(word_uniform_f32(x.z), s, c);
    a = 1.4142135623730951f * rn * c;
    b = -1.4142135623730951f * rn * s;
}

// Coefficients c[4t .. 4t+3] in either mode (mode is wave-uniform).
__device__ __forceinline__ void coef4_f32(uint64_t seed, uint64_t real, uint32_t t, int mode,
                                          float g[4]) {
    if (mode == 0) {
        gauss4_f32(seed, real, t, g);
    } else {
        eq3_pair_f32(seed, real, 2u * t, g[0], g[1]);
        eq3_pair_f32(seed, real, 2u * t + 1u, g[2], g[3]);
    }
}

// binary64 versions (FP64 path).
__device__ __forceinline__ void box_muller_f64(double u1, double u2, double& g0, double& g1) {
    double rho = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    g0 = rho * c;
    g1 = rho * s;
}

__device__ __forceinline__ void coef4_f64(uint64_t seed, uint64_t real, uint32_t t, int mode,
                                          double g[4]) {
    if (mode == 0) {
        U32x4 x = coef_block(seed, real, t);
        box_muller_f64(word_uniform_f64(x.x), word_uniform_f64(x.y), g[0], g[1]);
        box_muller_f64(word_uniform_f64(x.z), word_uniform_f64(x.w), g[2], g[3]);
    } else {
        for (int h = 0; h < 2; ++h) {
            U32x4 x = coef_block(seed, real, 2u * t + (uint32_t)h);
            double rn, unused;
            box_muller_f64(word_uniform_f64(x.x), word_uniform_f64(x.y), rn, unused);
            double s, c;
            sincospi(2.0 * word_uniform_f64(x.z), &s, &c);
            g[2 * h] = 1.4142135623730951 * rn * c;
            g[2 * h + 1] = -1.4142135623730951 * rn * s;
        }
    }
}

// ------------------------------------------------------ PSD and filter ----
__device__ __forceinline__ double psd_phase(int model, double c, double r0_m53, double inv_L02,
                                            double f) {
    double q = f * f + (model == 1 ? inv_L02 : 0.0);
    if (q == 0.0) return 0.0;
    return c * r0_m53 * pow(q, -11.0 / 6.0);
}

// 2^y for |y| < 1000 in binary64: n = rint(y) comes off exactly and
// 2^r = e^(r ln 2), |r| <= 1/2, is its Taylor series through r^13 (first
// omitted term below 5e-18), summed by Horner's rule; then ldexp.  Within
// 2 ulp of 2^y; no general-purpose exp with its range handling.
constexpr double kExp2[14] = {
    1.0, 0.6931471805599453, 0.24022650695910072, 0.05550410866482158,
    0.009618129107628477, 0.0013333558146428443, 0.0001540353039338161, 1.5252733804059841e-05,
    1.321548679014431e-06, 1.01780860092397e-07, 7.054911620801123e-09, 4.4455382718708116e-10,
    2.5678435993488206e-11, 1.3691488853904128e-12};

__device__ __forceinline__ double exp2_poly(double y) {
    const double n = rint(y);
    const double r = y - n;
    double p = kExp2[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) p = fma_s(p, r, kExp2[k]);
    return ldexp(p, (int)n);
}

// sqrt(a) for a >= 0 in binary64 within 1 ulp: the hardware reciprocal
// square-root estimate, two Newton steps on it, then one correction of
// s = a y; 0 for a = 0.
__device__ __forceinline__ double sqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = fma(y, fma(-h, y * y, 0.5), y);
    y = fma(y, fma(-h, y * y, 0.5), y);
    const double s = a * y;
    const double r = fma(fma(-s, s, a), 0.5 * y, s);
    return a > 0.0 ? r : 0.0;
}

// sqrt(a) for a >= 0 to ~1e-14 relative (not correctly rounded): the
// binary32 reciprocal square root of a rounded to binary32, then one binary64
// Newton correction of s = a y; sqrt_nr outside the binary32 range.  For
// arguments that feed binary32-accuracy values (the FP32-class filter).
__device__ __forceinline__ double sqrt_f32_nr(double a) {
    if (!(a > 0x1p-120 && a < 0x1p120)) return sqrt_nr(a);
    const double y = (double)__builtin_amdgcn_rsqf((float)a);
    const double s = a * y;
    return fma(fma(-s, s, a), 0.5 * y, s);
}

// Fractional part of t to [-1/2, 1/2] in binary64 (exact).
__device__ __forceinline__ double frac_centered(double t) { return t - rint(t); }

// t - floor(t) in [0, 1) in binary64 (exact; one v_fract_f64), as binary32
// revolutions for the hardware sine and cosine, which only need t modulo 1
// (rounding error at most 2^-25 revolution).
__device__ __forceinline__ float frac_rev_f32(double t) {
    return (float)__builtin_amdgcn_fract(t);
}

// sin and cos of 2 pi r for an argument already reduced to |r| <= 1/2
// revolutions, in FP64: q = rint(4 r) quarter turns come off exactly
// (z = r - q/4, |z| <= 1/8, Sterbenz), the Taylor series of sin(2 pi z)
// through z^15 and of cos(2 pi z) through z^16 (first omitted terms below
// 7e-17 at |z| = 1/8) are summed by Horner's rule in z^2, and the quarter
// turns are put back by an exact rotation.  Coefficients
// (-1)^k (2 pi)^n / n!; max error 2e-16 (measured over [-1/2, 1/2]).
constexpr double kSin2pi[8] = {
    -0.71812230177850056, 3.819952584848282, -15.09464257682299, 42.058693944897655,
    -76.705859753061389, 81.605249276075057, -41.341702240399762, 6.2831853071795862};
constexpr double kCos2pi[9] = {
    0.28200596845579123, -1.714390711088672, 7.9035363713184692, -26.426256783374399,
    60.244641371876661, -85.456817206693728, 64.939394022668296, -19.739208802178716, 1.0};

__device__ __forceinline__ void sincos2pi_reduced(double r, double& s, double& c) {
    const double q = rint(4.0 * r);
    const double z = fma(-0.25, q, r);
    const double w = z * z;
    double ps = kSin2pi[0];
#pragma unroll
    for (int n = 1; n < 8; ++n) ps = fma_s(ps, w, kSin2pi[n]);
    ps *= z;
    double pc = kCos2pi[0];
#pragma unroll
    for (int n = 1; n < 9; ++n) pc = fma_s(pc, w, kCos2pi[n]);
    // the quarter turns: cos(pi q / 2) = 1 - |q| and sin(pi q / 2) =
    // q (1 - |cos|) for |q| <= 2; one factor is 0 and the other +-1, so
    // the rotation below is exact
    const double cq = 1.0 - fabs(q);
    const double sq = q * (1.0 - fabs(cq));
    s = fma(ps, cq, pc * sq);
    c = fma(pc, cq, -(ps * sq));
}

// J1(x) / x at x = pi t, t >= 0, for the aperture filter (Eq. 7): the
// project's own binary64 Bessel function, from two published forms with
// coefficients fitted by gen_bessel_j1.py (mpmath, 60 digits):
//   x < 8:  a polynomial of degree 16 in x^2 - 32 (a fit of the entire
//           function J1(sqrt z)/sqrt z, whose series is DLMF 10.2.2);
//   x >= 8: Hankel's form (DLMF 10.17.3), J1(x) = sqrt(2/(pi x))
//           (P cos chi - Q sin chi), chi = x - 3 pi/4, P and x Q / 8 as
//           polynomials of degree 8 in (8/x)^2; chi / (2 pi) = t/2 - 3/8 is
//           reduced exactly in revolutions (t = D f carries the argument
//           without a product by pi).
// Largest error against mpmath over t in [1e-4, 1e4]: 1.8e-15 in J1 (at
// x ~ 9).  About 20 vector operations below x = 8 and 60 above, against
// ~230 for the general-purpose j1.
constexpr double kJ1Small[17] = {
    -5.8143827955991070062e-2,
    2.5330831370593110909e-3,
    1.4796547991998664591e-4,
    -7.9222065822122274542e-6,
    1.5123726303789079841e-7,
    -1.6315525237574344594e-9,
    1.1601312451302481623e-11,
    -5.9052821439999382497e-14,
    2.2691399989608718142e-16,
    -6.8342128144214883067e-19,
    1.6595192217706221997e-21,
    -3.3215324568230986011e-24,
    5.5782364823880244287e-27,
    -7.9770548836205354222e-30,
    9.8345524159862802883e-33,
    -1.0600016054226224458e-35,
    1.0005202774655931299e-38};
constexpr double kJ1P[9] = {
    1.0000000000000063026,
    1.8310546864401147473e-3,
    -3.5203963650765904047e-5,
    2.5806706940751284167e-6,
    -4.0847900600833073724e-7,
    1.0716140721535631355e-7,
    -3.5134116038796300254e-8,
    9.9892867642288659536e-9,
    -1.5349264495380014555e-9};
constexpr double kJ1Q[9] = {
    4.6874999999994663438e-2,
    -2.0027160554483289392e-4,
    8.4709355706355412661e-6,
    -9.5031068997007103812e-7,
    2.0142935950325627865e-7,
    -6.4943179103018863123e-8,
    2.421946037301421181e-8,
    -7.3884944031697531349e-9,
    1.1785917506900844651e-9};

__device__ __forceinline__ double j1x_pi(double t) {
    const double x = 3.141592653589793 * t;
    if (x < 8.0) {
        const double z = fma(x, x, -32.0);
        double acc = kJ1Small[16];
#pragma unroll
        for (int n = 15; n >= 0; --n) acc = fma_s(acc, z, kJ1Small[n]);
        return acc;
    }
    // 1/x and 1/sqrt(x): hardware estimates and two Newton steps each
    // (relative error ~1e-16, no full-precision division or square root)
    double inv = __builtin_amdgcn_rcp(x);
    inv = fma(fma(-x, inv, 1.0), inv, inv);
    inv = fma(fma(-x, inv, 1.0), inv, inv);
    double rs = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    rs = fma(rs, fma(-hx, rs * rs, 0.5), rs);
    rs = fma(rs, fma(-hx, rs * rs, 0.5), rs);
    const double w = 64.0 * inv * inv;
    double p = kJ1P[8], q = kJ1Q[8];
#pragma unroll
    for (int n = 7; n >= 0; --n) {
        p = fma_s(p, w, kJ1P[n]);
        q = fma_s(q, w, kJ1Q[n]);
    }
    const double u = fma(0.5, t, -0.375);
    double sn, cs;
    sincos2pi_reduced(u - rint(u), sn, cs);
    // sqrt(2 / (pi x)) / x (P cos chi - Q sin chi), Q = 8 q / x
    return 0.79788456080286536 * rs * inv * fma(p, cs, -(8.0 * q * inv) * sn);
}

// Circular aperture filter with central obstruction (Eq. 7), signed:
// F = 2 (D^2 J1(pi D f)/(pi D f) - d^2 J1(pi d f)/(pi d f)) / (D^2 - d^2).
__device__ __forceinline__ double aperture_filter(double D, double d, double f) {
    if (f == 0.0) return 1.0;
    if (d > 0.0)
        return 2.0 * (D * D * j1x_pi(D * f) - d * d * j1x_pi(d * f)) / (D * D - d * d);
    return 2.0 * j1x_pi(D * f);
}

// J1(x)/x at x = pi t for values that end in binary32 (FP32-class weights
// and basis values), from the same two forms as j1x_pi with fewer terms
// (tables from gen_bessel_j1.py): below x = 8 the polynomial of degree 10
// in x^2 - 32, in binary64 (fit error 1.2e-10; as fast as binary32 here,
// and free of the cancellation its terms would show in binary32); above,
// Hankel's form with P and x Q / 8 of degree 3 in (8/x)^2 (fit error 6e-11)
// in binary32, the phase t/2 - 3/8 reduced exactly in binary64 and the
// hardware revolution sine and cosine.  Absolute error ~1e-8 (at x ~ 8,
// from the binary32 amplitude and phase), i.e. relative to F(0) = 1.
constexpr double kJ1Small10[11] = {
    -5.8143827959149801797e-2,
    2.5330830965939728592e-3,
    1.4796548014204885492e-4,
    -7.922205792102602279e-6,
    1.5123726050846113425e-7,
    -1.6315568427913620373e-9,
    1.1601322986993743466e-11,
    -5.9043187723429959103e-14,
    2.2689416857908308261e-16,
    -6.9281557493016852692e-19,
    1.6767143093134783333e-21};
constexpr float kJ1P3[4] = {1.0f, 1.83098991e-3f, -3.48635387e-5f, 1.97684287e-6f};
constexpr float kJ1Q3[4] = {4.68749991e-2f, -2.00242639e-4f, 8.31696171e-6f, -6.70713004e-7f};

__device__ __forceinline__ double j1x_pi_f32(double t) {
    const double x = 3.141592653589793 * t;
    if (x < 8.0) {
        const double z = fma(x, x, -32.0);
        double acc = kJ1Small10[10];
#pragma unroll
        for (int n = 9; n >= 0; --n) acc = fma_s(acc, z, kJ1Small10[n]);
        return acc;
    }
    const float xf = (float)x;
    const float inv = __builtin_amdgcn_rcpf(xf);
    const float w = 64.0f * inv * inv;
    float p = kJ1P3[3], q = kJ1Q3[3];
#pragma unroll
    for (int n = 2; n >= 0; --n) {
        p = fmaf(p, w, kJ1P3[n]);
        q = fmaf(q, w, kJ1Q3[n]);
    }
    const double u = fma(0.5, t, -0.375);
    const float r = (float)(u - rint(u));
    const float sn = __builtin_amdgcn_sinf(r), cs = __builtin_amdgcn_cosf(r);
    return (double)(0.79788456f * __builtin_amdgcn_rsqf(xf) * inv *
                    fmaf(p, cs, -(8.0f * q * inv) * sn));
}

// The filter with j1x_pi_f32, for the FP32-class paths (weights that feed
// binary32 sums, and the per-aperture basis values of pistons and tilts).
__device__ __forceinline__ float aperture_filter_f32(double D, double d, double f) {
    if (f == 0.0) return 1.0f;
    if (d > 0.0)
        return (float)(2.0 * (D * D * j1x_pi_f32(D * f) - d * d * j1x_pi_f32(d * f)) /
                       (D * D - d * d));
    return (float)(2.0 * j1x_pi_f32(D * f));
}



// Piston basis: the amplitude factor and the argument shift (cycles) that
// turn the piston into its gradient along u when `grad` is set, with
// (gx, gy) = 2 pi u (d/dc [a cos 2 pi f.c + b sin 2 pi f.c]
// = 2 pi (u.f) [b cos - a sin], the same pair a quarter cycle on);
// 1 and 0 otherwise.
__device__ __forceinline__ double grad_factor(int32_t grad, double gx, double gy, double fx,
                                              double fy) {
    return grad ? gx * fx + gy * fy : 1.0;
}
__device__ __forceinline__ double grad_shift(int32_t grad) { return grad ? 0.25 : 0.0; }

}  // namespace qrfs
