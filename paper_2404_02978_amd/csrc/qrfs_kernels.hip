// qrfs_kernels.hip -- gfx950 kernels of the quasi-random frequency sampling
// path (arXiv 2404.02978): the fused coefficient x basis contraction of
// Eq. 3 (FP64 vector ALU, FP32 MFMA, split-BF16 and BF16x6 MFMA), its
// epilogues and the fixed-order structure-function reduction.  The sampler
// and the weights live in qrfs_frequencies.hip.
#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"
#include "qrfs_mfma.hpp"

namespace qrfs {


// --------------------------------------------------- tile bookkeeping ----
struct TileInfo {
    int64_t sl;         // set index within the launch
    int64_t rt;         // row tile within the set
    int64_t ct;         // column tile
    int64_t row_begin;  // first row of the tile
    int64_t row_end;    // one past the last valid row of the set
};

__device__ __forceinline__ TileInfo decode_tile(const SumArgs& a, int64_t row_tiles,
                                                int64_t col_tiles, int64_t MT) {
    TileInfo t;
    int64_t b = blockIdx.x;
    t.ct = b % col_tiles;
    b /= col_tiles;
    t.rt = b % row_tiles;
    t.sl = b / row_tiles;
    int64_t s = a.set0 + t.sl;
    t.row_begin = s * a.R_block + t.rt * MT;
    int64_t se = (s + 1) * a.R_block;
    t.row_end = se < a.R ? se : a.R;
    return t;
}

// -------------------------------------------------- FP64 vector kernel ----
// Tile: 32 rows x 32 columns, 256 threads; thread (tp, tg) owns column tp
// and rows 4 tg .. 4 tg + 3.  Per chunk of 32 frequencies the block builds
// the FP64 coefficient tile and the FP64 basis tile in LDS, then every
// thread accumulates its 4 rows in FP64, frequency by frequency.
constexpr int F64_TP = 32;
constexpr int F64_TG = 8;
constexpr int F64_RPT = 4;
constexpr int F64_TR = F64_TG * F64_RPT;
constexpr int F64_KC = 32;

template <int BASIS, int EPI>
__global__ __launch_bounds__(256) void k_sum_f64(SumArgs a, int64_t row_tiles,
                                                 int64_t col_tiles) {
    __shared__ double sBc[F64_KC][F64_TP];
    __shared__ double sBs[F64_KC][F64_TP];
    __shared__ double sC[F64_TR][2 * F64_KC + 1];
    __shared__ double sfx[F64_KC], sfy[F64_KC], sw[F64_KC];
    __shared__ double spx[F64_TP], spy[F64_TP], sD[F64_TP], sd[F64_TP];
    __shared__ double sred[F64_TG][F64_TP][2];

    const int tid = threadIdx.x;
    const int tp = tid % F64_TP;
    const int tg = tid / F64_TP;
    const TileInfo ti = decode_tile(a, row_tiles, col_tiles, F64_TR);
    const int64_t col0 = ti.ct * F64_TP;
    if (tid < F64_TP) {
        int64_t p = col0 + tid;
        bool ok = p < a.P;
        spx[tid] = ok ? a.px[p] : 0.0;
        spy[tid] = ok ? a.py[p] : 0.0;
        if (BASIS == BASIS_PISTON) {
            sD[tid] = ok ? a.apD[p] : 1.0;
            sd[tid] = ok ? a.apd[p] : 0.0;
        }
    }
    const double* fx = a.fx + ti.sl * a.K;
    const double* fy = a.fy + ti.sl * a.K;
    const double* w = a.w + ti.sl * a.K;
    const int64_t twoK = 2 * a.K;

    double acc[F64_RPT];
#pragma unroll
    for (int q = 0; q < F64_RPT; ++q) acc[q] = 0.0;

    for (int64_t k0 = 0; k0 < a.K; k0 += F64_KC) {
        __syncthreads();
        if (tid < F64_KC) {
            int64_t k = k0 + tid;
            bool ok = k < a.K;
            sfx[tid] = ok ? fx[k] : 0.0;
            sfy[tid] = ok ? fy[k] : 0.0;
            sw[tid] = ok ? w[k] : 0.0;
        }
        // coefficients: 32 rows x 16 Philox blocks (4 coefficients each)
        for (int i = tid; i < F64_TR * (F64_KC / 2); i += 256) {
            int rr = i / (F64_KC / 2);
            int bt = i % (F64_KC / 2);
            int64_t r = ti.row_begin + rr;
            double g[4] = {0.0, 0.0, 0.0, 0.0};
            if (r < ti.row_end) {
                if (a.coef) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int64_t j = 2 * k0 + 4 * bt + q;
                        g[q] = j < twoK ? a.coef[r * twoK + j] : 0.0;
                    }
                } else {
                    coef4_f64(a.seed, a.counter + (uint64_t)r, (uint32_t)(k0 / 2 + bt), a.mode, g);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) sC[rr][4 * bt + q] = g[q];
        }
        __syncthreads();
        for (int i = tid; i < F64_KC * F64_TP; i += 256) {
            int kk = i / F64_TP;
            int pp = i % F64_TP;
            double t = sfx[kk] * spx[pp] + sfy[kk] * spy[pp];
            if (BASIS == BASIS_PISTON) t += grad_shift(a.grad);
            double rf = frac_centered(t);
            double s, c;
            if (BASIS == BASIS_DIFF) {
                // sin and cos of pi rf: cos 2 pi rf - 1 = -2 sin^2, sin 2 pi rf = 2 sin cos
                double sh, ch;
                sincos2pi_reduced(0.5 * rf, sh, ch);
                c = -2.0 * sh * sh;
                s = 2.0 * sh * ch;
            } else {
                sincos2pi_reduced(rf, s, c);
            }
            double amp = sw[kk];
            if (BASIS == BASIS_PISTON)
                amp *= aperture_filter(sD[pp], sd[pp], sqrt(sfx[kk] * sfx[kk] + sfy[kk] * sfy[kk])) *
                       grad_factor(a.grad, a.gx, a.gy, sfx[kk], sfy[kk]);
            sBc[kk][pp] = amp * c;
            sBs[kk][pp] = amp * s;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < F64_KC; ++kk) {
            double cb = sBc[kk][tp];
            double sb = sBs[kk][tp];
#pragma unroll
            for (int q = 0; q < F64_RPT; ++q) {
                const double* cr = sC[tg * F64_RPT + q];
                acc[q] = fma(cr[2 * kk], cb, fma(cr[2 * kk + 1], sb, acc[q]));
            }
        }
    }

    const int64_t col = col0 + tp;
    if (EPI == EPI_STORE) {
        double* out = (double*)a.out;
#pragma unroll
        for (int q = 0; q < F64_RPT; ++q) {
            int64_t r = ti.row_begin + tg * F64_RPT + q;
            if (r < ti.row_end && col < a.P) out[r * a.P + col] = acc[q];
        }
    } else {
        double s2 = 0.0, s4 = 0.0;
#pragma unroll
        for (int q = 0; q < F64_RPT; ++q) {
            int64_t r = ti.row_begin + tg * F64_RPT + q;
            if (r < ti.row_end) {
                double d2 = acc[q] * acc[q];
                s2 += d2;
                s4 += d2 * d2;
            }
        }
        sred[tg][tp][0] = s2;
        sred[tg][tp][1] = s4;
        __syncthreads();
        if (tid < F64_TP && col < a.P) {
            double t2 = 0.0, t4 = 0.0;
            for (int g = 0; g < F64_TG; ++g) {
                t2 += sred[g][tid][0];
                t4 += sred[g][tid][1];
            }
            double* dst = a.partial + ((ti.sl * row_tiles + ti.rt) * a.P + col) * 2;
            dst[0] = t2;
            dst[1] = t4;
        }
    }
}

// ------------------------------------------- FP64, narrow frequency sets ----
// Sets of at most 8 realisations (the paper draws fresh frequencies for
// every realisation: R_block = 1): one point per thread, RB rows per block.
// Per chunk of 64 frequencies the block stages fx, fy, w and the RB rows'
// coefficients in LDS (drawn once per block); each thread evaluates its
// point's basis once per frequency and adds it into its RB rows, in the
// same order and with the same fused products as k_sum_f64.  A 32-row tile
// would spend most of its contraction on rows the set does not have.
constexpr int F64N_KC = 64;

template <int BASIS, int RB>
__global__ __launch_bounds__(256) void k_sum_f64n(SumArgs a, int64_t col_tiles) {
    __shared__ double sfx[F64N_KC], sfy[F64N_KC], sw[F64N_KC];
    __shared__ double sC[RB][2 * F64N_KC];
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int64_t ct = (int64_t)blockIdx.x % col_tiles;
    const int64_t sl = (int64_t)blockIdx.x / col_tiles;
    const int64_t set = a.set0 + sl;
    const int64_t row_begin = set * a.R_block;
    const int64_t set_end = (set + 1) * a.R_block < a.R ? (set + 1) * a.R_block : a.R;
    const int64_t row_end = row_begin + RB < set_end ? row_begin + RB : set_end;
    const int64_t p = ct * nt + tid;
    const bool pok = p < a.P;
    const double px = pok ? a.px[p] : 0.0;
    const double py = pok ? a.py[p] : 0.0;
    double pD = 1.0, pd = 0.0;
    if (BASIS == BASIS_PISTON && pok) {
        pD = a.apD[p];
        pd = a.apd[p];
    }
    const double* fx = a.fx + sl * a.K;
    const double* fy = a.fy + sl * a.K;
    const double* w = a.w + sl * a.K;
    const int64_t twoK = 2 * a.K;
    double acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = 0.0;

    for (int64_t k0 = 0; k0 < a.K; k0 += F64N_KC) {
        __syncthreads();
        if (tid < F64N_KC) {
            const int64_t k = k0 + tid;
            const bool ok = k < a.K;
            sfx[tid] = ok ? fx[k] : 0.0;
            sfy[tid] = ok ? fy[k] : 0.0;
            sw[tid] = ok ? w[k] : 0.0;
        }
        // RB rows x 32 Philox blocks (4 coefficients each)
        for (int i = tid; i < RB * (F64N_KC / 2); i += nt) {
            const int rr = i / (F64N_KC / 2);
            const int bt = i % (F64N_KC / 2);
            const int64_t r = row_begin + rr;
            double g[4] = {0.0, 0.0, 0.0, 0.0};
            if (r < row_end) {
                if (a.coef) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t j = 2 * k0 + 4 * bt + q;
                        g[q] = j < twoK ? a.coef[r * twoK + j] : 0.0;
                    }
                } else {
                    coef4_f64(a.seed, a.counter + (uint64_t)r, (uint32_t)(k0 / 2 + bt), a.mode, g);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) sC[rr][4 * bt + q] = g[q];
        }
        __syncthreads();
        const int nk = a.K - k0 < F64N_KC ? (int)(a.K - k0) : F64N_KC;
        for (int kk = 0; kk < nk; ++kk) {
            double t = sfx[kk] * px + sfy[kk] * py;
            if (BASIS == BASIS_PISTON) t += grad_shift(a.grad);
            const double rf = frac_centered(t);
            double sv, cv;
            if (BASIS == BASIS_DIFF) {
                double sh, ch;
                sincos2pi_reduced(0.5 * rf, sh, ch);
                cv = -2.0 * sh * sh;
                sv = 2.0 * sh * ch;
            } else {
                sincos2pi_reduced(rf, sv, cv);
            }
            double amp = sw[kk];
            if (BASIS == BASIS_PISTON)
                amp *= aperture_filter(pD, pd, sqrt(sfx[kk] * sfx[kk] + sfy[kk] * sfy[kk])) *
                       grad_factor(a.grad, a.gx, a.gy, sfx[kk], sfy[kk]);
            const double cb = amp * cv, sb = amp * sv;
#pragma unroll
            for (int q = 0; q < RB; ++q)
                acc[q] = fma(sC[q][2 * kk], cb, fma(sC[q][2 * kk + 1], sb, acc[q]));
        }
    }
    double* out = (double*)a.out;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int64_t r = row_begin + q;
        if (r < row_end && pok) out[r * a.P + p] = acc[q];
    }
}

// --------------------------------------------------------- MFMA kernel ----
// One block = WV waves (WV = blockDim.x / 64: 1..4, or 8 for the difference
// basis of up to 32 baselines in the split precisions, so that one block
// covers 256 rows and each set's basis is built once per 256 rows).  Wave v
// owns rows [32 MW v, 32 MW (v+1)) of the tile and all NT = 32 NB columns,
// so each lane draws exactly the coefficients its own MFMA A-operand needs
// (no LDS traffic for coefficients) while the basis tile is shared through
// LDS.
// A block covers the frequency range [ks * kspan, (ks + 1) * kspan) of its
// rows (split K: several blocks per row tile keep the grid balanced when
// the rows alone do not fill the chip evenly).
//
// Per chunk of KC = 32 frequencies:
//   - every thread evaluates the basis for one frequency (the next chunk's
//     f, w are prefetched into registers one chunk ahead) and a few
//     columns: t = f.x in FP64, r = t - floor(t), hardware sin/cos of 2 pi r
//     in FP32, times the weight (and the aperture filter for pistons);
//     stored as [column][2 KC] floats (FP32) or as 16-bit hi and lo planes
//     (split modes) in one of two LDS buffers, so one barrier per chunk
//     suffices;
//   - each lane then draws all Philox blocks of the chunk (independent
//     integer chains the scheduler interleaves with the MFMAs);
//   - FP32: 32 steps of v_mfma_f32_32x32x2_f32.  Lane (r, h) holds the 4
//     coefficients of Philox block t = k0/2 + 2m + h, so step (m, q) uses
//     chunk-local contraction index j = 8m + 4h + q on both operands (the
//     contraction order is permuted, the result is not);
//   - split-BF16: 4 steps of v_mfma_f32_32x32x16_bf16 x 3 (hi.hi, hi.lo,
//     lo.hi), ~16 significant bits.  BF16x6: operands split three ways
//     (hi + mid + lo, 24 bits) and six products (hi.hi, hi.mid, mid.hi,
//     hi.lo, mid.mid, lo.hi), FP32-class.  BF16 keeps the FP32 exponent
//     range, so no operand is ever subnormal.  FP16x3: operands scaled by
//     powers of two into the fp16 range and split two ways (fp16 hi + lo,
//     22 bits), three v_mfma_f32_32x32x16_f16 products (hi.hi, hi.lo,
//     lo.hi), FP32-class.  Lane (r, h) holds coefficients
//     j = 16 s + 8 h + 0..7, the natural order.
// FP32 MFMA runs on the vector datapath and never overlaps the VALU work of
// the generator; the BF16 MFMAs run on the matrix cores and do.
// The MFMA accumulators are added to a second FP32 accumulator after every
// chunk, which keeps the rounding error of long sums at
// ~u (sqrt(32) + sqrt(K/32)) instead of ~u sqrt(K).  (A fold every second
// chunk compiles to selects on every chunk, which cost more than the adds.)
constexpr int KC = 32;
constexpr int FLUSH = 1;
constexpr int STR_F32 = 2 * KC + 4;  // floats per basis column (16-byte rows, skewed banks)
constexpr int STR_H = 2 * KC + 8;    // 16-bit values per basis column

// CSRC: coefficient source, 0 = Gaussian cos/sin from Philox, 1 = Eq. 3
// form from Philox, 2 = caller-supplied array (compile-time, so the integer
// generator of the unused mode never reaches the instruction stream).
// CSRC 3: the Gaussian coefficients of CSRC 0 divided by sqrt(2 ln 2) (the
// caller folds the factor into its amplitudes).
template <int CSRC>
__device__ __forceinline__ void coef4_src(const SumArgs& a, int64_t row, bool rowok, uint32_t t,
                                          float g[4]) {
    if constexpr (CSRC == 2) {
        const int64_t twoK = 2 * a.K;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t j = 4 * (int64_t)t + q;
            g[q] = (rowok && j < twoK) ? (float)a.coef[row * twoK + j] : 0.0f;
        }
    } else {
        // rows past the end of the set only feed output rows that are never
        // stored or summed, so their (finite) coefficients need no masking;
        // masking would split the Philox chains into separate basic blocks
        if constexpr (CSRC == 0) gauss4_f32(a.seed, a.counter + (uint64_t)row, t, g);
        else if constexpr (CSRC == 3) gauss4_f32_log2(a.seed, a.counter + (uint64_t)row, t, g);
        else coef4_f32(a.seed, a.counter + (uint64_t)row, t, 1, g);
    }
}

// ------------------------------------- FP32 class, narrow frequency sets ----
// Sets of at most 8 realisations in the FP32-class precisions: a matrix-core
// tile needs 32 rows, so these run on the vector ALU, one point per thread
// and RB rows per block, with the arithmetic of the FP32 path (FP64 range
// reduction, the same FP32 basis and coefficients as the MFMA kernels, FP32
// sums folded into a second FP32 accumulator every 64 frequencies).  The
// split-BF16 and BF16x6 precisions get these FP32 sums too (at least their
// accuracy).
template <int BASIS, int RB, int CSRC>
__global__ __launch_bounds__(256) void k_sum_f32n(SumArgs a, int64_t col_tiles) {
    constexpr int KCN = 64;
    __shared__ double sfx[KCN], sfy[KCN], sw[KCN];
    __shared__ float sC[RB][2 * KCN];
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int64_t ct = (int64_t)blockIdx.x % col_tiles;
    const int64_t sl = (int64_t)blockIdx.x / col_tiles;
    const int64_t set = a.set0 + sl;
    const int64_t row_begin = set * a.R_block;
    const int64_t set_end = (set + 1) * a.R_block < a.R ? (set + 1) * a.R_block : a.R;
    const int64_t row_end = row_begin + RB < set_end ? row_begin + RB : set_end;
    const int64_t p = ct * nt + tid;
    const bool pok = p < a.P;
    const double px = pok ? a.px[p] : 0.0;
    const double py = pok ? a.py[p] : 0.0;
    double pD = 1.0, pd = 0.0;
    if (BASIS == BASIS_PISTON && pok) {
        pD = a.apD[p];
        pd = a.apd[p];
    }
    const double* fx = a.fx + sl * a.K;
    const double* fy = a.fy + sl * a.K;
    const double* w = a.w + sl * a.K;
    float acc[RB], mst[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = mst[q] = 0.0f;

    for (int64_t k0 = 0; k0 < a.K; k0 += KCN) {
        __syncthreads();
        if (tid < KCN) {
            const int64_t k = k0 + tid;
            const bool ok = k < a.K;
            sfx[tid] = ok ? fx[k] : 0.0;
            sfy[tid] = ok ? fy[k] : 0.0;
            sw[tid] = ok ? w[k] : 0.0;
        }
        for (int i = tid; i < RB * (KCN / 2); i += nt) {
            const int rr = i / (KCN / 2);
            const int bt = i % (KCN / 2);
            const int64_t r = row_begin + rr;
            float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (r < row_end) coef4_src<CSRC>(a, r, true, (uint32_t)(k0 / 2 + bt), g);
#pragma unroll
            for (int q = 0; q < 4; ++q) sC[rr][4 * bt + q] = g[q];
        }
        __syncthreads();
        const int nk = a.K - k0 < KCN ? (int)(a.K - k0) : KCN;
        for (int kk = 0; kk < nk; ++kk) {
            const double cfx = sfx[kk], cfy = sfy[kk];
            double t = cfx * px + cfy * py;
            double amp = sw[kk];
            if (BASIS == BASIS_PISTON) {
                amp *= (double)aperture_filter_f32(pD, pd, sqrt(cfx * cfx + cfy * cfy)) *
                       grad_factor(a.grad, a.gx, a.gy, cfx, cfy);
                t += grad_shift(a.grad);
            }
            float cb, sb;
            basis_pair<BASIS>(t, amp, cb, sb);
#pragma unroll
            for (int q = 0; q < RB; ++q)
                acc[q] = fmaf(sC[q][2 * kk], cb, fmaf(sC[q][2 * kk + 1], sb, acc[q]));
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            mst[q] += acc[q];
            acc[q] = 0.0f;
        }
    }
    float* out = (float*)a.out;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int64_t r = row_begin + q;
        if (r < row_end && pok) out[r * a.P + p] = mst[q];
    }
}

// ----------------------- structure function, one realisation per set ----
// Differential-piston structure function when every realisation has its
// own frequencies (R_block = 1, as the paper draws them) and there are at
// most NPM baselines.  One block per realisation: thread t draws Philox
// blocks t, t + 256, ... (frequencies 2 t and 2 t + 1 of each) and keeps one
// accumulator per baseline; the 256 partial differential pistons of a
// baseline are added in a fixed tree (lanes by xor shuffles, then the 4
// waves in order), and the block writes dp^2 and dp^4 as the set's partial
// sums.  T = float: the FP32 path's coefficients and basis; T = double:
// the FP64 path's.
// The binary32 variant for up to 32 baselines asks for five waves per SIMD:
// the compiler then fits it in 84 VGPRs without spills (119 by default) and
// the extra wave hides more of the sine and FP64 latency.
template <typename T, int NPM>
constexpr int sf_one_min_waves() {
    return (sizeof(T) == 4 && NPM == 32) ? 5 : 1;
}

template <typename T, int NPM, int CSRC>
__global__ __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(sf_one_min_waves<T, NPM>(), 8))) void k_sf_one(SumArgs a) {
    __shared__ double2 sB[NPM];
    __shared__ double red[4][NPM];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t sl = blockIdx.x;
    const int64_t row = (a.set0 + sl) * a.R_block;  // R_block == 1
    const int nb = (int)a.P;
    for (int b = tid; b < NPM; b += 256)
        sB[b] = b < nb ? make_double2(a.px[b], a.py[b]) : make_double2(0.0, 0.0);
    // baselines along x (every y component zero, the usual layout of a
    // structure function against baseline length): f.B is then the one
    // product fx Bx, which is exactly what fx Bx + fy 0 rounds to
    const bool along_x = __syncthreads_and(tid >= nb || a.py[tid < nb ? tid : 0] == 0.0);
    const double* fx = a.fx + sl * a.K;
    const double* fy = a.fy + sl * a.K;
    const double* w = a.w + sl * a.K;
    T acc[NPM];
#pragma unroll
    for (int b = 0; b < NPM; ++b) acc[b] = (T)0;
    const int64_t nblk = (a.K + 1) / 2;
    for (int64_t t = tid; t < nblk; t += 256) {
        T g[4];
        if constexpr (sizeof(T) == 4) {
            float gf[4];
            coef4_src<CSRC>(a, row, true, (uint32_t)t, gf);
#pragma unroll
            for (int q = 0; q < 4; ++q) g[q] = gf[q];
        } else if constexpr (CSRC == 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t j = 4 * t + q;
                g[q] = j < 2 * a.K ? a.coef[row * 2 * a.K + j] : 0.0;
            }
        } else {
            double gd[4];
            coef4_f64(a.seed, a.counter + (uint64_t)row, (uint32_t)t, CSRC, gd);
#pragma unroll
            for (int q = 0; q < 4; ++q) g[q] = gd[q];
        }
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int64_t k = 2 * t + h;
            if (k >= a.K) break;
            const double cfx = fx[k], cfy = fy[k], amp = w[k];
            // one realisation: the amplitude and the constant factors of the
            // difference basis, (cos 2 pi r - 1, sin 2 pi r) =
            // (-2 sin^2 pi r, 2 sin pi r cos pi r), go into this frequency's two
            // coefficients once instead of into every baseline's basis
            // baselines past nb are staged as (0, 0): their difference basis
            // is exactly 0 and their accumulators stay 0, so no branch.
            // The baselines are read from LDS (a broadcast) for every
            // frequency: an offset the compiler cannot see through (a scalar
            // register set to 0) keeps it from hoisting all NPM of them into
            // registers, which would leave room for only 1-2 waves per SIMD.
            int z;
            asm volatile("s_mov_b32 %0, 0" : "=s"(z));
            if constexpr (sizeof(T) == 4) {
                const float fa = (float)amp;
                const float ga = -2.0f * (g[2 * h] * fa), gb = g[2 * h + 1] * fa;
                if (along_x) {
#pragma unroll
                    for (int b = 0; b < NPM; ++b) {
                        const double bx = sB[b + z].x;
                        const float r = frac_rev_f32(cfx * bx);
                        const float sh = __builtin_amdgcn_sinf(0.5f * r);  // sin(pi r)
                        const float s2 = __builtin_amdgcn_sinf(r);         // sin(2 pi r)
                        acc[b] = fmaf(ga, sh * sh, fmaf(gb, s2, acc[b]));
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < NPM; ++b) {
                        const double2 B = sB[b + z];
                        const float r = frac_rev_f32(cfx * B.x + cfy * B.y);
                        const float sh = __builtin_amdgcn_sinf(0.5f * r);  // sin(pi r)
                        const float s2 = __builtin_amdgcn_sinf(r);         // sin(2 pi r)
                        acc[b] = fmaf(ga, sh * sh, fmaf(gb, s2, acc[b]));
                    }
                }
            } else {
                const double ga = -2.0 * (g[2 * h] * amp), gb = 2.0 * (g[2 * h + 1] * amp);
#pragma unroll
                for (int b = 0; b < NPM; ++b) {
                    const double2 B = sB[b + z];
                    double sh, ch;
                    sincos2pi_reduced(0.5 * frac_centered(cfx * B.x + cfy * B.y), sh, ch);
                    acc[b] = fma(ga, sh * sh, fma(gb, sh * ch, acc[b]));
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NPM; ++b) {
        if (b < nb) {
            double v = (double)acc[b];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wave][b] = v;
        }
    }
    __syncthreads();
    if (tid < nb) {
        const double dp = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        const double d2 = dp * dp;
        double* dst = a.partial + (sl * a.P + tid) * 2;
        dst[0] = d2;
        dst[1] = d2 * d2;
    }
}

// LDS of one block of the MFMA kernel
template <int PREC, int NB>
struct MfmaSmem {
    static constexpr int NT = 32 * NB;
    static constexpr int NPL = PREC == 3 ? 3 : 2;  // 16-bit planes per operand (split modes)
    static constexpr int NBF = PREC == 1 ? 2 * NT * STR_F32 : 4;
    static constexpr int NBH = PREC >= 2 ? 2 * NT * STR_H : 8;
    __attribute__((aligned(16))) float sBf[NBF];
    __attribute__((aligned(16))) __bf16 sBp[NPL][NBH];
    double sred[8][NT][2];
    double spx[NT], spy[NT], sD[NT], sd[NT];
    double smax[8];  // FP16x3: per-wave largest amplitude / coefficient
};

// Largest value over the block of a per-thread value (all threads call it;
// it synchronises the block).
template <int PREC, int NB>
__device__ __forceinline__ double block_max(double v, MfmaSmem<PREC, NB>& sm) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm.smax[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = sm.smax[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, sm.smax[i]);
    return m;
}

// One output tile: rows [row tile rt of set sl], columns [column tile ct],
// frequency range ks.  Called once per block by k_sum_mfma and once per
// work item by the persistent batch kernel; every thread of the block must
// call it (it synchronises the block).
template <int PREC, int BASIS, int EPI, int MW, int NB, int CSRC>
__device__ __forceinline__ void sum_tile(const SumArgs& a, int64_t row_tiles, int64_t sl,
                                         int64_t rt, int64_t ct, int64_t ks,
                                         MfmaSmem<PREC, NB>& sm) {
    constexpr int NT = 32 * NB;
    constexpr int NPL = MfmaSmem<PREC, NB>::NPL;
    // split precisions draw the Gaussians without the Box-Muller constant
    // and fold it into the basis amplitudes (one product per frequency and
    // column instead of one per pair of coefficients)
    constexpr int CS = (PREC >= 2 && CSRC == 0) ? 3 : CSRC;
    constexpr double kAmp = CS == 3 ? kBoxMullerLog2 : 1.0;
    float* sBf = sm.sBf;
    auto& sBp = sm.sBp;
    auto& sred = sm.sred;
    double* spx = sm.spx;
    double* spy = sm.spy;
    double* sD = sm.sD;
    double* sd = sm.sd;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int WV = blockDim.x >> 6;
    const int lr = lane & 31;
    const int lh = lane >> 5;
    const int64_t MT = 32 * MW * WV;
    const int64_t set = a.set0 + sl;
    const int64_t row_begin = set * a.R_block + rt * MT;
    const int64_t row_end = (set + 1) * a.R_block < a.R ? (set + 1) * a.R_block : a.R;
    const int64_t col0 = ct * NT;
    const int64_t kb = ks * a.kspan;
    const int64_t ke = kb + a.kspan < a.K ? kb + a.kspan : a.K;

    // basis work of this thread: frequency kk of every chunk, columns
    // pp0 + j * cstep
    const int kk = threadIdx.x % KC;
    const int pp0 = threadIdx.x / KC;
    const int cstep = blockDim.x / KC;
    for (int i = threadIdx.x; i < NT; i += blockDim.x) {
        int64_t p = col0 + i;
        bool ok = p < a.P;
        spx[i] = ok ? a.px[p] : 0.0;
        spy[i] = ok ? a.py[p] : 0.0;
        if (BASIS == BASIS_PISTON) {
            sD[i] = ok ? a.apD[p] : 1.0;
            sd[i] = ok ? a.apd[p] : 0.0;
        }
    }
    __syncthreads();

    int64_t myrow[MW];
    bool rowok[MW];
#pragma unroll
    for (int mw = 0; mw < MW; ++mw) {
        myrow[mw] = row_begin + (int64_t)(wave * MW + mw) * 32 + lr;
        rowok[mw] = myrow[mw] < row_end;
    }
    const double* fx = a.fx + sl * a.K;
    const double* fy = a.fy + sl * a.K;
    const double* w = a.w + sl * a.K;

    f32x16 acc[MW][NB];
    f32x16 mst[MW][NB];
#pragma unroll
    for (int mw = 0; mw < MW; ++mw)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                acc[mw][nb][i] = 0.0f;
                mst[mw][nb][i] = 0.0f;
            }
        }

    // FP16x3: the basis amplitudes of this frequency range (and caller-given
    // coefficients) are scaled by powers of two into the fp16 range; the sums
    // are scaled back exactly before the epilogue
    double wscale = 1.0, cscale = 1.0;
    float unscale = 1.0f;
    if constexpr (PREC == 4) {
        double m = 0.0;
        for (int64_t k = kb + threadIdx.x; k < ke; k += blockDim.x) {
            double v = fabs(w[k]);
            if (BASIS == BASIS_PISTON) v *= fabs(grad_factor(a.grad, a.gx, a.gy, fx[k], fy[k]));
            m = fmax(m, v);
        }
        f16_scale(block_max(m, sm) * kAmp, wscale, unscale);
        if constexpr (CSRC == 2) {
            const int64_t twoK = 2 * a.K;
            const int64_t r1 = row_begin + MT < row_end ? row_begin + MT : row_end;
            double mc = 0.0;
            for (int64_t r = row_begin; r < r1; ++r)
                for (int64_t j = 2 * kb + threadIdx.x; j < 2 * ke; j += blockDim.x)
                    mc = fmax(mc, fabs(a.coef[r * twoK + j]));
            float uc;
            f16_scale(block_max(mc, sm) * 0.25, cscale, uc);  // coefficients below 2^15
            unscale *= uc;
        }
    }

    const int64_t nchunks = (ke - kb + KC - 1) / KC;
    // frequency data of the first chunk for this thread's kk
    double nfx = 0.0, nfy = 0.0, nw = 0.0;
    if (kb + kk < ke) {
        nfx = fx[kb + kk];
        nfy = fy[kb + kk];
        nw = w[kb + kk];
    }
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int64_t k0 = kb + ch * KC;
        const int buf = (int)(ch & 1);
        const double cfx = nfx, cfy = nfy, cw = nw;
        {
            int64_t kn = k0 + KC + kk;
            if (kn < ke) {
                nfx = fx[kn];
                nfy = fy[kn];
                nw = w[kn];
            } else {
                nfx = nfy = nw = 0.0;
            }
        }
        // basis of this chunk into buffer `buf`
        const double fmag = BASIS == BASIS_PISTON ? sqrt(cfx * cfx + cfy * cfy) : 0.0;
        const double gw =
            BASIS == BASIS_PISTON ? cw * grad_factor(a.grad, a.gx, a.gy, cfx, cfy) : cw;
        const double sh = BASIS == BASIS_PISTON ? grad_shift(a.grad) : 0.0;
        for (int pp = pp0; pp < NT; pp += cstep) {
            double amp = gw * (kAmp * wscale);
            if (BASIS == BASIS_PISTON) amp *= (double)aperture_filter_f32(sD[pp], sd[pp], fmag);
            float cb, sb;
            double t = cfx * spx[pp] + cfy * spy[pp];
            if (BASIS == BASIS_PISTON) t += sh;  // (an add of 0 would not fold away)
            basis_pair<BASIS>(t, amp, cb, sb);
            if constexpr (PREC == 1) {
                float* dst = sBf + buf * NT * STR_F32 + pp * STR_F32 + 2 * kk;
                dst[0] = cb;
                dst[1] = sb;
            } else {
                const int o = buf * NT * STR_H + pp * STR_H + 2 * kk;  // even
                uint32_t pcs[NPL];
                if constexpr (PREC == 4)
                    split_f16x2<true>(cb, sb, pcs);
                else
                    split_bf16x2<NPL>(cb, sb, pcs);
#pragma unroll
                for (int i = 0; i < NPL; ++i) *(uint32_t*)&sBp[i][o] = pcs[i];
            }
        }

        if constexpr (PREC == 1) {
            // coefficients of the whole chunk: KC/4 Philox blocks per row block
            float av[KC / 4][MW][4];
#pragma unroll
            for (int m = 0; m < KC / 4; ++m) {
                const uint32_t t = (uint32_t)(k0 / 2) + 2u * m + (uint32_t)lh;
#pragma unroll
                for (int mw = 0; mw < MW; ++mw)
                    coef4_src<CSRC>(a, myrow[mw], rowok[mw], t, av[m][mw]);
            }
            __syncthreads();
            const float* B = sBf + buf * NT * STR_F32;
#pragma unroll
            for (int m = 0; m < KC / 4; ++m) {
                f32x4 bv[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    bv[nb] = *(const f32x4*)&B[(nb * 32 + lr) * STR_F32 + 8 * m + 4 * lh];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int mw = 0; mw < MW; ++mw)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[mw][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                av[m][mw][q], bv[nb][q], acc[mw][nb], 0, 0, 0);
            }
        } else if constexpr (PREC == 4) {
            // FP16x3: as below with two fp16 planes and three products
            __syncthreads();
#pragma unroll
            for (int sg = 0; sg < KC / 8; ++sg) {
                const uint32_t t = (uint32_t)(k0 / 2) + 4u * sg + 2u * (uint32_t)lh;
                f16x8 ap[MW][2];
#pragma unroll
                for (int mw = 0; mw < MW; ++mw) {
                    float g[8];
                    coef4_src<CS>(a, myrow[mw], rowok[mw], t, g);
                    coef4_src<CS>(a, myrow[mw], rowok[mw], t + 1u, g + 4);
                    if constexpr (CSRC == 2) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) g[q] = (float)((double)g[q] * cscale);
                    }
                    split8_f16(g, ap[mw]);
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int off = buf * NT * STR_H + (nb * 32 + lr) * STR_H + 16 * sg + 8 * lh;
                    const f16x8 b0 = *(const f16x8*)&sBp[0][off];
                    const f16x8 b1 = *(const f16x8*)&sBp[1][off];
#pragma unroll
                    for (int mw = 0; mw < MW; ++mw) {
                        f32x16 c = acc[mw][nb];
                        c = mfma_f16(ap[mw][1], b0, c);  // smallest products first
                        c = mfma_f16(ap[mw][0], b1, c);
                        c = mfma_f16(ap[mw][0], b0, c);
                        acc[mw][nb] = c;
                    }
                }
            }
        } else {
            // each group of 8 contraction values draws its coefficients right
            // before its MFMAs: the generator's vector work runs beside the
            // matrix cores, and only one group's operand planes are live
            __syncthreads();
#pragma unroll
            for (int sg = 0; sg < KC / 8; ++sg) {
                const uint32_t t = (uint32_t)(k0 / 2) + 4u * sg + 2u * (uint32_t)lh;
                bf16x8 ap[MW][NPL];
#pragma unroll
                for (int mw = 0; mw < MW; ++mw) {
                    float g[8];
                    coef4_src<CS>(a, myrow[mw], rowok[mw], t, g);
                    coef4_src<CS>(a, myrow[mw], rowok[mw], t + 1u, g + 4);
                    split8_bf16<NPL>(g, ap[mw]);
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int off = buf * NT * STR_H + (nb * 32 + lr) * STR_H + 16 * sg + 8 * lh;
                    bf16x8 bp[NPL];
#pragma unroll
                    for (int i = 0; i < NPL; ++i) bp[i] = *(const bf16x8*)&sBp[i][off];
#pragma unroll
                    for (int mw = 0; mw < MW; ++mw) {
                        f32x16 c = acc[mw][nb];
                        // smallest products first
                        if constexpr (NPL == 3) {
                            c = mfma_bf16(ap[mw][2], bp[0], c);
                            c = mfma_bf16(ap[mw][1], bp[1], c);
                            c = mfma_bf16(ap[mw][0], bp[2], c);
                        }
                        c = mfma_bf16(ap[mw][1], bp[0], c);
                        c = mfma_bf16(ap[mw][0], bp[1], c);
                        c = mfma_bf16(ap[mw][0], bp[0], c);
                        acc[mw][nb] = c;
                    }
                }
            }
        }

        if ((ch % FLUSH) == FLUSH - 1 || ch == nchunks - 1) {
#pragma unroll
            for (int mw = 0; mw < MW; ++mw)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    mst[mw][nb] += acc[mw][nb];
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[mw][nb][i] = 0.0f;
                }
        }
    }

    if constexpr (PREC == 4) {
#pragma unroll
        for (int mw = 0; mw < MW; ++mw)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int i = 0; i < 16; ++i) mst[mw][nb][i] *= unscale;
    }

    if (EPI == EPI_STORE) {
        float* out = (float*)a.out;
#pragma unroll
        for (int mw = 0; mw < MW; ++mw)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int64_t col = col0 + nb * 32 + lr;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int64_t r = row_begin + (int64_t)(wave * MW + mw) * 32 + 8 * (i / 4) + 4 * lh + (i % 4);
                    if (r < row_end && col < a.P) out[r * a.P + col] = mst[mw][nb][i];
                }
            }
    } else if (a.ksplit > 1) {
        // partial sums of this frequency range; squared after all ranges are in
#pragma unroll
        for (int mw = 0; mw < MW; ++mw)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int64_t col = col0 + nb * 32 + lr;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int64_t r = row_begin + (int64_t)(wave * MW + mw) * 32 + 8 * (i / 4) + 4 * lh + (i % 4);
                    if (r < row_end && col < a.P) a.phi_part[(ks * a.R + r) * a.P + col] = mst[mw][nb][i];
                }
            }
    } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            double s2 = 0.0, s4 = 0.0;
#pragma unroll
            for (int mw = 0; mw < MW; ++mw)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int64_t r = row_begin + (int64_t)(wave * MW + mw) * 32 + 8 * (i / 4) + 4 * lh + (i % 4);
                    if (r < row_end) {
                        double d = (double)mst[mw][nb][i];
                        double d2 = d * d;
                        s2 += d2;
                        s4 += d2 * d2;
                    }
                }
            s2 += __shfl_xor(s2, 32);
            s4 += __shfl_xor(s4, 32);
            if (lh == 0) {
                sred[wave][nb * 32 + lr][0] = s2;
                sred[wave][nb * 32 + lr][1] = s4;
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < NT; c += blockDim.x) {
            const int64_t col = col0 + c;
            if (col < a.P) {
                double t2 = 0.0, t4 = 0.0;
                for (int v = 0; v < WV; ++v) {
                    t2 += sred[v][c][0];
                    t4 += sred[v][c][1];
                }
                double* dst = a.partial + ((sl * row_tiles + rt) * a.P + col) * 2;
                dst[0] = t2;
                dst[1] = t4;
            }
        }
    }
}

// The one-tile structure-function kernels (MW = NB = 1, EPI_SFSUM) are bound by
// vector issue: asking for five waves per SIMD instead of the four their
// registers give (a handful of spills outside the frequency loop, 30 KB of
// LDS per block) hides more of the transcendental and MFMA latency; FP16x3
// fits six (80 registers, its one spill outside the loop).  BF16x6
// with Eq. 3 or caller-given coefficients keeps the default: at five waves
// it reloads spilled registers inside the frequency loop.
template <int PREC, int EPI, int MW, int NB, int CSRC>
constexpr int sum_mfma_min_waves() {
    return (EPI == EPI_SFSUM && MW * NB == 1 && (PREC < 3 || CSRC == 0)) ? (PREC == 4 ? 6 : 5) : 1;
}

// Blocks of the difference basis may hold 8 waves (256 rows), the others 4.
template <int BASIS>
constexpr int sum_mfma_max_threads() {
    return BASIS == BASIS_DIFF ? 512 : 256;
}

template <int PREC, int BASIS, int EPI, int MW, int NB, int CSRC>
__global__ __launch_bounds__(sum_mfma_max_threads<BASIS>()) __attribute__((
    amdgpu_waves_per_eu(sum_mfma_min_waves<PREC, EPI, MW, NB, CSRC>(), 8))) void
k_sum_mfma(SumArgs a, int64_t row_tiles, int64_t col_tiles) {
    __shared__ MfmaSmem<PREC, NB> sm;
    // tile: column tile fastest, then K split, row tile, set
    int64_t bidx = blockIdx.x;
    const int64_t ct = bidx % col_tiles;
    bidx /= col_tiles;
    const int64_t ks = bidx % a.ksplit;
    bidx /= a.ksplit;
    const int64_t rt = bidx % row_tiles;
    const int64_t sl = bidx / row_tiles;
    sum_tile<PREC, BASIS, EPI, MW, NB, CSRC>(a, row_tiles, sl, rt, ct, ks, sm);
}

// ----------------------------------------------------- batch kernels ----
// Persistent batch of uneven instances: a grid sized to the chip pulls work
// items (instance, set, row tile, column tile) from a global counter until
// the list is exhausted.  Items are ordered by decreasing cost (longest
// first), so the tail of the launch is made of small items.  The counter is
// advanced with a vector atomic by one lane; every wave of every block
// reaches the exit test on each iteration.  AP: some instances carry
// apertures (pistons or tilts, chosen per item from the instance); without
// it every item is a phase item.
template <int PREC, int MW, int NB, bool AP>
__global__ __launch_bounds__(256) void k_batch_persistent(const SumArgs* __restrict__ inst,
                                                          const BatchItem* __restrict__ items,
                                                          int n_items,
                                                          unsigned* __restrict__ counter) {
    __shared__ MfmaSmem<PREC, NB> sm;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const SumArgs a = inst[w.inst];
        const int64_t row_tiles = (a.R_block + 32 * MW * (blockDim.x >> 6) - 1) /
                                  (32 * MW * (blockDim.x >> 6));
        bool piston = false;
        if constexpr (AP) piston = a.apD != nullptr;
        if (piston) {
            if (a.mode == 0)
                sum_tile<PREC, BASIS_PISTON, EPI_STORE, MW, NB, 0>(a, row_tiles, w.set, w.rt, w.ct,
                                                                   0, sm);
            else
                sum_tile<PREC, BASIS_PISTON, EPI_STORE, MW, NB, 1>(a, row_tiles, w.set, w.rt, w.ct,
                                                                   0, sm);
        } else if (a.mode == 0) {
            sum_tile<PREC, BASIS_PHASE, EPI_STORE, MW, NB, 0>(a, row_tiles, w.set, w.rt, w.ct, 0, sm);
        } else {
            sum_tile<PREC, BASIS_PHASE, EPI_STORE, MW, NB, 1>(a, row_tiles, w.set, w.rt, w.ct, 0, sm);
        }
        __syncthreads();
    }
}

// Zeroes the work counter with a plain store (graph-capturable, no memset node).
__global__ void k_reset_counter(unsigned* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// ----------------------------------------------------- split-K squares ----
// Block (row block rb, column tile): 256 threads = 8 row groups x 32
// columns.  Adds the K-range partial sums of each differential piston in a
// fixed order, then accumulates its square and fourth power per column over
// the block's rows; the 8 row groups are combined in a fixed order.
constexpr int SF_ROWS = 64;  // rows per block: ~1600 blocks for 1e5 rows, enough to hide load latency

__global__ __launch_bounds__(256) void k_sfsum_rows(const float* __restrict__ phi, int ksplit,
                                                    int64_t R, int64_t P,
                                                    double* __restrict__ partial) {
    __shared__ double r2[8][32], r4[8][32];
    const int c = threadIdx.x & 31;
    const int rg = threadIdx.x >> 5;
    const int64_t col = (int64_t)blockIdx.y * 32 + c;
    const int64_t r0 = (int64_t)blockIdx.x * SF_ROWS;
    const int64_t r1 = r0 + SF_ROWS < R ? r0 + SF_ROWS : R;
    double s2 = 0.0, s4 = 0.0;
    if (col < P) {
        for (int64_t r = r0 + rg; r < r1; r += 8) {
            double v = 0.0;
            for (int k = 0; k < ksplit; ++k) v += (double)phi[((int64_t)k * R + r) * P + col];
            double v2 = v * v;
            s2 += v2;
            s4 += v2 * v2;
        }
    }
    r2[rg][c] = s2;
    r4[rg][c] = s4;
    __syncthreads();
    if (rg == 0 && col < P) {
        double t2 = 0.0, t4 = 0.0;
        for (int g = 0; g < 8; ++g) {
            t2 += r2[g][c];
            t4 += r4[g][c];
        }
        partial[((int64_t)blockIdx.x * P + col) * 2] = t2;
        partial[((int64_t)blockIdx.x * P + col) * 2 + 1] = t4;
    }
}

// ------------------------------------------------------------- reduce ----
// One block per column; partial sums over row tiles in a fixed order
// (strided by thread, then a fixed tree), so results are bit-reproducible.
__global__ __launch_bounds__(256) void k_reduce_sf(const double* __restrict__ partial,
                                                   int64_t n_tiles, int64_t P, int64_t R,
                                                   double* __restrict__ sf,
                                                   double* __restrict__ sf_stderr) {
    __shared__ double r2[256], r4[256];
    const int64_t p = blockIdx.x;
    double s2 = 0.0, s4 = 0.0;
    for (int64_t t = threadIdx.x; t < n_tiles; t += 256) {
        s2 += partial[(t * P + p) * 2];
        s4 += partial[(t * P + p) * 2 + 1];
    }
    r2[threadIdx.x] = s2;
    r4[threadIdx.x] = s4;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            r2[threadIdx.x] += r2[threadIdx.x + h];
            r4[threadIdx.x] += r4[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double S2 = r2[0], S4 = r4[0];
        double n = (double)R;
        sf[p] = S2 / n;
        if (sf_stderr) {
            double var = R > 1 ? (S4 - S2 * S2 / n) / (n - 1.0) : 0.0;
            sf_stderr[p] = sqrt(var > 0.0 ? var / n : 0.0);
        }
    }
}

// ----------------------------------------------------------- launchers ----
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_reduce_sf(const double* partial, int64_t n_tiles, int64_t P, int64_t R,
                            double* sf, double* sf_stderr, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_sf, dim3((unsigned)P), dim3(256), 0, st, partial, n_tiles, P, R, sf,
                       sf_stderr);
    return hipGetLastError();
}

// launch shapes of the MFMA kernel
struct MfmaShape {
    int MW, NB, WV;
};

static MfmaShape mfma_shape(int precision, int basis, int64_t R_block, int64_t P) {
    MfmaShape s;
    const bool wide = basis == BASIS_PHASE && P > 32;
    if (precision == 1) {  // FP32: one 32-row block per wave keeps 4 waves/SIMD
        s.MW = 1;
        s.NB = wide ? 2 : 1;
    } else {               // split modes: the A operand is reused over 2x2 blocks
        s.MW = wide ? 2 : 1;
        s.NB = wide ? 2 : 1;
    }
    int64_t wv = cdiv(R_block, 32 * s.MW);
    s.WV = (int)(wv > 4 ? 4 : wv);
    // differential pistons of at most 32 baselines: one block covers 256
    // rows, so each set's difference basis is built once per 256 rows
    if (precision >= 2 && basis == BASIS_DIFF && P <= 32 && wv >= 8) s.WV = 8;
    return s;
}

int64_t sum_row_tiles_per_set(int precision, int basis, int64_t R_block, int64_t P) {
    if (precision == 0) return cdiv(R_block, F64_TR);
    MfmaShape s = mfma_shape(precision, basis, R_block, P);
    return cdiv(R_block, 32 * s.MW * s.WV);
}

int64_t sum_col_tiles(int precision, int basis, int64_t R_block, int64_t P) {
    if (precision == 0) return cdiv(P, F64_TP);
    MfmaShape s = mfma_shape(precision, basis, R_block, P);
    return cdiv(P, 32 * s.NB);
}

bool sf_one_realisation(int64_t R_block, int64_t P) { return R_block == 1 && P <= 64; }

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Blocks of the structure-function kernel the current device holds at once
// (compute units x resident blocks per CU), for choosing the K split.
static int64_t sf_resident_slots(int precision, int64_t R_block, int64_t P) {
    const MfmaShape s = mfma_shape(precision, BASIS_DIFF, R_block, P);
    const void* kern = nullptr;
    if (precision == 1) kern = (const void*)k_sum_mfma<1, BASIS_DIFF, EPI_SFSUM, 1, 1, 0>;
    else if (precision == 2) kern = (const void*)k_sum_mfma<2, BASIS_DIFF, EPI_SFSUM, 1, 1, 0>;
    else if (precision == 3) kern = (const void*)k_sum_mfma<3, BASIS_DIFF, EPI_SFSUM, 1, 1, 0>;
    else kern = (const void*)k_sum_mfma<4, BASIS_DIFF, EPI_SFSUM, 1, 1, 0>;
    int dev = 0, ncu = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu < 1)
        ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 64 * s.WV, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    (void)hipGetLastError();
    return (int64_t)ncu * nb;
}

size_t sf_plan_bytes(const SfPlan& p, int64_t P) {
    return round256((size_t)(p.n_partial_tiles * P) * 2 * sizeof(double)) +
           round256(p.phi_floats * sizeof(float));
}

SfPlan sf_plan(int precision, int64_t K, int64_t R, int64_t R_block, int64_t P,
               size_t max_bytes) {
    SfPlan p;
    const int64_t n_sets = cdiv(R, R_block);
    const int64_t rts = sum_row_tiles_per_set(precision, BASIS_DIFF, R_block, P);
    const int64_t cts = sum_col_tiles(precision, BASIS_DIFF, R_block, P);
    const int64_t base = n_sets * rts * cts;
    int64_t ks = 1;
    // one realisation per set: k_sf_one spreads the frequencies over a block
    if (precision != 0 && !sf_one_realisation(R_block, P)) {
        // split K so that the blocks fill the chip's resident slots in whole
        // rounds: the launch takes about ceil(base ks / slots) rounds of
        // blocks 1/ks as long, plus the split-K partial sums' traffic (a
        // few microseconds per range at these sizes)
        const int64_t slots = sf_resident_slots(precision, R_block, P);
        const int64_t nch = cdiv(K, KC);
        int64_t kmax = nch / 2 < 16 ? nch / 2 : 16;
        double best = 1e300;
        for (int64_t k = 1; k <= (kmax < 1 ? 1 : kmax); ++k) {
            if (k > 1 && (double)k * R * P * 4.0 > (double)((size_t)1 << 30)) break;
            const double cost = (double)cdiv(base * k, slots) / (double)k + 0.003 * (double)k;
            if (cost < best - 1e-12) {
                best = cost;
                ks = k;
            }
        }
    }
    for (;;) {
        p.ksplit = (int)ks;
        p.kspan = cdiv(cdiv(K, ks), KC) * KC;  // whole chunks, even frequency offsets
        p.phi_floats = ks > 1 ? (size_t)ks * R * P : 0;
        p.n_partial_tiles = ks > 1 ? cdiv(R, SF_ROWS) : n_sets * rts;
        if (ks == 1 || max_bytes == 0 || sf_plan_bytes(p, P) <= max_bytes) break;
        --ks;
    }
    return p;
}

template <int BASIS, int RB>
static hipError_t launch_f64n(const SumArgs& a, hipStream_t st) {
    const int nt = a.P >= 256 ? 256 : (a.P >= 128 ? 128 : 64);
    const int64_t col_tiles = cdiv(a.P, nt);
    const int64_t blocks = (a.set1 - a.set0) * col_tiles;
    hipLaunchKernelGGL((k_sum_f64n<BASIS, RB>), dim3((unsigned)blocks), dim3(nt), 0, st, a,
                       col_tiles);
    return hipGetLastError();
}

template <int BASIS, int EPI>
static hipError_t launch_f64(const SumArgs& a, hipStream_t st) {
    if constexpr (EPI == EPI_STORE) {
        // sets of at most 8 realisations: one point per thread, no empty rows
        if (a.R_block == 1) return launch_f64n<BASIS, 1>(a, st);
        if (a.R_block == 2) return launch_f64n<BASIS, 2>(a, st);
        if (a.R_block <= 4) return launch_f64n<BASIS, 4>(a, st);
        if (a.R_block <= 8) return launch_f64n<BASIS, 8>(a, st);
    }
    int64_t row_tiles = cdiv(a.R_block, F64_TR);
    int64_t col_tiles = cdiv(a.P, F64_TP);
    int64_t blocks = (a.set1 - a.set0) * row_tiles * col_tiles;
    hipLaunchKernelGGL((k_sum_f64<BASIS, EPI>), dim3((unsigned)blocks), dim3(256), 0, st, a,
                       row_tiles, col_tiles);
    return hipGetLastError();
}

template <int PREC, int BASIS, int EPI, int MW, int NB>
static hipError_t launch_mfma_t(const SumArgs& a, int WV, hipStream_t st) {
    int64_t MT = 32 * MW * WV;
    int64_t row_tiles = cdiv(a.R_block, MT);
    int64_t col_tiles = cdiv(a.P, 32 * NB);
    int64_t blocks = (a.set1 - a.set0) * row_tiles * col_tiles * a.ksplit;
    dim3 g((unsigned)blocks), b(64 * WV);
    if (a.coef)
        hipLaunchKernelGGL((k_sum_mfma<PREC, BASIS, EPI, MW, NB, 2>), g, b, 0, st, a, row_tiles,
                           col_tiles);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_sum_mfma<PREC, BASIS, EPI, MW, NB, 1>), g, b, 0, st, a, row_tiles,
                           col_tiles);
    else
        hipLaunchKernelGGL((k_sum_mfma<PREC, BASIS, EPI, MW, NB, 0>), g, b, 0, st, a, row_tiles,
                           col_tiles);
    return hipGetLastError();
}

template <int PREC, int BASIS, int EPI>
static hipError_t launch_mfma(const SumArgs& a, hipStream_t st) {
    MfmaShape s = mfma_shape(PREC, BASIS, a.R_block, a.P);
    if constexpr (PREC == 1) {
        if (s.NB == 2) return launch_mfma_t<PREC, BASIS, EPI, 1, 2>(a, s.WV, st);
        return launch_mfma_t<PREC, BASIS, EPI, 1, 1>(a, s.WV, st);
    } else {
        if (s.MW == 2) return launch_mfma_t<PREC, BASIS, EPI, 2, 2>(a, s.WV, st);
        return launch_mfma_t<PREC, BASIS, EPI, 1, 1>(a, s.WV, st);
    }
}

template <int BASIS, int RB>
static hipError_t launch_f32n_r(const SumArgs& a, hipStream_t st) {
    const int nt = a.P >= 256 ? 256 : (a.P >= 128 ? 128 : 64);
    const int64_t col_tiles = cdiv(a.P, nt);
    const dim3 g((unsigned)((a.set1 - a.set0) * col_tiles)), b(nt);
    if (a.coef)
        hipLaunchKernelGGL((k_sum_f32n<BASIS, RB, 2>), g, b, 0, st, a, col_tiles);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_sum_f32n<BASIS, RB, 1>), g, b, 0, st, a, col_tiles);
    else
        hipLaunchKernelGGL((k_sum_f32n<BASIS, RB, 0>), g, b, 0, st, a, col_tiles);
    return hipGetLastError();
}

template <int BASIS>
static hipError_t launch_f32n(const SumArgs& a, hipStream_t st) {
    if (a.R_block == 1) return launch_f32n_r<BASIS, 1>(a, st);
    if (a.R_block == 2) return launch_f32n_r<BASIS, 2>(a, st);
    if (a.R_block <= 4) return launch_f32n_r<BASIS, 4>(a, st);
    return launch_f32n_r<BASIS, 8>(a, st);
}

template <typename T, int NPM>
static hipError_t launch_sf_one_t(const SumArgs& a, hipStream_t st) {
    const dim3 g((unsigned)(a.set1 - a.set0)), b(256);
    if (a.coef)
        hipLaunchKernelGGL((k_sf_one<T, NPM, 2>), g, b, 0, st, a);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_sf_one<T, NPM, 1>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((k_sf_one<T, NPM, 0>), g, b, 0, st, a);
    return hipGetLastError();
}

static hipError_t launch_sf_one(int precision, const SumArgs& a, hipStream_t st) {
    if (precision == 0)
        return a.P <= 32 ? launch_sf_one_t<double, 32>(a, st) : launch_sf_one_t<double, 64>(a, st);
    return a.P <= 32 ? launch_sf_one_t<float, 32>(a, st) : launch_sf_one_t<float, 64>(a, st);
}

template <int BASIS, int EPI>
static hipError_t launch_be(int precision, const SumArgs& a, hipStream_t st) {
    if constexpr (EPI == EPI_SFSUM)
        if (sf_one_realisation(a.R_block, a.P)) return launch_sf_one(precision, a, st);
    if (precision == 0) return launch_f64<BASIS, EPI>(a, st);
    // FP32 class, sets of at most 8 realisations: vector ALU (see k_sum_f32n)
    if constexpr (EPI == EPI_STORE)
        if (a.R_block <= 8) return launch_f32n<BASIS>(a, st);
    if (precision == 1) return launch_mfma<1, BASIS, EPI>(a, st);
    if (precision == 2) return launch_mfma<2, BASIS, EPI>(a, st);
    if (precision == 4) return launch_mfma<4, BASIS, EPI>(a, st);
    return launch_mfma<3, BASIS, EPI>(a, st);
}

hipError_t launch_sum(int precision, int basis, int epi, const SumArgs& a, hipStream_t st) {
    if (a.set1 <= a.set0) return hipSuccess;
    if (epi == EPI_STORE) {
        if (basis == BASIS_PHASE) return launch_be<BASIS_PHASE, EPI_STORE>(precision, a, st);
        if (basis == BASIS_PISTON) return launch_be<BASIS_PISTON, EPI_STORE>(precision, a, st);
        return launch_be<BASIS_DIFF, EPI_STORE>(precision, a, st);
    }
    return launch_be<BASIS_DIFF, EPI_SFSUM>(precision, a, st);
}

// Batch launch shapes the autotuner chooses from: (MW, NB) per precision
// and the number of resident blocks per CU of the persistent grid.
static const BatchShape kShapesF32[] = {{1, 2, 2, 0}, {1, 2, 3, 0}, {1, 1, 4, 0}, {1, 2, 4, 0},
                                        {0, 0, 1, 1}};
static const BatchShape kShapesSplit[] = {{2, 2, 1, 0}, {2, 2, 2, 0}, {1, 2, 2, 0}, {1, 2, 3, 0},
                                          {0, 0, 1, 1}};

int batch_shape_count(int precision) { return precision == 1 ? 5 : 5; }

hipError_t launch_reset_counter(unsigned* counter, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

BatchShape batch_shape(int precision, int id) {
    return precision == 1 ? kShapesF32[id] : kShapesSplit[id];
}

template <int PREC, int MW, int NB>
static hipError_t launch_batch_t(bool ap, const SumArgs* inst, const BatchItem* items, int n_items,
                                 unsigned* counter, int n_blocks, hipStream_t st) {
    if (ap)
        hipLaunchKernelGGL((k_batch_persistent<PREC, MW, NB, true>), dim3((unsigned)n_blocks),
                           dim3(256), 0, st, inst, items, n_items, counter);
    else
        hipLaunchKernelGGL((k_batch_persistent<PREC, MW, NB, false>), dim3((unsigned)n_blocks),
                           dim3(256), 0, st, inst, items, n_items, counter);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_batch_p(int MW, int NB, bool ap, const SumArgs* inst,
                                 const BatchItem* items, int n_items, unsigned* counter,
                                 int n_blocks, hipStream_t st) {
    if (MW == 2 && NB == 2) {
        if constexpr (PREC != 1)
            return launch_batch_t<PREC, 2, 2>(ap, inst, items, n_items, counter, n_blocks, st);
        return hipErrorInvalidValue;
    }
    if (MW == 1 && NB == 2)
        return launch_batch_t<PREC, 1, 2>(ap, inst, items, n_items, counter, n_blocks, st);
    if (MW == 1 && NB == 1)
        return launch_batch_t<PREC, 1, 1>(ap, inst, items, n_items, counter, n_blocks, st);
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int precision, BatchShape shape, bool has_ap, const SumArgs* inst,
                        const BatchItem* items, int n_items, unsigned* counter, int n_blocks,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int MW = shape.MW, NB = shape.NB;
    if (precision == 1)
        return launch_batch_p<1>(MW, NB, has_ap, inst, items, n_items, counter, n_blocks, st);
    if (precision == 2)
        return launch_batch_p<2>(MW, NB, has_ap, inst, items, n_items, counter, n_blocks, st);
    if (precision == 4)
        return launch_batch_p<4>(MW, NB, has_ap, inst, items, n_items, counter, n_blocks, st);
    return launch_batch_p<3>(MW, NB, has_ap, inst, items, n_items, counter, n_blocks, st);
}

hipError_t launch_sfsum_rows(const float* phi, int ksplit, int64_t R, int64_t P, double* partial,
                             hipStream_t st) {
    dim3 g((unsigned)cdiv(R, SF_ROWS), (unsigned)cdiv(P, 32));
    hipLaunchKernelGGL(k_sfsum_rows, g, dim3(256), 0, st, phi, ksplit, R, P, partial);
    return hipGetLastError();
}

}  // namespace qrfs
