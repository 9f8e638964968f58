// qrfs_wide.hip -- two-phase contraction of Eq. 3 for wide point sets
// (large phase screens, many apertures): gfx950.
//
// When P is large, the fused kernel regenerates every coefficient once per
// column tile, which makes the integer generator, not the MFMA, the bound.
// Here the work is split in two phases:
//   1. k_coef_tiles draws every coefficient of the launch once (Philox +
//      Box-Muller, or the caller's array), splits it into the MFMA operand
//      format (FP32, 2 / 3 BF16 planes, or 2 fp16 planes scaled per set by
//      k_set_scale) and writes it to HBM already in
//      the per-lane order of the MFMA A operand: one 1 KiB fragment per
//      (32 rows, 8 or 16 contraction values, plane), lane (r, h) holding
//      row r and contraction values j = j0 + 4h + q (FP32, 4 values) or
//      j = j0 + 8h + e (BF16, 8 values).  Contraction value j = 2k is the
//      cosine term of frequency k, j = 2k + 1 the sine term (natural order).
//   2. k_wide computes 256 x 256 output tiles with 8 waves of 64 x 128
//      (8 accumulators of 32 x 32 per wave, 2 waves per SIMD, so one wave's
//      VALU work can run beside the other's MFMAs).  Each thread owns one
//      column and half of each chunk's frequencies: it evaluates their
//      basis (FP64 range reduction, hardware sin/cos of revolutions,
//      operand split) into the other of two LDS buffers, interleaved with
//      the MFMAs of the current chunk.  Coefficient fragments are loaded one
//      contraction step ahead, the frequencies two chunks ahead (lanes
//      0..KCH-1 hold one frequency each).  BF16 precisions stage each
//      chunk's frequencies in LDS and read them by broadcast; FP32 reads
//      them from the holding lanes (readlane).
// Blocks are remapped so that the blocks one XCD runs together share a row
// panel and walk the column tiles: each XCD streams a coefficient panel
// through its own L2 once per round of blocks.
// FP32-class precisions (FP32, BF16x6, FP16x3) contract K in ranges of about
// 2048 frequencies; at the end of each range a block stores (first range) or
// adds (posted float atomics, later ranges) its accumulators into its output
// tile and clears them, so FP32 accumulation error grows with the square
// root of the range, not of K.
#include "qrfs_mfma.hpp"

namespace qrfs {

constexpr int WT = 256;  // rows and columns of a block tile

#ifndef QRFS_WIDE_WAVES
#define QRFS_WIDE_WAVES 8
#endif
#ifndef QRFS_WIDE_PHASE
#define QRFS_WIDE_PHASE 1
#endif
#ifndef QRFS_WIDE_ATOMIC_ADD
#define QRFS_WIDE_ATOMIC_ADD 1
#endif

template <int PREC>
struct WideCfg;
template <>
struct WideCfg<1> {             // FP32 MFMA 32x32x2
    static constexpr int KCH = 16;  // frequencies per chunk
    static constexpr int NPL = 1;   // operand planes
    static constexpr int GF = 2;    // frequencies per LDS store
    static constexpr int KB = 8;    // contraction values per fragment
    static constexpr int STR = 2 * KCH + 4;  // elements per LDS column (144 B)
    typedef float T;
    typedef f32x4 Frag;
};
template <>
struct WideCfg<2> {  // split-BF16, 3 products
    static constexpr int KCH = 16;
    static constexpr int NPL = 2;
    static constexpr int GF = 4;
    static constexpr int KB = 16;
    static constexpr int STR = 2 * KCH + 8;  // 80 B
    typedef __bf16 T;
    typedef bf16x8 Frag;
};
template <>
struct WideCfg<3> {  // BF16x6, 6 products
    static constexpr int KCH = 8;
    static constexpr int NPL = 3;
    static constexpr int GF = 4;
    static constexpr int KB = 16;
    static constexpr int STR = 2 * KCH + 8;  // 48 B
    typedef __bf16 T;
    typedef bf16x8 Frag;
};

template <>
struct WideCfg<4> {  // FP16x3: fp16 hi + lo planes (coefficients scaled per set), 3 products
    static constexpr int KCH = 16;
    static constexpr int NPL = 2;
    static constexpr int GF = 4;
    static constexpr int KB = 16;
    static constexpr int STR = 2 * KCH + 8;  // 80 B
    typedef _Float16 T;
    typedef f16x8 Frag;
};

int wide_chunk(int precision) { return precision == 3 ? 8 : 16; }

size_t wide_frag_bytes_per_row32(int precision, int64_t nkv) {
    // one fragment (1 KiB) per plane per KB contraction values
    if (precision == 1) return (size_t)(nkv / 8) * 1024;
    return (size_t)(nkv / 16) * 1024 * (precision == 3 ? 3 : 2);
}

// The 16-bit operand planes of a split precision: bf16 (split-BF16, BF16x6)
// or fp16 (FP16x3), and the matching MFMA.
template <int PREC>
__device__ __forceinline__ void split8_planes(const float (&v)[8],
                                              typename WideCfg<PREC>::Frag (&o)[WideCfg<PREC>::NPL]) {
    if constexpr (PREC == 4)
        split8_f16<false>(v, o);  // interleaved with the MFMAs
    else
        split8_bf16<WideCfg<PREC>::NPL>(v, o);
}
__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) { return mfma_bf16(a, b, c); }
__device__ __forceinline__ f32x16 mfma16(f16x8 a, f16x8 b, f32x16 c) { return mfma_f16(a, b, c); }

// FP16x3: the power of two that puts a set's largest coefficient-tile value
// in [2^13, 2^14) (fp16 holds up to 65504): |w_k c_rk| <= max_k |w_k| times
// the largest coefficient the generators can draw, 8.2 (Box-Muller radius
// sqrt(-2 ln 2^-24) = 5.77 for the Gaussian pair, times sqrt(2) in the Eq. 3
// form).  One block of 1024 threads per set: each set is read once and the
// reduction is latency-bound, so the block is made wide.
constexpr double kCoefMax = 8.2;

__global__ __launch_bounds__(1024) void k_set_scale(const double* __restrict__ w, int64_t K,
                                                    double* __restrict__ ascale) {
    __shared__ double red[16];
    const double* ws = w + (int64_t)blockIdx.x * K;
    double m = 0.0;
    for (int64_t k = threadIdx.x; k < K; k += 1024) m = fmax(m, fabs(ws[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 1; i < 16; ++i) m = fmax(m, red[i]);
        double sc;
        float us;
        f16_scale(m * kCoefMax, sc, us);
        ascale[blockIdx.x] = sc;
    }
}

// ------------------------------------------------------ phase 1 ----
// One thread per (set, 32-row tile, fragment column, lane).  The tiles hold
// w_k c_rk: the frequency's amplitude is applied once per coefficient here
// rather than once per (frequency, point, row tile) in the basis.
template <int PREC, int CSRC>
__global__ __launch_bounds__(256) void k_coef_tiles(WideArgs wa, int64_t n_threads) {
    using C = WideCfg<PREC>;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n_threads) return;
    const SumArgs& a = wa.s;
    const int lane = (int)(g & 63);
    const int64_t NKB = wa.nkv / C::KB;
    int64_t rest = g >> 6;
    const int64_t kb = rest % NKB;
    rest /= NKB;
    const int64_t rt = rest % wa.rt32;
    const int64_t sl = rest / wa.rt32;
    const int64_t set = a.set0 + sl;
    const int64_t set_rows = a.R - set * a.R_block < a.R_block ? a.R - set * a.R_block : a.R_block;
    const int64_t lim = wa.row_off + wa.rows < set_rows ? wa.row_off + wa.rows : set_rows;
    const int64_t row = wa.row_off + rt * 32 + (lane & 31);
    const bool ok = row < lim;
    const uint64_t real = (uint64_t)(set * a.R_block + row);
    const int h = lane >> 5;
    const int64_t twoK = 2 * a.K;
    const double* wk = a.w + sl * a.K;
    const double sc = PREC == 4 ? wa.ascale[sl] : 1.0;  // FP16x3: into the fp16 range
    constexpr int NV = C::KB / 2;  // values per lane: 4 (FP32) or 8 (16-bit planes)
    const int64_t j0 = kb * C::KB + (int64_t)h * NV;
    float v[NV];
#pragma unroll
    for (int q = 0; q < NV; q += 4) {
        float g4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (ok) {
            if constexpr (CSRC == 2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t j = j0 + q + e;
                    g4[e] = j < twoK ? (float)a.coef[(int64_t)real * twoK + j] : 0.0f;
                }
            } else {
                const uint32_t t = (uint32_t)((j0 + q) >> 2);
                if constexpr (CSRC == 0) gauss4_f32(a.seed, a.counter + real, t, g4);
                else coef4_f32(a.seed, a.counter + real, t, 1, g4);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (j0 + q + e >= twoK) g4[e] = 0.0f;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + q + e;
            v[q + e] = j < twoK ? (float)((double)g4[e] * wk[j >> 1] * sc) : 0.0f;
        }
    }
    const int64_t frag = (sl * wa.rt32 + rt) * NKB + kb;
    if constexpr (PREC == 1) {
        f32x4 o = {v[0], v[1], v[2], v[3]};
        ((f32x4*)wa.ctile)[frag * 64 + lane] = o;
    } else {
        typedef typename C::Frag Frag;
        Frag o[C::NPL];
        split8_planes<PREC>(v, o);
#pragma unroll
        for (int p = 0; p < C::NPL; ++p) ((Frag*)wa.ctile)[(frag * C::NPL + p) * 64 + lane] = o[p];
    }
}

// ------------------------------------------------------ phase 2 ----
template <int PREC>
struct WideSmem {
    typedef typename WideCfg<PREC>::T T;
    static constexpr int NPL = WideCfg<PREC>::NPL;
    static constexpr int STR = WideCfg<PREC>::STR;
    __attribute__((aligned(16))) T b[2][NPL][WT * STR];
    // BF16 precisions: (fx, fy) of the chunk whose basis is being built,
    // slot = lane, zeros past the chunk
    double2 fq[PREC >= 2 ? 2 : 1][64];
};

__device__ __forceinline__ double bcast_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Per-block state of the wide kernel: WV waves (4 or 8) in a 2-column
// arrangement, each computing 32 MB rows x 128 columns; every thread
// evaluates the basis of column (tid mod 256) for one of NPART = WV / 4
// interleaved subsets of each chunk's frequency groups.
template <int PREC, int BASIS, int WV>
struct WideTile {
    using C = WideCfg<PREC>;
    typedef typename C::Frag Frag;
    static constexpr int KCH = C::KCH, NPL = C::NPL, STR = C::STR, GF = C::GF;
    static constexpr int MB = 16 / WV;             // 32-row blocks per wave
    static constexpr int NPART = WV / 4;           // threads per column
    static constexpr int NSTEP = 2 * KCH / C::KB;  // fragments per chunk and row block
    static constexpr int NSLOT = NSTEP * 4;        // (step, column block) groups per chunk
    static constexpr int NGRP = KCH / GF / NPART;  // basis groups per thread and chunk
    static_assert(NSLOT == 2 * NPART * NGRP, "one basis group every 2 NPART MFMA groups");

    WideSmem<PREC>& sm;
    const SumArgs& a;
    int lane, r, h, wm, wn, part;
    int64_t sl, c0, nch, NKB;
    const double* fx;
    const double* fy;
    const double* w;
    const Frag* ap;  // this wave's first fragment
    double px, py, pD, pd;
    f32x16 acc[MB][4];

    __device__ __forceinline__ WideTile(WideSmem<PREC>& s, const WideArgs& wa, int64_t sl_,
                                        int64_t rt, int64_t ct)
        : sm(s), a(wa.s), sl(sl_) {
        const int tid = threadIdx.x;
        lane = tid & 63;
        r = lane & 31;
        h = lane >> 5;
        const int wave = tid >> 6;
        wm = wave >> 1;
        wn = wave & 1;
        part = __builtin_amdgcn_readfirstlane(tid >> 8);
        c0 = wa.ch0;
        nch = wa.ch1 - wa.ch0;
        NKB = wa.nkv / C::KB;
        fx = a.fx + sl * a.K;
        fy = a.fy + sl * a.K;
        w = a.w + sl * a.K;
        const int64_t pcol = ct * WT + (tid & (WT - 1));
        const bool pok = pcol < a.P;
        px = pok ? a.px[pcol] : 0.0;
        py = pok ? a.py[pcol] : 0.0;
        pD = 1.0;
        pd = 0.0;
        if (BASIS == BASIS_PISTON && pok) {
            pD = a.apD[pcol];
            pd = a.apd[pcol];
        }
        ap = (const Frag*)wa.ctile + (sl * wa.rt32 + rt * 8 + wm * MB) * NKB * NPL * 64 + lane;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[mb][nb][i] = 0.0f;
    }

    // lanes < KCH load frequency `(c0 + ch) * KCH + lane` (zeros past K);
    // every lane loads from a valid address and selects, without a branch
    __device__ __forceinline__ void load_freq(int64_t ch, double& f0, double& f1, double& f2) const {
        const int64_t k = (c0 + ch) * KCH + lane;
        const bool ok = lane < KCH && k < a.K;
        const int64_t kc = ok ? k : 0;
        f0 = fx[kc];
        f1 = fy[kc];
        f2 = w[kc];
        if (!ok) f0 = f1 = f2 = 0.0;
    }

    // BF16: every wave writes its copy of a chunk's frequencies (identical
    // values; lanes past the chunk hold zeros) into frequency buffer fb
    __device__ __forceinline__ void stage(int fb, const double (&f)[3]) {
        if constexpr (PREC >= 2) sm.fq[fb][lane] = make_double2(f[0], f[1]);
    }

    // fragments of contraction step kb (all row blocks and planes)
    __device__ __forceinline__ void load_step(int64_t kb, Frag (&fa)[MB][NPL]) const {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int p = 0; p < NPL; ++p) fa[mb][p] = ap[((mb * NKB + kb) * NPL + p) * 64];
    }

    // basis of frequencies g*GF .. g*GF+GF-1 of a chunk, this lane's column,
    // into LDS buffer `buf`; (f0, f1, f2) hold the chunk's frequencies in
    // lanes 0 .. KCH-1
    __device__ __forceinline__ void produce(int g, int buf, double f0, double f1, double f2) {
        float v[2 * GF];
#pragma unroll
        for (int i = 0; i < GF; ++i) {
            const int kk = g * GF + i;  // wave-uniform
            // BF16: one LDS read at a wave-uniform address (a broadcast)
            // instead of four lane reads on the vector ALU; FP32, whose
            // MFMAs leave the ALU idle longer, keeps the lane reads
            double cfx, cfy;
            if constexpr (PREC >= 2) {
                const double2 fk = sm.fq[buf][kk];
                cfx = fk.x;
                cfy = fk.y;
            } else {
                cfx = bcast_lane(f0, kk);
                cfy = bcast_lane(f1, kk);
            }
            double t = cfx * px + cfy * py;
            // the amplitude w_k sits in the coefficient tiles; pistons add
            // their aperture's filter (and the gradient factor) here
            double amp = 1.0;
            if (BASIS == BASIS_PISTON) {
                amp = (double)aperture_filter_f32(pD, pd, sqrt(cfx * cfx + cfy * cfy)) *
                      grad_factor(a.grad, a.gx, a.gy, cfx, cfy);
                t += grad_shift(a.grad);
            }
            basis_pair<BASIS>(t, amp, v[2 * i], v[2 * i + 1]);
        }
        const int col = threadIdx.x & (WT - 1);
        if constexpr (PREC == 1) {
            f32x4 o = {v[0], v[1], v[2], v[3]};
            *(f32x4*)&sm.b[buf][0][col * STR + 4 * g] = o;
        } else {
            Frag o[NPL];
            split8_planes<PREC>(v, o);
#pragma unroll
            for (int p = 0; p < NPL; ++p) *(Frag*)&sm.b[buf][p][col * STR + 8 * g] = o[p];
        }
    }

    // MFMAs of one (step, column block) group of the chunk in buffer `buf`
    __device__ __forceinline__ void mfma_group(int st, int nb, int buf, const Frag (&fa)[MB][NPL]) {
        const int col = wn * 128 + nb * 32 + r;
        if constexpr (PREC == 1) {
            const f32x4 bv = *(const f32x4*)&sm.b[buf][0][col * STR + 8 * st + 4 * h];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[mb][0][q], bv[q],
                                                                       acc[mb][nb], 0, 0, 0);
        } else {
            Frag bp[NPL];
#pragma unroll
            for (int p = 0; p < NPL; ++p)
                bp[p] = *(const Frag*)&sm.b[buf][p][col * STR + 16 * st + 8 * h];
            // product-major, so consecutive MFMAs update different
            // accumulators; smallest products first
            constexpr int NPR = NPL == 3 ? 6 : 3;
            // (A plane, B plane) of each product; split-BF16 uses the last 3
            constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
            constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
            constexpr int OFF = 6 - NPR;
#pragma unroll
            for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][nb] = mfma16(fa[mb][PA[pr + OFF]], bp[PB[pr + OFF]], acc[mb][nb]);
        }
    }

    // one chunk: MFMAs of chunk ch (buffer ch & 1) with the fragments of its
    // steps, which alternate between F[PAR] and F[PAR ^ 1]; each step loads
    // the next step's fragments into the other half.  The basis of chunk
    // ch + 1 (frequencies `fcur`) goes into the other buffer, and chunk
    // ch + 2's frequencies are loaded into `fnxt`.
    template <int PAR>
    __device__ __forceinline__ void chunk(int64_t ch, Frag (&F)[2][MB][NPL],
                                          const double (&fcur)[3], double (&fnxt)[3]) {
        const int buf = (int)(ch & 1);
        load_freq(ch + 2, fnxt[0], fnxt[1], fnxt[2]);
#pragma unroll
        for (int st = 0; st < NSTEP; ++st) {
            const int64_t kn = (c0 + ch) * NSTEP + st + 1;
            load_step(kn < (c0 + nch) * NSTEP ? kn : kn - 1, F[(PAR + st + 1) & 1]);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                mfma_group(st, nb, buf, F[(PAR + st) & 1]);
                const int s = st * 4 + nb;
                // the last chunk fills the spare buffer with unused values
#if QRFS_WIDE_PHASE
                if constexpr (NPART == 2 && PREC >= 2) {
                    // the two waves of a SIMD work in opposite phases: the
                    // first four evaluate their basis groups early in the
                    // chunk, the other four late, so one wave's VALU work
                    // runs beside the other's (BF16, matrix-core) MFMAs
                    // instead of in lockstep
                    if (part == 0 ? s < NGRP : s >= NSLOT - NGRP)
                        produce((part == 0 ? s : s - (NSLOT - NGRP)) * NPART + part, buf ^ 1,
                                fcur[0], fcur[1], fcur[2]);
                } else
#endif
                if (s % (2 * NPART) == 2 * NPART - 1)
                    produce((s / (2 * NPART)) * NPART + part, buf ^ 1, fcur[0], fcur[1], fcur[2]);
            }
        }
        // chunk ch + 2 goes into the frequency buffer chunk ch's basis was
        // built from; its last readers passed the barrier ending chunk ch - 1
        stage(buf, fnxt);
    }

    // stores the accumulators into the output (first range of the tile) or
    // adds them to it (later ranges), then clears them.  Elements outside
    // the output go to the sink by a select, not a branch.  The base address
    // and the lane's limits pass through an empty asm statement, so the
    // compiler cannot hoist the element addresses out of the chunk loop.
    __device__ __forceinline__ void store(const WideArgs& wa, int64_t rt, int64_t ct, bool add) {
        const int64_t set = a.set0 + sl;
        const int64_t set_rows =
            a.R - set * a.R_block < a.R_block ? a.R - set * a.R_block : a.R_block;
        const int64_t lim = wa.row_off + wa.rows < set_rows ? wa.row_off + wa.rows : set_rows;
        const int64_t row0 = wa.row_off + rt * WT + wm * 32 * MB + 4 * h;
        const int64_t col0 = ct * WT + wn * 128 + r;
        int64_t base = (set * a.R_block + row0) * a.P + col0;
        int32_t rrem = (int32_t)(lim - row0 < 256 ? lim - row0 : 256);
        int32_t crem = (int32_t)(a.P - col0 < 256 ? a.P - col0 : 256);
        asm volatile("" : "+v"(base), "+v"(rrem), "+v"(crem));
        float* o = (float*)a.out + base;
        float* sink = wa.sink + lane;
        if constexpr (PREC == 4) {
            // FP16x3: the coefficient tiles' power of two comes off exactly
            const float us = (float)(1.0 / wa.ascale[sl]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[mb][nb][i] *= us;
        }
        if (add) {
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int c = mb * 32 + 8 * (i / 4) + (i % 4);
                        const bool ok = c < rrem && nb * 32 < crem;
#if QRFS_WIDE_ATOMIC_ADD
                        // posted float atomic adds (no return value): the
                        // block goes on with the next range while they drain.
                        // Each element is added to by one lane only, in
                        // program order, so the sums are deterministic.
                        if (ok) unsafeAtomicAdd(o + (int64_t)c * a.P + nb * 32, acc[mb][nb][i]);
#else
                        float* p = ok ? o + (int64_t)c * a.P + nb * 32 : sink;
                        *p += acc[mb][nb][i];
#endif
                    }
        } else {
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int c = mb * 32 + 8 * (i / 4) + (i % 4);
                        const bool ok = c < rrem && nb * 32 < crem;
                        float* p = ok ? o + (int64_t)c * a.P + nb * 32 : sink;
                        *p = acc[mb][nb][i];
                    }
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[mb][nb][i] = 0.0f;
    }
};

// One 256 x 256 output tile: rows [rt] of set sl, columns [ct], all
// chunks of wa; every thread of the block calls it (it synchronises).
template <int PREC, int BASIS, int WV>
__device__ __forceinline__ void wide_tile_run(WideSmem<PREC>& sm, const WideArgs& wa, int64_t sl,
                                              int64_t rt, int64_t ct) {
    using Tile = WideTile<PREC, BASIS, WV>;
    typedef typename Tile::Frag Frag;
    constexpr int NSTEP = Tile::NSTEP, NPL = Tile::NPL, MB = Tile::MB, NPART = Tile::NPART;
    Tile T(sm, wa, sl, rt, ct);
    Frag F[2][MB][NPL];
    double fq0[3], fq1[3], fq2[3];
    // prologue: basis of the first chunk, fragments of the first step,
    // frequencies of the second chunk
    T.load_freq(0, fq2[0], fq2[1], fq2[2]);
    T.load_step(T.c0 * NSTEP, F[0]);
    T.load_freq(1, fq0[0], fq0[1], fq0[2]);
    if constexpr (PREC >= 2) {
        T.stage(0, fq2);
        T.stage(1, fq0);
        __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < Tile::NGRP; ++g) T.produce(g * NPART + T.part, 0, fq2[0], fq2[1], fq2[2]);
    __syncthreads();

    // ranges of wa.range_ch chunks (even, so every range starts with the
    // same buffer parity), each ending with a store or an add of the tile;
    // within a range, chunks in pairs, so that the fragment and frequency
    // buffers are named at compile time (NSTEP steps per chunk flip the
    // fragment half NSTEP times).  The pipeline runs on across range ends.
    const int64_t nch = T.nch;
    for (int64_t rs = 0; rs < nch; rs += wa.range_ch) {
        const int64_t re = rs + wa.range_ch < nch ? rs + wa.range_ch : nch;
        for (int64_t ch = rs; ch < re; ch += 2) {
            T.template chunk<0>(ch, F, fq0, fq1);
            __syncthreads();
            if (ch + 1 < re) {
                T.template chunk<NSTEP & 1>(ch + 1, F, fq1, fq0);
                __syncthreads();
            }
        }
        T.store(wa, rt, ct, wa.accumulate || rs > 0);
    }
}

template <int PREC, int BASIS, int WV>
__global__ __launch_bounds__(64 * WV) void k_wide(WideArgs wa) {
    __shared__ WideSmem<PREC> sm;
    // XCD-aware order: consecutive tiles (same row panel, successive column
    // tiles) go to the blocks one XCD runs (blocks are dealt to the 8 XCDs
    // round robin)
    const int64_t nblk = gridDim.x;
    const int64_t b = blockIdx.x;
    const int64_t per = nblk / 8;
    const int64_t t = b < 8 * per ? (b % 8) * per + b / 8 : b;
    const int64_t ct = t % wa.cts;
    const int64_t rt = (t / wa.cts) % wa.rts;
    const int64_t sl = t / (wa.cts * wa.rts);
    wide_tile_run<PREC, BASIS, WV>(sm, wa, sl, rt, ct);
}

// Persistent batch of uneven instances (two-phase form): one block per CU
// pulls work items (instance, set, 256-row tile, 256-column tile) from a
// global counter until the list is exhausted; items come longest first.
// The counter is advanced with a vector atomic by one lane, and every wave
// reaches the exit test on each iteration.  AP: some instances carry
// apertures (pistons or tilts, chosen per item); without it every item is
// a phase item.
template <int PREC, int WV, bool AP>
__global__ __launch_bounds__(64 * WV) void k_wide_batch(const WideArgs* __restrict__ inst,
                                                        const BatchItem* __restrict__ items,
                                                        int n_items,
                                                        unsigned* __restrict__ counter) {
    __shared__ WideSmem<PREC> sm;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const WideArgs wa = inst[w.inst];
        bool piston = false;
        if constexpr (AP) piston = wa.s.apD != nullptr;
        if (piston)
            wide_tile_run<PREC, BASIS_PISTON, WV>(sm, wa, w.set, w.rt, w.ct);
        else
            wide_tile_run<PREC, BASIS_PHASE, WV>(sm, wa, w.set, w.rt, w.ct);
        __syncthreads();
    }
}

// ----------------------------------------------------------- launchers ----
static inline int64_t wcdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int PREC>
static hipError_t launch_coef_t(const WideArgs& wa, hipStream_t st) {
    using C = WideCfg<PREC>;
    const int64_t n_sets = wa.s.set1 - wa.s.set0;
    const int64_t n_threads = n_sets * wa.rt32 * (wa.nkv / C::KB) * 64;
    const dim3 gc((unsigned)wcdiv(n_threads, 256));
    if (wa.s.coef)
        hipLaunchKernelGGL((k_coef_tiles<PREC, 2>), gc, dim3(256), 0, st, wa, n_threads);
    else if (wa.s.mode == 1)
        hipLaunchKernelGGL((k_coef_tiles<PREC, 1>), gc, dim3(256), 0, st, wa, n_threads);
    else
        hipLaunchKernelGGL((k_coef_tiles<PREC, 0>), gc, dim3(256), 0, st, wa, n_threads);
    return hipGetLastError();
}

hipError_t launch_wide_coef(int precision, const WideArgs& wa, hipStream_t st) {
    if (wa.s.set1 <= wa.s.set0) return hipSuccess;
    if (precision == 1) return launch_coef_t<1>(wa, st);
    if (precision == 2) return launch_coef_t<2>(wa, st);
    if (precision == 3) return launch_coef_t<3>(wa, st);
    if (precision == 4) return launch_coef_t<4>(wa, st);
    return hipErrorInvalidValue;
}

hipError_t launch_wide_scale(const double* w, int64_t K, int64_t n_sets, double* ascale,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_set_scale, dim3((unsigned)n_sets), dim3(1024), 0, st, w, K, ascale);
    return hipGetLastError();
}


template <int PREC, int BASIS>
static hipError_t launch_sum_t(const WideArgs& wa, hipStream_t st) {
    constexpr int WV = QRFS_WIDE_WAVES;
    const int64_t blocks = (wa.s.set1 - wa.s.set0) * wa.rts * wa.cts;
    hipLaunchKernelGGL((k_wide<PREC, BASIS, WV>), dim3((unsigned)blocks), dim3(64 * WV), 0, st,
                       wa);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_sum_p(int basis, const WideArgs& wa, hipStream_t st) {
    if (basis == BASIS_PHASE) return launch_sum_t<PREC, BASIS_PHASE>(wa, st);
    if (basis == BASIS_PISTON) return launch_sum_t<PREC, BASIS_PISTON>(wa, st);
    return launch_sum_t<PREC, BASIS_DIFF>(wa, st);
}

template <int PREC>
static hipError_t launch_wide_batch_t(bool ap, const WideArgs* inst, const BatchItem* items,
                                      int n_items, unsigned* counter, int n_blocks,
                                      hipStream_t st) {
    constexpr int WV = QRFS_WIDE_WAVES;
    if (ap)
        hipLaunchKernelGGL((k_wide_batch<PREC, WV, true>), dim3((unsigned)n_blocks), dim3(64 * WV),
                           0, st, inst, items, n_items, counter);
    else
        hipLaunchKernelGGL((k_wide_batch<PREC, WV, false>), dim3((unsigned)n_blocks),
                           dim3(64 * WV), 0, st, inst, items, n_items, counter);
    return hipGetLastError();
}

hipError_t launch_wide_batch(int precision, bool has_ap, const WideArgs* inst,
                             const BatchItem* items, int n_items, unsigned* counter, int n_blocks,
                             hipStream_t st) {
    hipError_t e = launch_reset_counter(counter, st);
    if (e != hipSuccess) return e;
    if (precision == 1)
        return launch_wide_batch_t<1>(has_ap, inst, items, n_items, counter, n_blocks, st);
    if (precision == 2)
        return launch_wide_batch_t<2>(has_ap, inst, items, n_items, counter, n_blocks, st);
    if (precision == 3)
        return launch_wide_batch_t<3>(has_ap, inst, items, n_items, counter, n_blocks, st);
    if (precision == 4)
        return launch_wide_batch_t<4>(has_ap, inst, items, n_items, counter, n_blocks, st);
    return hipErrorInvalidValue;
}

hipError_t launch_wide_sum(int precision, int basis, const WideArgs& wa, hipStream_t st) {
    if (wa.s.set1 <= wa.s.set0 || wa.ch1 <= wa.ch0) return hipSuccess;
    if (precision == 1) return launch_sum_p<1>(basis, wa, st);
    if (precision == 2) return launch_sum_p<2>(basis, wa, st);
    if (precision == 3) return launch_sum_p<3>(basis, wa, st);
    if (precision == 4) return launch_sum_p<4>(basis, wa, st);
    return hipErrorInvalidValue;
}

}  // namespace qrfs
