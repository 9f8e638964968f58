// qrfs_internal.hpp -- launchers shared by the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrfs {

// Exact Kolmogorov constant of the phase PSD in cycles/m,
// Gamma(11/6)^2 / (2 pi^(11/3)) (24/5 Gamma(6/5))^(5/6) (Eq. 7 prints 0.02289).
constexpr double kPsdConstant = 0.022895587108555181;

// The PSD constant the weight kernels use: c (or kPsdConstant for c <= 0),
// times (lambda / 2 pi)^2 when outputs are optical path (wavelength > 0):
// w = sqrt(W area) is then lambda / (2 pi) times the phase weight (Sec. 4.4).
inline double psd_constant(double c, double wavelength) {
    double k = c > 0.0 ? c : kPsdConstant;
    if (wavelength > 0.0) {
        const double s = wavelength / (2.0 * 3.141592653589793);
        k *= s * s;
    }
    return k;
}

enum Basis : int {
    BASIS_PHASE = 0,   // (cos, sin)(2 pi f.x_p) w_k
    BASIS_PISTON = 1,  // (cos, sin)(2 pi f.c_p) w_k F(D_p, d_p, |f_k|)
    BASIS_DIFF = 2,    // (cos 2 pi f.B_p - 1, sin 2 pi f.B_p) w_k
};

enum Epilogue : int {
    EPI_STORE = 0,  // write the sums [R][P]
    EPI_SFSUM = 1,  // per column: sum of squares and fourth powers over rows
};

// One launch of the fused coefficient x basis contraction over the sets
// [set0, set1).  Frequency arrays hold those sets contiguously: set s at
// offset (s - set0) * K.
struct SumArgs {
    int64_t K;
    const double* fx;
    const double* fy;
    const double* w;
    int64_t P;
    const double* px;
    const double* py;
    const double* apD;  // BASIS_PISTON only
    const double* apd;
    int64_t R;
    int64_t R_block;
    int64_t set0;
    int64_t set1;
    uint64_t seed;
    uint64_t counter;
    int32_t mode;
    const double* coef;  // [R][2K] or nullptr
    void* out;           // EPI_STORE: float or double [R][P]
    double* partial;     // EPI_SFSUM, ksplit == 1: [row tiles of this launch][P][2]
    int32_t ksplit;      // frequency ranges per row tile (MFMA kernels, EPI_SFSUM)
    int64_t kspan;       // frequencies per range (multiple of the chunk length)
    float* phi_part;     // EPI_SFSUM, ksplit > 1: [ksplit][R][P] partial sums
    // BASIS_PISTON, grad != 0: the gradient of the piston along u (G-tilt)
    // instead of the piston: amplitudes times gx f_x + gy f_y with
    // (gx, gy) = 2 pi u, arguments shifted by a quarter cycle
    int32_t grad;
    double gx, gy;
};

// The two-phase contraction (wide point sets) over the sets [s.set0,
// s.set1), rows [row_off, row_off + rows) of each set: launch_wide_coef
// writes the coefficient tiles of all frequencies, then launch_wide_sum
// contracts the frequency chunks [ch0, ch1) into 256 x 256 output tiles
// (EPI_STORE, float output).
struct WideArgs {
    SumArgs s;        // fx / fy / w start at set s.set0
    int64_t row_off;  // first row of each set covered by this launch
    int64_t rows;     // rows of each set covered (the last set may hold fewer)
    int64_t rt32;     // 32-row coefficient tiles per set in `ctile` (8 per block tile)
    int64_t rts;      // 256-row block tiles per set
    int64_t cts;      // 256-column block tiles
    int64_t nkv;      // contraction length 2K padded to whole chunks
    int64_t ch0, ch1; // chunks [ch0, ch1) of frequencies this launch contracts
    int64_t range_ch; // chunks per accumulation range (even), each ending with
                      // an add of the tile into the output
    int32_t accumulate;  // 0: the first range stores its sums, 1: it adds them
    void* ctile;      // coefficient tiles
    float* sink;      // 64 floats that absorb the stores of elements outside the output
    const double* ascale;  // FP16x3: per set of the launch, the power of two of its tiles
};
// frequencies per chunk of the two-phase kernel, and the bytes of
// coefficient tiles per 32 rows for a padded contraction length nkv
int wide_chunk(int precision);
size_t wide_frag_bytes_per_row32(int precision, int64_t nkv);
hipError_t launch_wide_coef(int precision, const WideArgs& wa, hipStream_t st);
// FP16x3: per set, the power of two that scales its coefficient tiles into
// the fp16 range (from the set's largest weight); n_sets blocks.
hipError_t launch_wide_scale(const double* w, int64_t K, int64_t n_sets, double* ascale,
                             hipStream_t st);
hipError_t launch_wide_sum(int precision, int basis, const WideArgs& wa, hipStream_t st);

// How the structure-function sums are split for a problem: ksplit
// frequency ranges per row tile, the FP32 partial-sum buffer it needs, and
// the number of partial rows the final reduction reads.
struct SfPlan {
    int ksplit;
    int64_t kspan;
    size_t phi_floats;
    int64_t n_partial_tiles;
};
// max_bytes > 0 bounds the scratch the plan needs (split-K partial sums
// plus per-tile partials, each rounded up to 256 bytes) by taking fewer
// frequency ranges; the plan may still exceed it with one range.
SfPlan sf_plan(int precision, int64_t K, int64_t R, int64_t R_block, int64_t P,
               size_t max_bytes = 0);
size_t sf_plan_bytes(const SfPlan& p, int64_t P);
// Sets of one realisation and at most 64 baselines: the structure function
// runs in k_sf_one (one block per realisation, one partial tile per set).
bool sf_one_realisation(int64_t R_block, int64_t P);

// One work item of a persistent batch: instance, set, row tile, column tile.
struct BatchItem {
    int32_t inst;
    int32_t set;
    int32_t rt;
    int32_t ct;
};

// Launch shape of the persistent batch kernel: rows per wave (32 MW),
// columns per block (32 NB), resident blocks per CU of the grid; `wide`
// selects the two-phase form (coefficient tiles, 256 x 256 items).
struct BatchShape {
    int MW, NB, blocks_per_cu, wide;
};
int batch_shape_count(int precision);
BatchShape batch_shape(int precision, int id);

// Resets the work counter and launches the persistent kernel (256 threads
// per block, n_blocks blocks) over items[0 .. n_items).
// has_ap: some instance carries apertures (a.apD set), and the kernel
// chooses the piston basis for its items.
hipError_t launch_batch(int precision, BatchShape shape, bool has_ap, const SumArgs* inst,
                        const BatchItem* items, int n_items, unsigned* counter, int n_blocks,
                        hipStream_t st);

// Resets the work counter and launches the persistent two-phase kernel
// (n_blocks blocks) over items[0 .. n_items) of the instances `inst`
// (device array; coefficient tiles already written).
hipError_t launch_wide_batch(int precision, bool has_ap, const WideArgs* inst,
                             const BatchItem* items, int n_items, unsigned* counter, int n_blocks,
                             hipStream_t st);
hipError_t launch_reset_counter(unsigned* counter, hipStream_t st);

// Point-set measures (qrfs_measures.hip): per set, `part` holds
// measure_tiles(K) * 4 doubles of partial results.
int64_t measure_tiles(int64_t K);
hipError_t launch_point_set_measures(int64_t n_sets, int64_t K, const double* fx,
                                     const double* fy, double x0, double y0, double Lx, double Ly,
                                     double r_clash, double* part, double* min_dist,
                                     int64_t* n_clash, double* l2_star, hipStream_t st);
hipError_t launch_set_sf(int64_t n_sets, int64_t K, const double* fx, const double* fy,
                         const double* w, int64_t nB, const double* bx, const double* by,
                         double* S, hipStream_t st);

// squares of the K-range partial sums, summed per column over blocks of
// rows: partial[ceil(R/256)][P][2]
hipError_t launch_sfsum_rows(const float* phi, int ksplit, int64_t R, int64_t P, double* partial,
                             hipStream_t st);

// Row tiles one set occupies in `launch_sum` for this precision and R_block
// (needed to size the partial-sum buffer).
int64_t sum_row_tiles_per_set(int precision, int basis, int64_t R_block, int64_t P);
int64_t sum_col_tiles(int precision, int basis, int64_t R_block, int64_t P);

hipError_t launch_sum(int precision, int basis, int epi, const SumArgs& a, hipStream_t st);

hipError_t launch_sample(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_sets,
                         int64_t K, int32_t N, double df, double fmin, double fmax, double* fx,
                         double* fy, double* area, hipStream_t st);

// f32: weights for FP32-class sums (every factor to binary32 accuracy, the
// filter by the binary32-class J1); 0: every step in binary64.
hipError_t launch_weights(int model, double c, double r0, double L0, int has_ap, double D,
                          double d, int f32, int64_t n, const double* fx, const double* fy,
                          const double* area, double* w, hipStream_t st);

// launch_sample followed by launch_weights in one kernel (the same values),
// writing the frequencies and the weights but not the cell areas.
hipError_t launch_sample_weights(int scheme, uint64_t s0x, uint64_t s0y, uint64_t index,
                                 int64_t n_sets, int64_t K, int32_t N, double df, double fmin,
                                 double fmax, int model, double c, double r0, double L0,
                                 int has_ap, double D, double d, int f32, double* fx,
                                 double* fy, double* w, hipStream_t st);

// Frozen-flow temporal structure function (time series of M <= 4096 points).
constexpr int TEMPORAL_MAX_M = 4096;
constexpr int TEMPORAL_ROWS_PER_BLOCK = 8;
// points c1 - v m dt (m < M), then c2 - v m dt
hipError_t launch_taylor_points(const double c1[2], const double c2[2], const double v[2],
                                double dt, int64_t M, double* px, double* py, hipStream_t st);
// blocks of TEMPORAL_ROWS_PER_BLOCK realisations that launch_temporal_rows uses
int64_t temporal_blocks(int64_t R);
// pist [R][2][M] (double when fp64, else float) -> part[temporal_blocks(R)][M][2]
hipError_t launch_temporal_rows(bool fp64, const void* pist, int64_t R, int64_t M, double* part,
                                hipStream_t st);

// sf[p] = S2/R, stderr[p] from partial[n_tiles][P][2] in a fixed order.
hipError_t launch_reduce_sf(const double* partial, int64_t n_tiles, int64_t P, int64_t R,
                            double* sf, double* sf_stderr, hipStream_t st);

}  // namespace qrfs
