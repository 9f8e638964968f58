// qrfs_proposal.hpp -- sizes and launchers of the learned proposal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrfs {

constexpr int HID = 128;  // hidden width of the 5 -> 128 -> 128 -> 2 network
// flat parameter layout: W1[H][5], b1[H], W2[H][H], b2[H], W3[2][H], b3[2]
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + 5 * HID;
constexpr int OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID;
constexpr int OFF_B3 = OFF_W3 + 2 * HID;
constexpr int NPARAM = OFF_B3 + 2;  // 17538
constexpr int MAX_CELLS = 1024;     // cells of a sampling table

hipError_t prop_launch_forward(const float* prm, int64_t n, const double* ell, const double* ctx4,
                               double lmin, double Lw, float* out, hipStream_t st);
hipError_t prop_launch_rows(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_ctx, int64_t m,
                            const double* ctx4, double c_psd, double r0, double fmin, double fmax,
                            double* ell, double* theta, double* h, hipStream_t st);
size_t prop_step_scratch_floats(int64_t n_sample, int64_t n_grid);
hipError_t prop_launch_loss_grad(const float* prm, int64_t n_ctx, int64_t m, const int32_t* ctxlist,
                                 const double* ctx4, const double* ell, const double* theta,
                                 const double* h, int G, double lmin, double Lw, float* og,
                                 float* wgrid, double* dscratch, float* gpart, float* grad,
                                 double* loss, hipStream_t st);
hipError_t prop_launch_adam(float* prm, float* m1, float* m2, const float* grad, float lr,
                            int64_t t, hipStream_t st);
hipError_t prop_launch_table(const float* o, int64_t nB, int n_cells, const double* bth,
                             double Lw, double beta, double* p, double* alpha, double* phi,
                             double* cdf, double* scratch, hipStream_t st);
hipError_t prop_launch_sample(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n, int64_t K,
                              double lmin, double Lw, int n_cells, const double* p,
                              const double* alpha, const double* phi, const double* cdf,
                              double* fx, double* fy, double* area, hipStream_t st);

}  // namespace qrfs
