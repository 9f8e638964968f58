// qrfs_proposal.hip -- learned proposal density for the frequency sampler:
// the 5 -> 128 -> 128 -> 2 network (forward, fused forward + backward,
// fixed-order gradient reduction, Adam), the sampling table (mixture over
// baselines plus a defensive share of the plain density, inverse CDF) and
// the learned R2 sampler with 1/q cell areas.
//
// Density over (ell = ln|f|, theta) for aperture D, outer scale L0 and a
// baseline of length |B| and direction theta_B:
//   q = p(ell) (1 + alpha(ell) cos 2(theta - theta_B)) / (2 pi),
//   p proportional to exp(o0), alpha = 0.9 tanh(o1),
// o = network(2 (ell - lmin)/Lw - 1, 2 theta_B/pi - 1, ln D / 4,
//             ln L0 / 4 - 1, ln|B| / 4 - 1/2).
#include <hip/hip_runtime.h>

#include "qrfs_device.hpp"
#include "qrfs_proposal.hpp"

namespace qrfs {
namespace prop {

constexpr int ROWS = 64;   // rows per block of the network kernels
constexpr int HP = 65;     // padded row stride of the activation tiles

struct RowSpec {
    // rows [0, n_sample) are training samples of context ctxlist[q / m];
    // rows [n_sample, n_sample + n_grid) are normaliser grid points of
    // context ctxlist[(q - n_sample) / G]
    int64_t n_sample, n_grid, m;
    int G;
    const int32_t* ctxlist;
    const double* ctx4;     // [n_ctx][4] = D, L0, |B|, theta_B
    const double* ell;      // training rows
    const double* theta;
    const double* h;
    const float* wgrid;     // dL/do0 of grid rows
    const double* invH;     // 1 / sum of h over the step's sample rows
    double lmin, Lw;
};

__device__ __forceinline__ void features(double ell, const double* c, double lmin, double Lw,
                                         float x[5]) {
    x[0] = (float)(2.0 * (ell - lmin) / Lw - 1.0);
    x[1] = (float)(2.0 * c[3] / 3.141592653589793 - 1.0);
    x[2] = (float)(log(c[0]) / 4.0);
    x[3] = (float)(log(c[1]) / 4.0 - 1.0);
    x[4] = (float)(log(c[2]) / 4.0 - 0.5);
}

struct NetSmem {
    float W1[HID * 5];
    float b1[HID];
    float W2T[HID][HID];   // W2T[k][i] = W2[i][k]
    float b2[HID];
    float W3[2 * HID];
    float b3[2];
    float h1T[HID][HP];    // activations, unit-major, padded
    float h2T[HID][HP];    // layer-2 activations, then dL/d(pre-activation 2)
    float x[ROWS][5];
    float dout[ROWS][2];
    float red[4][ROWS][2];
};

__device__ void load_params(const float* __restrict__ prm, NetSmem& s) {
    for (int i = threadIdx.x; i < HID * 5; i += blockDim.x) s.W1[i] = prm[OFF_W1 + i];
    for (int i = threadIdx.x; i < HID; i += blockDim.x) {
        s.b1[i] = prm[OFF_B1 + i];
        s.b2[i] = prm[OFF_B2 + i];
    }
    for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) {
        const int r = i / HID, k = i % HID;  // W2[r][k]
        s.W2T[k][r] = prm[OFF_W2 + i];
    }
    for (int i = threadIdx.x; i < 2 * HID; i += blockDim.x) s.W3[i] = prm[OFF_W3 + i];
    if (threadIdx.x < 2) s.b3[threadIdx.x] = prm[OFF_B3 + threadIdx.x];
}

// forward of the block's rows (features already in s.x); thread t owns row
// r = t % 64 and units [32 g, 32 g + 32), g = t / 64.  Leaves h1T, h2T and
// writes o[r][2] through `red`.
__device__ void forward_block(NetSmem& s, float o[2]) {
    const int r = threadIdx.x % ROWS;
    const int g = threadIdx.x / ROWS;
    float xr[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) xr[j] = s.x[r][j];
#pragma unroll 4
    for (int ii = 0; ii < 32; ++ii) {
        const int i = 32 * g + ii;
        float a = s.b1[i];
#pragma unroll
        for (int j = 0; j < 5; ++j) a = fmaf(s.W1[i * 5 + j], xr[j], a);
        s.h1T[i][r] = tanhf(a);
    }
    __syncthreads();
    float acc[32];
#pragma unroll
    for (int ii = 0; ii < 32; ++ii) acc[ii] = s.b2[32 * g + ii];
    for (int k = 0; k < HID; ++k) {
        const float hv = s.h1T[k][r];
#pragma unroll
        for (int ii = 0; ii < 32; ++ii) acc[ii] = fmaf(s.W2T[k][32 * g + ii], hv, acc[ii]);
    }
    float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
    for (int ii = 0; ii < 32; ++ii) {
        const int i = 32 * g + ii;
        const float hv = tanhf(acc[ii]);
        s.h2T[i][r] = hv;
        p0 = fmaf(s.W3[i], hv, p0);
        p1 = fmaf(s.W3[HID + i], hv, p1);
    }
    s.red[g][r][0] = p0;
    s.red[g][r][1] = p1;
    __syncthreads();
    o[0] = s.b3[0] + s.red[0][r][0] + s.red[1][r][0] + s.red[2][r][0] + s.red[3][r][0];
    o[1] = s.b3[1] + s.red[0][r][1] + s.red[1][r][1] + s.red[2][r][1] + s.red[3][r][1];
}

__device__ void row_input(const RowSpec& rs, int64_t q, double& ell, const double*& c) {
    if (q < rs.n_sample) {
        const int64_t cs = q / rs.m;
        const int64_t i = (int64_t)rs.ctxlist[cs] * rs.m + q % rs.m;
        ell = rs.ell[i];
        c = rs.ctx4 + 4 * rs.ctxlist[cs];
    } else {
        const int64_t gq = q - rs.n_sample;
        const int64_t cs = gq / rs.G;
        const int j = (int)(gq % rs.G);
        ell = rs.lmin + (j + 0.5) * rs.Lw / rs.G;
        c = rs.ctx4 + 4 * rs.ctxlist[cs];
    }
}

// Forward only: out[q][2] for rows q < n_rows (ell[q], ctx4[q]) or, with
// rs given, for the training/grid rows it describes.
__global__ __launch_bounds__(256) void k_forward(const float* __restrict__ prm, int64_t n_rows,
                                                 const double* __restrict__ ell,
                                                 const double* __restrict__ ctx4, double lmin,
                                                 double Lw, float* __restrict__ out) {
    __shared__ NetSmem s;
    load_params(prm, s);
    const int64_t base = (int64_t)blockIdx.x * ROWS;
    if (threadIdx.x < ROWS) {
        const int64_t q = base + threadIdx.x;
        float x[5] = {0, 0, 0, 0, 0};
        if (q < n_rows) features(ell[q], ctx4 + 4 * q, lmin, Lw, x);
#pragma unroll
        for (int j = 0; j < 5; ++j) s.x[threadIdx.x][j] = x[j];
    }
    __syncthreads();
    float o[2];
    forward_block(s, o);
    const int64_t q = base + threadIdx.x % ROWS;
    if (threadIdx.x < ROWS && q < n_rows) {
        out[2 * q] = o[0];
        out[2 * q + 1] = o[1];
    }
}

// Grid rows of a step: o0 for every (context slot, grid point).
__global__ __launch_bounds__(256) void k_forward_grid(const float* __restrict__ prm,
                                                      RowSpec rs, float* __restrict__ og) {
    __shared__ NetSmem s;
    load_params(prm, s);
    const int64_t base = (int64_t)blockIdx.x * ROWS;
    if (threadIdx.x < ROWS) {
        const int64_t gq = base + threadIdx.x;
        float x[5] = {0, 0, 0, 0, 0};
        if (gq < rs.n_grid) {
            double ell;
            const double* c;
            row_input(rs, rs.n_sample + gq, ell, c);
            features(ell, c, rs.lmin, rs.Lw, x);
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) s.x[threadIdx.x][j] = x[j];
    }
    __syncthreads();
    float o[2];
    forward_block(s, o);
    const int64_t gq = base + threadIdx.x % ROWS;
    if (threadIdx.x < ROWS && gq < rs.n_grid) og[gq] = o[0];
}

// H_c: sum of h over the sample rows of context slot blockIdx.x (fixed order).
__global__ __launch_bounds__(256) void k_hsum(RowSpec rs, double* __restrict__ Hc) {
    __shared__ double r[256];
    const int64_t cs = blockIdx.x;
    const int64_t base = (int64_t)rs.ctxlist[cs] * rs.m;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < rs.m; i += 256) a += rs.h[base + i];
    r[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) Hc[cs] = r[0];
}

// One block: H = sum H_c, 1/H, per context logZ_c = log(sum_j exp(o0_j) Lw/G),
// dL/do0 of the grid rows (H_c/H) softmax_j, and the loss constant
// sum_c (H_c/H) logZ_c.
__global__ __launch_bounds__(256) void k_grid_prep(int64_t n_ctx, int G, double Lw,
                                                   const double* __restrict__ Hc,
                                                   const float* __restrict__ og,
                                                   float* __restrict__ wgrid,
                                                   double* __restrict__ invH,
                                                   double* __restrict__ loss_const) {
    __shared__ double s_invH;
    __shared__ double s_lz[1024];
    if (threadIdx.x == 0) {
        double H = 0.0;
        for (int64_t c = 0; c < n_ctx; ++c) H += Hc[c];
        s_invH = H > 0.0 ? 1.0 / H : 0.0;
        *invH = s_invH;
    }
    __syncthreads();
    for (int64_t c = threadIdx.x; c < n_ctx; c += 256) {
        const float* o = og + c * G;
        double mx = -1e300;
        for (int j = 0; j < G; ++j) mx = fmax(mx, (double)o[j]);
        double se = 0.0;
        for (int j = 0; j < G; ++j) se += exp((double)o[j] - mx);
        const double wc = Hc[c] * s_invH;
        for (int j = 0; j < G; ++j) wgrid[c * G + j] = (float)(wc * exp((double)o[j] - mx) / se);
        if (c < 1024) s_lz[c] = wc * (mx + log(se * Lw / G));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0.0;
        for (int64_t c = 0; c < n_ctx && c < 1024; ++c) L += s_lz[c];
        *loss_const = L;
    }
}

// Fused forward + backward over the step's rows; writes this block's
// gradient contribution gpart[block][NPARAM] and loss contribution.
__global__ __launch_bounds__(256) void k_train(const float* __restrict__ prm, RowSpec rs,
                                               float* __restrict__ gpart,
                                               double* __restrict__ lpart) {
    __shared__ NetSmem s;
    __shared__ float s_wg[ROWS], s_wa[ROWS], s_C[ROWS], s_lw[ROWS];
    __shared__ double s_loss[ROWS];
    load_params(prm, s);
    const int64_t n_rows = rs.n_sample + rs.n_grid;
    const int64_t base = (int64_t)blockIdx.x * ROWS;
    if (threadIdx.x < ROWS) {
        const int64_t q = base + threadIdx.x;
        float x[5] = {0, 0, 0, 0, 0};
        float wg = 0.0f, wa = 0.0f, C = 0.0f, lw = 0.0f;
        if (q < n_rows) {
            double ell;
            const double* c;
            row_input(rs, q, ell, c);
            features(ell, c, rs.lmin, rs.Lw, x);
            if (q < rs.n_sample) {
                const int64_t cs = q / rs.m;
                const int64_t i = (int64_t)rs.ctxlist[cs] * rs.m + q % rs.m;
                const double wi = -rs.h[i] * (*rs.invH);
                wg = (float)wi;
                wa = (float)wi;
                lw = (float)wi;
                C = (float)cos(2.0 * (rs.theta[i] - c[3]));
            } else {
                wg = rs.wgrid[q - rs.n_sample];
            }
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) s.x[threadIdx.x][j] = x[j];
        s_wg[threadIdx.x] = wg;
        s_wa[threadIdx.x] = wa;
        s_C[threadIdx.x] = C;
        s_lw[threadIdx.x] = lw;
    }
    __syncthreads();
    float o[2];
    forward_block(s, o);
    const int r = threadIdx.x % ROWS;
    const int g = threadIdx.x / ROWS;
    if (g == 0) {
        const float ta = tanhf(o[1]);
        const float alpha = 0.9f * ta;
        const float C = s_C[r];
        s.dout[r][0] = s_wg[r];
        s.dout[r][1] = s_wa[r] * C / (1.0f + alpha * C) * 0.9f * (1.0f - ta * ta);
        s_loss[r] = (double)s_lw[r] * ((double)o[0] + log(1.0 + (double)alpha * (double)C));
    }
    __syncthreads();
    float* gp = gpart + (int64_t)blockIdx.x * NPARAM;
    // layer 3: W3[c][i], b3
    {
        const int c = threadIdx.x / HID, i = threadIdx.x % HID;
        float a = 0.0f;
        for (int rr = 0; rr < ROWS; ++rr) a = fmaf(s.dout[rr][c], s.h2T[i][rr], a);
        gp[OFF_W3 + c * HID + i] = a;
        if (threadIdx.x < 2) {
            float b = 0.0f;
            for (int rr = 0; rr < ROWS; ++rr) b += s.dout[rr][threadIdx.x];
            gp[OFF_B3 + threadIdx.x] = b;
        }
    }
    __syncthreads();
    // dL/d(pre-activation 2), overwriting h2T
#pragma unroll 4
    for (int ii = 0; ii < 32; ++ii) {
        const int i = 32 * g + ii;
        const float hv = s.h2T[i][r];
        const float d = s.dout[r][0] * s.W3[i] + s.dout[r][1] * s.W3[HID + i];
        s.h2T[i][r] = d * (1.0f - hv * hv);
    }
    __syncthreads();
    // layer 2: W2[i][k] += sum_r d2[r][i] h1[r][k]; 8 x 8 tile per thread
    {
        const int i0 = (threadIdx.x / 16) * 8, k0 = (threadIdx.x % 16) * 8;
        float acc[8][8];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = 0.0f;
        for (int rr = 0; rr < ROWS; ++rr) {
            float dv[8], hv[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) dv[a] = s.h2T[i0 + a][rr];
#pragma unroll
            for (int b = 0; b < 8; ++b) hv[b] = s.h1T[k0 + b][rr];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] = fmaf(dv[a], hv[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) gp[OFF_W2 + (i0 + a) * HID + k0 + b] = acc[a][b];
        if (threadIdx.x < HID) {
            float b = 0.0f;
            for (int rr = 0; rr < ROWS; ++rr) b += s.h2T[threadIdx.x][rr];
            gp[OFF_B2 + threadIdx.x] = b;
        }
    }
    // dL/d(pre-activation 1): d1[r][k] = (sum_i W2[i][k] d2[r][i]) (1 - h1^2)
    float d1[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) d1[kk] = 0.0f;
    for (int i = 0; i < HID; ++i) {
        const float dv = s.h2T[i][r];
#pragma unroll
        for (int kk = 0; kk < 32; ++kk) d1[kk] = fmaf(s.W2T[32 * g + kk][i], dv, d1[kk]);
    }
    __syncthreads();  // every thread done reading h1T / h2T as layer-2 inputs
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
        const int k = 32 * g + kk;
        const float hv = s.h1T[k][r];
        s.h2T[k][r] = d1[kk] * (1.0f - hv * hv);  // reuse h2T for d1
    }
    __syncthreads();
    // layer 1: W1[k][j] += sum_r d1[r][k] x[r][j]; b1
    for (int e = threadIdx.x; e < HID * 6; e += blockDim.x) {
        const int k = e / 6, j = e % 6;
        float a = 0.0f;
        if (j < 5) {
            for (int rr = 0; rr < ROWS; ++rr) a = fmaf(s.h2T[k][rr], s.x[rr][j], a);
            gp[OFF_W1 + k * 5 + j] = a;
        } else {
            for (int rr = 0; rr < ROWS; ++rr) a += s.h2T[k][rr];
            gp[OFF_B1 + k] = a;
        }
    }
    if (threadIdx.x == 0) {
        double L = 0.0;
        for (int rr = 0; rr < ROWS; ++rr) L += s_loss[rr];
        lpart[blockIdx.x] = L;
    }
}

// grad[p] = sum over blocks (fixed order); loss = sum lpart + loss_const.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ gpart,
                                                     int64_t n_blocks,
                                                     const double* __restrict__ lpart,
                                                     const double* __restrict__ loss_const,
                                                     float* __restrict__ grad,
                                                     double* __restrict__ loss) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        double a = 0.0;
        for (int64_t b = 0; b < n_blocks; ++b) a += (double)gpart[b * NPARAM + p];
        grad[p] = (float)a;
    }
    if (p == 0 && loss) {
        double L = *loss_const;
        for (int64_t b = 0; b < n_blocks; ++b) L += lpart[b];
        *loss = L;
    }
}

// Adam (Kingma & Ba, 2015) with bias correction, step t >= 1.
__global__ void k_adam(float* __restrict__ prm, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float v = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    prm[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Training rows: context c, row r uses R2 point index + 1 + c m + r;
// h = f^2 W F^2 2 (1 - cos(2 pi f |B| cos(theta - theta_B))).
__global__ void k_rows(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_ctx, int64_t m,
                       const double* __restrict__ ctx4, double c_psd, double r0_m53,
                       double fmin, double Lw, double* __restrict__ ell,
                       double* __restrict__ theta, double* __restrict__ h) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ctx * m) return;
    const double* c = ctx4 + 4 * (i / m);
    double ux, uy;
    r2_point(s0x, s0y, index + 1u + (uint64_t)i, ux, uy);
    const double l = log(fmin) + Lw * ux;
    const double th = 2.0 * 3.141592653589793 * uy;
    const double f = exp(l);
    const double W = psd_phase(1, c_psd, r0_m53, 1.0 / (c[1] * c[1]), f);
    const double F = aperture_filter(c[0], 0.0, f);
    const double proj = f * c[2] * cos(th - c[3]);
    ell[i] = l;
    theta[i] = th;
    h[i] = f * f * W * F * F * 2.0 * (1.0 - cospi(2.0 * proj));
}

// Sampling table from the network outputs o[b][j][2] on the cell midpoints
// (one block): per baseline p_b = exp(o0)/Z_b, alpha_b = 0.9 tanh(o1);
// mixture over baselines, defensive share beta of the plain density, CDF.
__global__ __launch_bounds__(256) void k_table(const float* __restrict__ o, int64_t nB,
                                               int n_cells, const double* __restrict__ bth,
                                               double Lw, double beta, double* __restrict__ p,
                                               double* __restrict__ alpha,
                                               double* __restrict__ phi,
                                               double* __restrict__ cdf,
                                               double* __restrict__ scratch) {
    // scratch: [nB] max, [nB] Z
    double* mx = scratch;
    double* Z = scratch + nB;
    const double dl = Lw / n_cells;
    for (int64_t b = threadIdx.x; b < nB; b += blockDim.x) {
        double m = -1e300;
        for (int j = 0; j < n_cells; ++j) m = fmax(m, (double)o[(b * n_cells + j) * 2]);
        double z = 0.0;
        for (int j = 0; j < n_cells; ++j) z += exp((double)o[(b * n_cells + j) * 2] - m) * dl;
        mx[b] = m;
        Z[b] = z;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_cells; j += blockDim.x) {
        double pb = 0.0, A = 0.0, B = 0.0;
        for (int64_t b = 0; b < nB; ++b) {
            const double pj = exp((double)o[(b * n_cells + j) * 2] - mx[b]) / Z[b];
            const double al = 0.9 * tanh((double)o[(b * n_cells + j) * 2 + 1]);
            pb += pj / (double)nB;
            A += pj * al * cos(2.0 * bth[b]) / (double)nB;
            B += pj * al * sin(2.0 * bth[b]) / (double)nB;
        }
        const double pp = (1.0 - beta) * pb + beta / Lw;
        p[j] = pp;
        alpha[j] = (1.0 - beta) * sqrt(A * A + B * B) / pp;
        phi[j] = 0.5 * atan2(B, A);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int j = 0; j < n_cells; ++j) tot += p[j] * dl;
        double run = 0.0;
        for (int j = 0; j < n_cells; ++j) {
            p[j] /= tot;
            cdf[j] = run;
            run += p[j] * dl;
        }
    }
}

// Learned sampler: point n = index + 1 + i; cell j = max{c : cdf[c] <= u1};
// ell = lmin + j dl + (u1 - cdf[j]) / p[j]; t + (alpha/2) sin 2t = 2 pi u2 by
// 12 Newton steps from 2 pi u2; theta = t + phi[j]; area = f^2 / (K q).
__global__ __launch_bounds__(256) void k_sample_learned(
    uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n, int64_t K, double lmin, double Lw,
    int n_cells, const double* __restrict__ tp, const double* __restrict__ ta,
    const double* __restrict__ tphi, const double* __restrict__ tcdf, double* __restrict__ fx,
    double* __restrict__ fy, double* __restrict__ area) {
    __shared__ double sp[MAX_CELLS], sa[MAX_CELLS], sphi[MAX_CELLS], scdf[MAX_CELLS];
    for (int j = threadIdx.x; j < n_cells; j += blockDim.x) {
        sp[j] = tp[j];
        sa[j] = ta[j];
        sphi[j] = tphi[j];
        scdf[j] = tcdf[j];
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ux, uy;
    r2_point(s0x, s0y, index + 1u + (uint64_t)i, ux, uy);
    int lo = 0, hi = n_cells - 1;  // largest j with cdf[j] <= ux (cdf[0] = 0)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (scdf[mid] <= ux) lo = mid;
        else hi = mid - 1;
    }
    const int j = lo;
    const double dl = Lw / n_cells;
    const double ell = lmin + j * dl + (ux - scdf[j]) / sp[j];
    const double target = 2.0 * 3.141592653589793 * uy;
    double t = target;
    const double al = sa[j];
    for (int it = 0; it < 12; ++it) t -= (t + 0.5 * al * sin(2.0 * t) - target) / (1.0 + al * cos(2.0 * t));
    const double th = t + sphi[j];
    const double f = exp(ell);
    const double q = sp[j] * (1.0 + al * cos(2.0 * t)) / (2.0 * 3.141592653589793);
    double s, c;
    sincos(th, &s, &c);
    fx[i] = f * c;
    fy[i] = f * s;
    area[i] = f * f / ((double)K * q);
}

}  // namespace prop

// ----------------------------------------------------------- launchers ----
static inline int64_t cdivp(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t prop_launch_forward(const float* prm, int64_t n, const double* ell, const double* ctx4,
                               double lmin, double Lw, float* out, hipStream_t st) {
    hipLaunchKernelGGL(prop::k_forward, dim3((unsigned)cdivp(n, prop::ROWS)), dim3(256), 0, st,
                       prm, n, ell, ctx4, lmin, Lw, out);
    return hipGetLastError();
}

hipError_t prop_launch_rows(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n_ctx, int64_t m,
                            const double* ctx4, double c_psd, double r0, double fmin, double fmax,
                            double* ell, double* theta, double* h, hipStream_t st) {
    const int64_t n = n_ctx * m;
    hipLaunchKernelGGL(prop::k_rows, dim3((unsigned)cdivp(n, 256)), dim3(256), 0, st, s0x, s0y,
                       index, n_ctx, m, ctx4, c_psd, pow(r0, -5.0 / 3.0), fmin, log(fmax / fmin),
                       ell, theta, h);
    return hipGetLastError();
}

size_t prop_step_scratch_floats(int64_t n_sample, int64_t n_grid) {
    return (size_t)cdivp(n_sample + n_grid, prop::ROWS) * NPARAM;
}

hipError_t prop_launch_loss_grad(const float* prm, int64_t n_ctx, int64_t m, const int32_t* ctxlist,
                                 const double* ctx4, const double* ell, const double* theta,
                                 const double* h, int G, double lmin, double Lw, float* og,
                                 float* wgrid, double* dscratch, float* gpart, float* grad,
                                 double* loss, hipStream_t st) {
    // dscratch: [n_ctx] Hc, invH, loss_const, [n_blocks] lpart
    prop::RowSpec rs;
    rs.n_sample = n_ctx * m;
    rs.n_grid = n_ctx * G;
    rs.m = m;
    rs.G = G;
    rs.ctxlist = ctxlist;
    rs.ctx4 = ctx4;
    rs.ell = ell;
    rs.theta = theta;
    rs.h = h;
    rs.wgrid = wgrid;
    rs.lmin = lmin;
    rs.Lw = Lw;
    double* Hc = dscratch;
    double* invH = dscratch + n_ctx;
    double* lconst = invH + 1;
    double* lpart = lconst + 1;
    rs.invH = invH;
    const int64_t n_blocks = cdivp(rs.n_sample + rs.n_grid, prop::ROWS);
    hipLaunchKernelGGL(prop::k_forward_grid, dim3((unsigned)cdivp(rs.n_grid, prop::ROWS)),
                       dim3(256), 0, st, prm, rs, og);
    hipLaunchKernelGGL(prop::k_hsum, dim3((unsigned)n_ctx), dim3(256), 0, st, rs, Hc);
    hipLaunchKernelGGL(prop::k_grid_prep, dim3(1), dim3(256), 0, st, n_ctx, G, Lw, Hc, og, wgrid,
                       invH, lconst);
    hipLaunchKernelGGL(prop::k_train, dim3((unsigned)n_blocks), dim3(256), 0, st, prm, rs, gpart,
                       lpart);
    hipLaunchKernelGGL(prop::k_grad_reduce, dim3((unsigned)cdivp(NPARAM, 256)), dim3(256), 0, st,
                       gpart, n_blocks, lpart, lconst, grad, loss);
    return hipGetLastError();
}

hipError_t prop_launch_adam(float* prm, float* m1, float* m2, const float* grad, float lr,
                            int64_t t, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(prop::k_adam, dim3((unsigned)cdivp(NPARAM, 256)), dim3(256), 0, st, prm, m1,
                       m2, grad, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t prop_launch_table(const float* o, int64_t nB, int n_cells, const double* bth,
                             double Lw, double beta, double* p, double* alpha, double* phi,
                             double* cdf, double* scratch, hipStream_t st) {
    hipLaunchKernelGGL(prop::k_table, dim3(1), dim3(256), 0, st, o, nB, n_cells, bth, Lw, beta, p,
                       alpha, phi, cdf, scratch);
    return hipGetLastError();
}

hipError_t prop_launch_sample(uint64_t s0x, uint64_t s0y, uint64_t index, int64_t n, int64_t K,
                              double lmin, double Lw, int n_cells, const double* p,
                              const double* alpha, const double* phi, const double* cdf,
                              double* fx, double* fy, double* area, hipStream_t st) {
    hipLaunchKernelGGL(prop::k_sample_learned, dim3((unsigned)cdivp(n, 256)), dim3(256), 0, st,
                       s0x, s0y, index, n, K, lmin, Lw, n_cells, p, alpha, phi, cdf, fx, fy, area);
    return hipGetLastError();
}

}  // namespace qrfs
