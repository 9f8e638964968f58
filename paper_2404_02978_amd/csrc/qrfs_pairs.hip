// qrfs_pairs.hip -- point-set measures of frequency sets: the clashes,
// gaps and discrepancy that Sec. 3.1-3.2 weigh the samplers by.  Built
// without IEEE-mode NaN quieting: every input is a finite coordinate, and
// minima of values loaded from LDS then need no canonicalising instruction.
#include "qrfs_device.hpp"
#include "qrfs_internal.hpp"

namespace qrfs {

constexpr int PM_THREADS = 256;

// Block b = s * n_tiles + bt (set s, point tile bt): thread t owns point
// i = bt * 256 + t of set s, mapped to the unit square
// u = ((fx - x0) / Lx, (fy - y0) / Ly), and visits the points j > i of the
// set (staged 256 at a time in LDS as (x, y) and (1 - x, 1 - y), from its
// own tile on), forming
//   min over j > i of |u_i - u_j|^2,  #{j > i : |u_i - u_j| < r},
//   g(i, i) + 2 sum over j > i of g(i, j),
//       g(i, j) = (1 - max(x_i, x_j)) (1 - max(y_i, y_j))
//               = min(1 - x_i, 1 - x_j) min(1 - y_i, 1 - y_j)
// (rounding is monotone, so both forms give the same factors; Warnock's
// double sum is symmetric in i and j, so each pair is visited once), and
// (1 - x_i^2)(1 - y_i^2).  The block combines its threads in a fixed tree
// and writes part[(s * n_tiles + bt) * 4 + 0..3] = (min d^2, clashes,
// double-sum share, single-sum share).  Squared distances are formed
// without fused multiply-adds, so they round exactly as the plain
// definition does.
__global__ __launch_bounds__(PM_THREADS) void k_pair_measures(const double* __restrict__ fx,
                                                              const double* __restrict__ fy,
                                                              int64_t K, double x0, double y0,
                                                              double Lx, double Ly, double r2,
                                                              int64_t n_tiles,
                                                              double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double2 sxy[PM_THREADS], scc[PM_THREADS];
    __shared__ double red[4][PM_THREADS];
    const int t = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x / n_tiles;
    const int64_t bt = (int64_t)blockIdx.x % n_tiles;
    const int64_t i = bt * PM_THREADS + t;
    const double* px = fx + s * K;
    const double* py = fy + s * K;
    const bool own = i < K;
    const double xi = own ? (px[i] - x0) / Lx : 0.0;
    const double yi = own ? (py[i] - y0) / Ly : 0.0;
    const double cxi = 1.0 - xi, cyi = 1.0 - yi;
    double dmin2 = INFINITY, warn = 0.0;
    uint32_t clash = 0;
    for (int64_t j0 = bt * PM_THREADS; j0 < K; j0 += PM_THREADS) {
        __syncthreads();
        const int64_t jl = j0 + t;
        const double xl = jl < K ? (px[jl] - x0) / Lx : 0.0;
        const double yl = jl < K ? (py[jl] - y0) / Ly : 0.0;
        sxy[t] = make_double2(xl, yl);
        scc[t] = make_double2(1.0 - xl, 1.0 - yl);
        __syncthreads();
        const int nj = K - j0 < PM_THREADS ? (int)(K - j0) : PM_THREADS;
        // in the block's own tile only j > i counts; later tiles are all j > i
        const int jstart = j0 == bt * PM_THREADS ? t + 1 : 0;
#pragma unroll 4
        for (int jj = jstart; jj < nj; ++jj) {
            const double2 p = sxy[jj];
            const double2 c = scc[jj];
            warn = fma(fmin(cxi, c.x), fmin(cyi, c.y), warn);
            const double dx = xi - p.x, dy = yi - p.y;
            const double d2 = dx * dx + dy * dy;
            dmin2 = fmin(dmin2, d2);
            clash += d2 < r2 ? 1u : 0u;
        }
    }
    const double single = own ? (1.0 - xi * xi) * (1.0 - yi * yi) : 0.0;
    const double dbl = own ? cxi * cyi + 2.0 * warn : 0.0;
    red[0][t] = own ? dmin2 : INFINITY;
    red[1][t] = own ? (double)clash : 0.0;
    red[2][t] = dbl;
    red[3][t] = single;
    __syncthreads();
    for (int w = PM_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] = fmin(red[0][t], red[0][t + w]);
            red[1][t] += red[1][t + w];
            red[2][t] += red[2][t + w];
            red[3][t] += red[3][t + w];
        }
        __syncthreads();
    }
    if (t < 4) part[(s * n_tiles + bt) * 4 + t] = red[t][0];
}

// One thread per set: combines the tiles in order and forms the minimum
// distance, the clash count and the L2 star discrepancy
// T = sqrt(1/9 - single / (2K) + double / K^2).
__global__ void k_measures_finish(const double* __restrict__ part, int64_t n_sets,
                                  int64_t n_tiles, int64_t K, double* __restrict__ min_dist,
                                  int64_t* __restrict__ n_clash, double* __restrict__ l2_star) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    double m = INFINITY, c = 0.0, w = 0.0, sg = 0.0;
    for (int64_t b = 0; b < n_tiles; ++b) {
        const double* p = part + (s * n_tiles + b) * 4;
        m = fmin(m, p[0]);
        c += p[1];
        w += p[2];
        sg += p[3];
    }
    const double Kd = (double)K;
    const double T2 = 1.0 / 9.0 - sg / (2.0 * Kd) + w / (Kd * Kd);
    min_dist[s] = sqrt(m);
    n_clash[s] = (int64_t)c;
    l2_star[s] = sqrt(T2 > 0.0 ? T2 : 0.0);
}

static inline int64_t pcdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t measure_tiles(int64_t K) { return pcdiv(K, PM_THREADS); }

hipError_t launch_point_set_measures(int64_t n_sets, int64_t K, const double* fx,
                                     const double* fy, double x0, double y0, double Lx, double Ly,
                                     double r_clash, double* part, double* min_dist,
                                     int64_t* n_clash, double* l2_star, hipStream_t st) {
    const int64_t nt = measure_tiles(K);
    hipLaunchKernelGGL(k_pair_measures, dim3((unsigned)(nt * n_sets)), dim3(PM_THREADS), 0, st, fx,
                       fy, K, x0, y0, Lx, Ly, r_clash * r_clash, nt, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_measures_finish, dim3((unsigned)pcdiv(n_sets, 256)), dim3(256), 0, st,
                       part, n_sets, nt, K, min_dist, n_clash, l2_star);
    return hipGetLastError();
}

}  // namespace qrfs
