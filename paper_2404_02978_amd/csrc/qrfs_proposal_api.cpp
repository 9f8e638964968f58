// qrfs_proposal_api.cpp -- C ABI of the learned proposal: parameters and
// Adam state, training loop, sampling table, learned sampler dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "qrfs.h"
#include "qrfs_internal.hpp"
#include "qrfs_proposal.hpp"

// rows of one loss/gradient or training step (plus at most 4M grid rows):
// the network kernels take 64 rows per 256-thread block, so this keeps a
// launch well within 2^32 work-items
static constexpr int64_t kMaxStepRows = (int64_t)1 << 29;

namespace qrfs {
qrfs_status api_fail(qrfs_status s, const char* fmt, ...);
qrfs_status api_ok();
int api_context_device(const qrfs_context* ctx);
}  // namespace qrfs

struct qrfs_proposal {
    int device = 0;
    double fmin = 0, fmax = 0, lmin = 0, Lw = 0;
    float* prm = nullptr;  // [NPARAM]
    float* m1 = nullptr;
    float* m2 = nullptr;
    float* grad = nullptr;
    int64_t t = 0;  // Adam steps taken
    int n_cells = 0;
    double* table = nullptr;  // p, alpha, phi, cdf: 4 x MAX_CELLS
    void* ws = nullptr;
    size_t ws_size = 0;
};

namespace {

using qrfs::api_fail;
using qrfs::api_ok;

struct Guard {
    int prev = -1;
    bool okay = false;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        okay = hipSetDevice(dev) == hipSuccess;
    }
    ~Guard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

qrfs_status hfail(hipError_t e, const char* what) {
    return api_fail(QRFS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool al8(const void* p) { return ((uintptr_t)p & 7u) == 0; }
bool al4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

qrfs_status workspace(qrfs_proposal* p, size_t bytes) {
    if (bytes <= p->ws_size) return QRFS_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hfail(e, "synchronise before workspace growth");
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_size = 0;
    e = hipMalloc(&p->ws, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return api_fail(QRFS_ERR_OUT_OF_MEMORY, "proposal workspace of %zu bytes", bytes);
    }
    p->ws_size = bytes;
    return QRFS_OK;
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// scratch of one loss/gradient evaluation over n_ctx contexts
struct StepScratch {
    float* og;
    float* wgrid;
    double* dscr;
    float* gpart;
    int32_t* ctxlist;
};

qrfs_status step_scratch(qrfs_proposal* p, int64_t n_ctx, int64_t m, int G, int64_t list_len,
                         StepScratch& s) {
    const int64_t n_grid = n_ctx * G;
    const int64_t n_blocks = (n_ctx * m + n_grid + 63) / 64;
    size_t o = 0;
    const size_t og = o;
    o += a256(sizeof(float) * n_grid);
    const size_t wg = o;
    o += a256(sizeof(float) * n_grid);
    const size_t ds = o;
    o += a256(sizeof(double) * (n_ctx + 2 + n_blocks));
    const size_t gp = o;
    o += a256(sizeof(float) * qrfs::prop_step_scratch_floats(n_ctx * m, n_grid));
    const size_t cl = o;
    o += a256(sizeof(int32_t) * list_len);
    qrfs_status st = workspace(p, o);
    if (st) return st;
    char* b = (char*)p->ws;
    s.og = (float*)(b + og);
    s.wgrid = (float*)(b + wg);
    s.dscr = (double*)(b + ds);
    s.gpart = (float*)(b + gp);
    s.ctxlist = (int32_t*)(b + cl);
    return QRFS_OK;
}

// splitmix64 (Steele, Lea, Flood 2014): context order of each epoch
uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

namespace qrfs {
// used by the sampler entry points for QRFS_SAMPLER_LEARNED
qrfs_status proposal_check_ready(const qrfs_proposal* p) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "LEARNED sampler without a proposal");
    if (p->n_cells <= 0)
        return api_fail(QRFS_ERR_INVALID_ARG, "the proposal has no sampling table yet");
    return QRFS_OK;
}

hipError_t proposal_sample(const qrfs_proposal* p, uint64_t s0x, uint64_t s0y, uint64_t index,
                           int64_t n_sets, int64_t K, double* fx, double* fy, double* area,
                           hipStream_t st) {
    const double* T = p->table;
    return prop_launch_sample(s0x, s0y, index, n_sets * K, K, p->lmin, p->Lw, p->n_cells, T,
                              T + MAX_CELLS, T + 2 * MAX_CELLS, T + 3 * MAX_CELLS, fx, fy, area,
                              st);
}
}  // namespace qrfs

extern "C" {

qrfs_status qrfs_proposal_create(qrfs_context* ctx, double fmin, double fmax,
                                 const float* init_params, qrfs_proposal** out) {
    if (!out) return api_fail(QRFS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!(fmin > 0.0) || !(fmax > fmin) || !std::isfinite(fmax))
        return api_fail(QRFS_ERR_INVALID_ARG, "needs 0 < fmin < fmax");
    if (!init_params || !al4(init_params))
        return api_fail(QRFS_ERR_INVALID_ARG, "init_params NULL or misaligned");
    if (!ctx) return api_fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    const int dev = qrfs::api_context_device(ctx);
    Guard g(dev);
    if (!g.okay) return api_fail(QRFS_ERR_DEVICE, "cannot select device %d", dev);
    qrfs_proposal* p = new (std::nothrow) qrfs_proposal();
    if (!p) return api_fail(QRFS_ERR_OUT_OF_MEMORY, "host allocation of the proposal");
    p->device = dev;
    p->fmin = fmin;
    p->fmax = fmax;
    p->lmin = std::log(fmin);
    p->Lw = std::log(fmax / fmin);
    hipError_t e = hipMalloc(&p->prm, sizeof(float) * qrfs::NPARAM * 4);
    if (e == hipSuccess) e = hipMalloc(&p->table, sizeof(double) * 4 * qrfs::MAX_CELLS);
    if (e != hipSuccess) {
        qrfs_proposal_destroy(p);
        return api_fail(QRFS_ERR_OUT_OF_MEMORY, "proposal buffers");
    }
    p->m1 = p->prm + qrfs::NPARAM;
    p->m2 = p->m1 + qrfs::NPARAM;
    p->grad = p->m2 + qrfs::NPARAM;
    e = hipMemcpy(p->prm, init_params, sizeof(float) * qrfs::NPARAM, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemset(p->m1, 0, sizeof(float) * qrfs::NPARAM * 2);
    if (e != hipSuccess) {
        qrfs_proposal_destroy(p);
        return hfail(e, "proposal initialisation");
    }
    *out = p;
    return api_ok();
}

qrfs_status qrfs_proposal_destroy(qrfs_proposal* p) {
    if (!p) return api_ok();
    {
        Guard g(p->device);
        (void)hipDeviceSynchronize();
        if (p->prm) (void)hipFree(p->prm);
        if (p->table) (void)hipFree(p->table);
        if (p->ws) (void)hipFree(p->ws);
    }
    delete p;
    return api_ok();
}

qrfs_status qrfs_proposal_get_params(const qrfs_proposal* p, float* dst, void* stream) {
    if (!p || !dst || !al4(dst)) return api_fail(QRFS_ERR_INVALID_ARG, "bad proposal or dst");
    Guard g(p->device);
    hipError_t e = hipMemcpyAsync(dst, p->prm, sizeof(float) * qrfs::NPARAM,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? api_ok() : hfail(e, "copy parameters");
}

qrfs_status qrfs_proposal_set_params(qrfs_proposal* p, const float* src, void* stream) {
    if (!p || !src || !al4(src)) return api_fail(QRFS_ERR_INVALID_ARG, "bad proposal or src");
    Guard g(p->device);
    hipError_t e = hipMemcpyAsync(p->prm, src, sizeof(float) * qrfs::NPARAM,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? api_ok() : hfail(e, "copy parameters");
}

qrfs_status qrfs_proposal_forward(qrfs_proposal* p, int64_t n, const double* ell,
                                  const double* ctx4, float* out, void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    // 64 points per 256-thread block: at most 2^30 - 2^16 points keep the
    // launch within 2^32 work-items
    if (n <= 0 || n > ((int64_t)1 << 30) - ((int64_t)1 << 16))
        return api_fail(QRFS_ERR_INVALID_ARG, "n must be in 1..2^30 - 2^16");
    if (!ell || !ctx4 || !out || !al8(ell) || !al8(ctx4) || !al4(out))
        return api_fail(QRFS_ERR_INVALID_ARG, "NULL or misaligned array");
    Guard g(p->device);
    hipError_t e = qrfs::prop_launch_forward(p->prm, n, ell, ctx4, p->lmin, p->Lw, out,
                                             (hipStream_t)stream);
    return e == hipSuccess ? api_ok() : hfail(e, "forward launch");
}

qrfs_status qrfs_proposal_rows(qrfs_proposal* p, qrfs_sampler* plain, int64_t n_ctx, int64_t m,
                               const double* ctx4, double r0, double c_psd, double* ell,
                               double* theta, double* h, void* stream) {
    if (!p || !plain) return api_fail(QRFS_ERR_INVALID_ARG, "proposal or sampler is NULL");
    if (plain->scheme != QRFS_SAMPLER_R2_LOGPOLAR)
        return api_fail(QRFS_ERR_INVALID_ARG, "training rows need the plain log-polar sampler");
    if (plain->fmin != p->fmin || plain->fmax != p->fmax)
        return api_fail(QRFS_ERR_INVALID_ARG, "sampler band differs from the proposal's");
    if (n_ctx <= 0 || m <= 0 || n_ctx > QRFS_MAX_POINTS_PER_CALL / m)
        return api_fail(QRFS_ERR_INVALID_ARG,
                        "n_ctx and m must be >= 1 with n_ctx * m <= QRFS_MAX_POINTS_PER_CALL");
    if (!(r0 > 0.0)) return api_fail(QRFS_ERR_INVALID_ARG, "r0 must be > 0");
    if (!ctx4 || !ell || !theta || !h || !al8(ctx4) || !al8(ell) || !al8(theta) || !al8(h))
        return api_fail(QRFS_ERR_INVALID_ARG, "NULL or misaligned array");
    Guard g(p->device);
    const double c = c_psd > 0.0 ? c_psd : qrfs::kPsdConstant;
    hipError_t e = qrfs::prop_launch_rows(plain->seed_x, plain->seed_y, plain->index, n_ctx, m,
                                          ctx4, c, r0, p->fmin, p->fmax, ell, theta, h,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hfail(e, "rows launch");
    plain->index += (uint64_t)(n_ctx * m);
    return api_ok();
}

qrfs_status qrfs_proposal_loss_grad(qrfs_proposal* p, int64_t n_ctx, int64_t m,
                                    const double* ctx4, const double* ell, const double* theta,
                                    const double* h, int32_t G, float* grad, double* loss,
                                    void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    if (n_ctx <= 0 || n_ctx > 1024 || m <= 0 || G < 1 || G > 4096)
        return api_fail(QRFS_ERR_INVALID_ARG, "need 1 <= n_ctx <= 1024, m >= 1, 1 <= G <= 4096");
    // rows of one step, 64 per 256-thread block, within 2^32 work-items
    if (n_ctx * m > kMaxStepRows)
        return api_fail(QRFS_ERR_INVALID_ARG, "n_ctx * m must be <= 2^29");
    if (!ctx4 || !ell || !theta || !h || !grad || !al8(ctx4) || !al8(ell) || !al8(theta) ||
        !al8(h) || !al4(grad) || (loss && !al8(loss)))
        return api_fail(QRFS_ERR_INVALID_ARG, "NULL or misaligned array");
    Guard g(p->device);
    StepScratch s;
    qrfs_status st = step_scratch(p, n_ctx, m, G, n_ctx, s);
    if (st) return st;
    std::vector<int32_t> ids(n_ctx);
    for (int64_t c = 0; c < n_ctx; ++c) ids[c] = (int32_t)c;
    hipStream_t strm = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(s.ctxlist, ids.data(), sizeof(int32_t) * n_ctx,
                                  hipMemcpyHostToDevice, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    if (e == hipSuccess)
        e = qrfs::prop_launch_loss_grad(p->prm, n_ctx, m, s.ctxlist, ctx4, ell, theta, h, G,
                                        p->lmin, p->Lw, s.og, s.wgrid, s.dscr, s.gpart, grad,
                                        loss, strm);
    return e == hipSuccess ? api_ok() : hfail(e, "loss/gradient");
}

qrfs_status qrfs_proposal_train(qrfs_proposal* p, int64_t n_ctx, int64_t m, const double* ctx4,
                                const double* ell, const double* theta, const double* h,
                                int64_t ctx_per_step, int64_t steps, int32_t G, double lr,
                                uint64_t shuffle_seed, double* loss_log, void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    if (n_ctx <= 0 || m <= 0 || ctx_per_step <= 0 || ctx_per_step > 1024 ||
        ctx_per_step > n_ctx || steps <= 0 || G < 1 || G > 4096 || !(lr > 0.0))
        return api_fail(QRFS_ERR_INVALID_ARG, "bad training sizes or learning rate");
    if (n_ctx > 0x7fffffff) return api_fail(QRFS_ERR_INVALID_ARG, "too many contexts");
    if (ctx_per_step * m > kMaxStepRows)
        return api_fail(QRFS_ERR_INVALID_ARG, "ctx_per_step * m must be <= 2^29");
    if (!ctx4 || !ell || !theta || !h || !al8(ctx4) || !al8(ell) || !al8(theta) || !al8(h) ||
        (loss_log && !al8(loss_log)))
        return api_fail(QRFS_ERR_INVALID_ARG, "NULL or misaligned array");
    Guard g(p->device);
    // context order of every step, epochs reshuffled (Fisher-Yates)
    std::vector<int32_t> order(n_ctx), list((size_t)(steps * ctx_per_step));
    for (int64_t c = 0; c < n_ctx; ++c) order[c] = (int32_t)c;
    uint64_t rs = shuffle_seed;
    int64_t pos = n_ctx;
    for (int64_t i = 0; i < steps * ctx_per_step; ++i) {
        if (pos == n_ctx) {
            for (int64_t k = n_ctx - 1; k > 0; --k) {
                int64_t j = (int64_t)(splitmix(rs) % (uint64_t)(k + 1));
                std::swap(order[k], order[j]);
            }
            pos = 0;
        }
        list[i] = order[pos++];
    }
    // a context may repeat inside one step only if ctx_per_step straddles
    // an epoch boundary; each step still sees ctx_per_step contexts
    StepScratch s;
    qrfs_status st = step_scratch(p, ctx_per_step, m, G, (int64_t)list.size(), s);
    if (st) return st;
    hipStream_t strm = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(s.ctxlist, list.data(), sizeof(int32_t) * list.size(),
                                  hipMemcpyHostToDevice, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    if (e != hipSuccess) return hfail(e, "upload of the context order");
    for (int64_t k = 0; k < steps; ++k) {
        e = qrfs::prop_launch_loss_grad(p->prm, ctx_per_step, m, s.ctxlist + k * ctx_per_step,
                                        ctx4, ell, theta, h, G, p->lmin, p->Lw, s.og, s.wgrid,
                                        s.dscr, s.gpart, p->grad,
                                        loss_log ? loss_log + k : nullptr, strm);
        if (e != hipSuccess) return hfail(e, "training step");
        p->t += 1;
        e = qrfs::prop_launch_adam(p->prm, p->m1, p->m2, p->grad, (float)lr, p->t, strm);
        if (e != hipSuccess) return hfail(e, "Adam step");
    }
    return api_ok();
}

qrfs_status qrfs_proposal_tabulate(qrfs_proposal* p, double D, double L0, int64_t nB,
                                   const double* blen, const double* bth, int32_t n_cells,
                                   double beta, void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    if (!(D > 0.0) || !(L0 > 0.0) || nB <= 0 || nB > 65536 || !blen || !bth)
        return api_fail(QRFS_ERR_INVALID_ARG, "bad geometry");
    for (int64_t b = 0; b < nB; ++b)
        if (!(blen[b] > 0.0) || !std::isfinite(bth[b]))
            return api_fail(QRFS_ERR_INVALID_ARG, "baseline %lld: length must be > 0",
                            (long long)b);
    if (n_cells < 1 || n_cells > qrfs::MAX_CELLS)
        return api_fail(QRFS_ERR_INVALID_ARG, "n_cells must be in [1, %d]", qrfs::MAX_CELLS);
    if (!(beta > 0.0) || beta > 1.0) return api_fail(QRFS_ERR_INVALID_ARG, "beta must be in (0, 1]");
    Guard g(p->device);
    const int64_t rows = nB * n_cells;
    // rows: ell (rows), ctx4 (4 rows), bth (nB), out (2 rows floats), scratch (2 nB)
    const size_t need = a256(sizeof(double) * rows) + a256(sizeof(double) * 4 * rows) +
                        a256(sizeof(double) * nB) + a256(sizeof(float) * 2 * rows) +
                        a256(sizeof(double) * 2 * nB);
    qrfs_status st = workspace(p, need);
    if (st) return st;
    std::vector<double> ell(rows), ctx(4 * rows);
    const double dl = p->Lw / n_cells;
    for (int64_t b = 0; b < nB; ++b)
        for (int j = 0; j < n_cells; ++j) {
            const int64_t r = b * n_cells + j;
            ell[r] = p->lmin + (j + 0.5) * dl;
            ctx[4 * r] = D;
            ctx[4 * r + 1] = L0;
            ctx[4 * r + 2] = blen[b];
            ctx[4 * r + 3] = bth[b];
        }
    char* base = (char*)p->ws;
    double* d_ell = (double*)base;
    double* d_ctx = (double*)(base + a256(sizeof(double) * rows));
    double* d_bth = (double*)((char*)d_ctx + a256(sizeof(double) * 4 * rows));
    float* d_out = (float*)((char*)d_bth + a256(sizeof(double) * nB));
    double* d_scr = (double*)((char*)d_out + a256(sizeof(float) * 2 * rows));
    hipStream_t strm = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_ell, ell.data(), sizeof(double) * rows, hipMemcpyHostToDevice, strm);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ctx, ctx.data(), sizeof(double) * 4 * rows, hipMemcpyHostToDevice, strm);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_bth, bth, sizeof(double) * nB, hipMemcpyHostToDevice, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    if (e != hipSuccess) return hfail(e, "table inputs");
    e = qrfs::prop_launch_forward(p->prm, rows, d_ell, d_ctx, p->lmin, p->Lw, d_out, strm);
    if (e == hipSuccess) {
        double* T = p->table;
        e = qrfs::prop_launch_table(d_out, nB, n_cells, d_bth, p->Lw, beta, T, T + qrfs::MAX_CELLS,
                                    T + 2 * qrfs::MAX_CELLS, T + 3 * qrfs::MAX_CELLS, d_scr, strm);
    }
    if (e != hipSuccess) return hfail(e, "table launch");
    p->n_cells = n_cells;
    return api_ok();
}

qrfs_status qrfs_proposal_get_table(const qrfs_proposal* p, int32_t* n_cells, double* tp,
                                    double* talpha, double* tphi, double* tcdf, void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    if (n_cells) *n_cells = p->n_cells;
    if (p->n_cells <= 0) return api_fail(QRFS_ERR_INVALID_ARG, "no table yet");
    Guard g(p->device);
    double* dst[4] = {tp, talpha, tphi, tcdf};
    for (int i = 0; i < 4; ++i) {
        if (!dst[i]) continue;
        hipError_t e = hipMemcpyAsync(dst[i], p->table + i * qrfs::MAX_CELLS,
                                      sizeof(double) * p->n_cells, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream);
        if (e != hipSuccess) return hfail(e, "table copy");
    }
    return api_ok();
}

qrfs_status qrfs_proposal_set_table(qrfs_proposal* p, int32_t n_cells, const double* tp,
                                    const double* talpha, const double* tphi, const double* tcdf,
                                    void* stream) {
    if (!p) return api_fail(QRFS_ERR_INVALID_ARG, "proposal is NULL");
    if (n_cells < 1 || n_cells > qrfs::MAX_CELLS)
        return api_fail(QRFS_ERR_INVALID_ARG, "n_cells must be in [1, %d]", qrfs::MAX_CELLS);
    if (!tp || !talpha || !tphi || !tcdf) return api_fail(QRFS_ERR_INVALID_ARG, "NULL table array");
    Guard g(p->device);
    const double* src[4] = {tp, talpha, tphi, tcdf};
    for (int i = 0; i < 4; ++i) {
        hipError_t e = hipMemcpyAsync(p->table + i * qrfs::MAX_CELLS, src[i],
                                      sizeof(double) * n_cells, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream);
        if (e != hipSuccess) return hfail(e, "table copy");
    }
    p->n_cells = n_cells;
    return api_ok();
}

qrfs_status qrfs_proposal_save(const qrfs_proposal* p, const char* path) {
    if (!p || !path) return api_fail(QRFS_ERR_INVALID_ARG, "proposal or path is NULL");
    Guard g(p->device);
    std::vector<float> h(qrfs::NPARAM);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), p->prm, sizeof(float) * qrfs::NPARAM, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hfail(e, "parameter download");
    FILE* f = fopen(path, "wb");
    if (!f) return api_fail(QRFS_ERR_INVALID_ARG, "cannot open %s for writing", path);
    bool ok = fwrite("QRFSPRP1", 1, 8, f) == 8 && fwrite(&p->fmin, 8, 1, f) == 1 &&
              fwrite(&p->fmax, 8, 1, f) == 1 &&
              fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? api_ok() : api_fail(QRFS_ERR_INVALID_ARG, "write to %s failed", path);
}

qrfs_status qrfs_proposal_load(qrfs_proposal* p, const char* path) {
    if (!p || !path) return api_fail(QRFS_ERR_INVALID_ARG, "proposal or path is NULL");
    FILE* f = fopen(path, "rb");
    if (!f) return api_fail(QRFS_ERR_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    double fmin = 0, fmax = 0;
    std::vector<float> h(qrfs::NPARAM);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "QRFSPRP1", 8) == 0 &&
              fread(&fmin, 8, 1, f) == 1 && fread(&fmax, 8, 1, f) == 1 &&
              fread(h.data(), sizeof(float), h.size(), f) == h.size();
    fclose(f);
    if (!ok) return api_fail(QRFS_ERR_INVALID_ARG, "%s is not a proposal file", path);
    if (fmin != p->fmin || fmax != p->fmax)
        return api_fail(QRFS_ERR_INVALID_ARG, "%s has a different frequency band", path);
    Guard g(p->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(p->prm, h.data(), sizeof(float) * qrfs::NPARAM, hipMemcpyHostToDevice);
    return e == hipSuccess ? api_ok() : hfail(e, "parameter upload");
}

}  // extern "C"
