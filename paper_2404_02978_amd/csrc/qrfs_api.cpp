// qrfs_api.cpp -- the C ABI of libqrfs: argument checks, the context and
// its device workspace, and the host-side orchestration of the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>

#include "qrfs.h"
#include "qrfs_internal.hpp"

namespace qrfs {
qrfs_status proposal_check_ready(const qrfs_proposal* p);
hipError_t proposal_sample(const qrfs_proposal* p, uint64_t s0x, uint64_t s0y, uint64_t index,
                           int64_t n_sets, int64_t K, double* fx, double* fy, double* area,
                           hipStream_t st);
}  // namespace qrfs

struct qrfs_context {
    int device = 0;
    void* ws = nullptr;
    size_t ws_size = 0;
    size_t ws_cap = 0;          // 0: unbounded
    int wide_path = 0;          // QRFS_TUNE_WIDE_PATH
    int64_t range_freqs = 2048;  // QRFS_TUNE_RANGE_FREQS
    size_t tile_cap = (size_t)2 << 30;  // QRFS_TUNE_TILE_BYTES
};

// Scratch of the allocation-free structure-function entry point: a static
// device array (each GPU the library runs on holds its own copy until the
// process ends), never allocated or freed by the library.  In host code
// `scratch` names a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

thread_local std::string g_detail;

qrfs_status fail(qrfs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_detail = buf;
    return s;
}

qrfs_status ok() {
    g_detail.clear();
    return QRFS_OK;
}

// Makes ctx->device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool okay = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        okay = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

qrfs_status hip_fail(hipError_t e, const char* what) {
    return fail(QRFS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

// Looks up the device address of `scratch` on `device` (which must be
// current) once per device.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipSuccess;  // entry point then refuses
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

qrfs_status sf_sets_enqueue(const qrfs::SfPlan& plan, char* base, int64_t K, const double* fx,
                            const double* fy, const double* w, int64_t nB, const double* bx,
                            const double* by, int64_t R, int64_t R_block, const qrfs_rng* rng,
                            int32_t precision, double* sf, double* sf_stderr, hipStream_t stream);

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

#define CHECK_PTR(p)                                                                 \
    do {                                                                             \
        if ((p) == nullptr) return fail(QRFS_ERR_INVALID_ARG, "%s is NULL", #p);     \
        if (!aligned8(p)) return fail(QRFS_ERR_INVALID_ARG, "%s is not 8-byte aligned", #p); \
    } while (0)

qrfs_status ensure_workspace(qrfs_context* ctx, size_t bytes) {
    if (bytes <= ctx->ws_size) return QRFS_OK;
    if (ctx->ws_cap && bytes > ctx->ws_cap)
        return fail(QRFS_ERR_OUT_OF_MEMORY, "workspace of %zu bytes exceeds the context cap of %zu",
                    bytes, ctx->ws_cap);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before workspace growth");
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_size = 0;
    size_t sz = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (ctx->ws_cap && sz > ctx->ws_cap) sz = bytes;
    e = hipMalloc(&ctx->ws, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(QRFS_ERR_OUT_OF_MEMORY, "workspace of %zu bytes: %s", sz, hipGetErrorString(e));
    }
    ctx->ws_size = sz;
    return QRFS_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

qrfs_status check_psd(const qrfs_psd* psd) {
    if (!psd) return fail(QRFS_ERR_INVALID_ARG, "psd is NULL");
    if (psd->model != QRFS_PSD_KOLMOGOROV && psd->model != QRFS_PSD_VON_KARMAN)
        return fail(QRFS_ERR_INVALID_ARG, "unknown PSD model %d", psd->model);
    if (!(psd->r0 > 0.0) || !std::isfinite(psd->r0))
        return fail(QRFS_ERR_INVALID_ARG, "r0 must be > 0 (got %g)", psd->r0);
    if (psd->model == QRFS_PSD_VON_KARMAN && (!(psd->L0 > 0.0) || !std::isfinite(psd->L0)))
        return fail(QRFS_ERR_INVALID_ARG, "von Karman L0 must be > 0 (got %g)", psd->L0);
    if (!std::isfinite(psd->c)) return fail(QRFS_ERR_INVALID_ARG, "PSD constant is not finite");
    if (!(psd->wavelength >= 0.0) || !std::isfinite(psd->wavelength))
        return fail(QRFS_ERR_INVALID_ARG, "wavelength must be >= 0 (got %g)", psd->wavelength);
    return QRFS_OK;
}

qrfs_status check_ap(const qrfs_aperture* ap) {
    if (!(ap->D > 0.0) || !std::isfinite(ap->D))
        return fail(QRFS_ERR_INVALID_ARG, "aperture D must be > 0 (got %g)", ap->D);
    if (!(ap->d >= 0.0) || !(ap->d < ap->D))
        return fail(QRFS_ERR_INVALID_ARG, "obstruction d must satisfy 0 <= d < D (got %g, D=%g)",
                    ap->d, ap->D);
    return QRFS_OK;
}

qrfs_status check_sampler(const qrfs_sampler* s, int64_t K) {
    if (!s) return fail(QRFS_ERR_INVALID_ARG, "sampler is NULL");
    const int sc = s->scheme;
    if (sc == QRFS_SAMPLER_LEARNED) return qrfs::proposal_check_ready(s->proposal);
    if (sc == QRFS_SAMPLER_R2_CARTESIAN || sc == QRFS_SAMPLER_RANDOM_CARTESIAN ||
        sc == QRFS_SAMPLER_JITTER) {
        if (s->N <= 0) return fail(QRFS_ERR_INVALID_ARG, "Cartesian N must be > 0 (got %d)", s->N);
        if (!(s->df > 0.0) || !std::isfinite(s->df))
            return fail(QRFS_ERR_INVALID_ARG, "Cartesian df must be > 0 (got %g)", s->df);
        if (sc == QRFS_SAMPLER_JITTER && K != (int64_t)s->N * s->N)
            return fail(QRFS_ERR_INVALID_ARG, "jittered grid needs K = N^2 (K=%lld, N=%d)",
                        (long long)K, s->N);
    } else if (sc == QRFS_SAMPLER_R2_LOGPOLAR || sc == QRFS_SAMPLER_RANDOM_LOGPOLAR) {
        if (!(s->fmin > 0.0) || !(s->fmax > s->fmin) || !std::isfinite(s->fmax))
            return fail(QRFS_ERR_INVALID_ARG, "log-polar band needs 0 < fmin < fmax (got %g, %g)",
                        s->fmin, s->fmax);
    } else if (sc == QRFS_SAMPLER_R2_DISC || sc == QRFS_SAMPLER_RANDOM_DISC) {
        if (!(s->fmax > 0.0) || !std::isfinite(s->fmax))
            return fail(QRFS_ERR_INVALID_ARG, "disc radius fmax must be > 0 (got %g)", s->fmax);
    } else {
        return fail(QRFS_ERR_INVALID_ARG, "unknown sampler scheme %d", sc);
    }
    return QRFS_OK;
}

qrfs_status check_sum_common(int64_t K, int64_t P, int64_t R, int64_t R_block,
                             const qrfs_rng* rng, const double* coef, int32_t precision) {
    if (K <= 0) return fail(QRFS_ERR_INVALID_ARG, "K must be > 0 (got %lld)", (long long)K);
    if (P <= 0) return fail(QRFS_ERR_INVALID_ARG, "number of points must be > 0 (got %lld)", (long long)P);
    if (R <= 0) return fail(QRFS_ERR_INVALID_ARG, "R must be > 0 (got %lld)", (long long)R);
    if (R_block < 1 || R_block > R)
        return fail(QRFS_ERR_INVALID_ARG, "R_block must be in [1, R] (got %lld, R=%lld)",
                    (long long)R_block, (long long)R);
    if (K > ((int64_t)1 << 33))
        return fail(QRFS_ERR_INVALID_ARG, "K too large for the 32-bit Philox block counter");
    if (precision != QRFS_PREC_FP64 && precision != QRFS_PREC_FP32 &&
        precision != QRFS_PREC_SPLIT_BF16 && precision != QRFS_PREC_BF16X6 &&
        precision != QRFS_PREC_FP16X3)
        return fail(QRFS_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (!coef) {
        if (!rng) return fail(QRFS_ERR_INVALID_ARG, "rng is NULL and no coefficients were given");
        if (rng->mode != QRFS_COEF_GAUSS_CS && rng->mode != QRFS_COEF_EQ3)
            return fail(QRFS_ERR_INVALID_ARG, "unknown coefficient mode %d", rng->mode);
    } else if (!aligned8(coef)) {
        return fail(QRFS_ERR_INVALID_ARG, "coef is not 8-byte aligned");
    }
    return QRFS_OK;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// R2 sampling with any scheme: sets [0, n_sets) starting at `index`
hipError_t sample_any(const qrfs_sampler* s, uint64_t index, int64_t n_sets, int64_t K,
                      double* fx, double* fy, double* area, hipStream_t st) {
    if (s->scheme == QRFS_SAMPLER_LEARNED)
        return qrfs::proposal_sample(s->proposal, s->seed_x, s->seed_y, index, n_sets, K, fx, fy,
                                     area, st);
    return qrfs::launch_sample(s->scheme, s->seed_x, s->seed_y, index, n_sets, K, s->N, s->df,
                               s->fmin, s->fmax, fx, fy, area, st);
}

// Frequencies and weights of n_sets sets for a pipeline that needs no cell
// areas: one fused kernel for the R2, pseudo-random and jittered samplers;
// the learned sampler writes its areas to `area` and the weights follow.
// f32: weights for FP32-class sums (qrfs_weights' precision argument).
hipError_t sample_weights_any(const qrfs_sampler* s, uint64_t index, int64_t n_sets, int64_t K,
                              const qrfs_psd* psd, double c, const qrfs_aperture* ap, int f32,
                              double* fx, double* fy, double* area, double* w, hipStream_t st) {
    const int has_ap = ap ? 1 : 0;
    const double D = ap ? ap->D : 0.0, d = ap ? ap->d : 0.0;
    if (s->scheme == QRFS_SAMPLER_LEARNED) {
        hipError_t e = sample_any(s, index, n_sets, K, fx, fy, area, st);
        if (e != hipSuccess) return e;
        return qrfs::launch_weights(psd->model, c, psd->r0, psd->L0, has_ap, D, d, f32,
                                    n_sets * K, fx, fy, area, w, st);
    }
    return qrfs::launch_sample_weights(s->scheme, s->seed_x, s->seed_y, index, n_sets, K, s->N,
                                       s->df, s->fmin, s->fmax, psd->model, c, psd->r0, psd->L0,
                                       has_ap, D, d, f32, fx, fy, w, st);
}

// Largest grid of one launch: the work-items of a dispatch (blocks x
// threads, at most 1024 threads per block here) must fit in 32 bits.
constexpr int64_t kMaxLaunchBlocks = (int64_t)1 << 22;

// Runs launch_sum over all sets, splitting the grid so no launch exceeds
// kMaxLaunchBlocks blocks.
qrfs_status run_sum(int precision, int basis, int epi, qrfs::SumArgs a, int64_t n_sets,
                    hipStream_t st) {
    int64_t rts = qrfs::sum_row_tiles_per_set(precision, basis, a.R_block, a.P);
    int64_t cts = qrfs::sum_col_tiles(precision, basis, a.R_block, a.P);
    int64_t per_set = rts * cts * (a.ksplit > 1 ? a.ksplit : 1);
    int64_t max_sets = kMaxLaunchBlocks / (per_set > 0 ? per_set : 1);
    if (max_sets < 1) return fail(QRFS_ERR_INVALID_ARG, "problem too large for one set");
    const double* fx0 = a.fx;
    const double* fy0 = a.fy;
    const double* w0 = a.w;
    double* part0 = a.partial;
    for (int64_t s0 = 0; s0 < n_sets; s0 += max_sets) {
        int64_t s1 = s0 + max_sets < n_sets ? s0 + max_sets : n_sets;
        a.set0 = s0;
        a.set1 = s1;
        a.fx = fx0 + s0 * a.K;
        a.fy = fy0 + s0 * a.K;
        a.w = w0 + s0 * a.K;
        if (part0) a.partial = part0 + s0 * rts * a.P * 2;
        hipError_t e = qrfs::launch_sum(precision, basis, epi, a, st);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return QRFS_OK;
}

// Whether the two-phase kernel contracts this problem: MFMA precisions,
// outputs wide enough to amortise the coefficient tiles, and enough
// 256 x 256 tiles to fill the chip (or forced by the context).
bool use_wide(const qrfs_context* ctx, int precision, int64_t P, int64_t R, int64_t R_block,
              bool caller_coef) {
    if (precision == QRFS_PREC_FP64 || ctx->wide_path == 1) return false;
    // FP16X3 scales the coefficient tiles by the largest value the generators
    // can draw; caller-given coefficients contract in the fused kernel
    if (precision == QRFS_PREC_FP16X3 && caller_coef) return false;
    if (P > ((int64_t)1 << 22)) return false;  // 256 rows of output within 32-bit tile offsets
    if (ctx->wide_path == 2) return true;
    const int64_t tiles = cdiv(R, R_block) * cdiv(R_block, 256) * cdiv(P, 256);
    return P >= 1024 && R_block >= 128 && tiles >= 512;
}

// Two-phase contraction (EPI_STORE) over all sets: per piece, the
// coefficient tiles, then one contraction launch (FP32-class precisions sum
// ranges of ctx->range_freqs frequencies in FP32 and add each into the
// output; split-BF16 uses a single range).
qrfs_status wide_sum(qrfs_context* ctx, int precision, int basis, qrfs::SumArgs a,
                     int64_t n_sets, hipStream_t st) {
    const int KCH = qrfs::wide_chunk(precision);
    const int64_t nch = cdiv(a.K, KCH);
    const int64_t nkv = nch * 2 * KCH;
    const size_t row32 = qrfs::wide_frag_bytes_per_row32(precision, nkv);
    const int64_t cts = cdiv(a.P, 256);
    const int64_t rts_set = cdiv(a.R_block, 256);
    // coefficient tiles take at most ctx->tile_cap of workspace per piece
    // (one 256-row block of one set at least); behind them the store sink
    // (256 B) and, for FP16X3, one scale per set
    const size_t scale_bytes =
        precision == QRFS_PREC_FP16X3 ? align256((size_t)n_sets * sizeof(double)) : 0;
    size_t cap = ctx->tile_cap;
    const size_t extra = 512 + scale_bytes;
    if (ctx->ws_cap && ctx->ws_cap < cap + extra) cap = ctx->ws_cap > extra ? ctx->ws_cap - extra : 0;
    const size_t set_bytes = (size_t)rts_set * 8 * row32;
    int64_t sets_piece = 1, rows_piece = a.R_block;
    if (set_bytes <= cap) {
        sets_piece = (int64_t)(cap / set_bytes);
        const int64_t max_blocks = kMaxLaunchBlocks;
        if (sets_piece * rts_set * cts > max_blocks) sets_piece = max_blocks / (rts_set * cts);
        if (sets_piece < 1) return fail(QRFS_ERR_INVALID_ARG, "problem too large for one set");
        if (sets_piece > n_sets) sets_piece = n_sets;
    } else {
        int64_t tiles = (int64_t)(cap / (8 * row32));
        rows_piece = (tiles < 1 ? 1 : tiles) * 256;
    }
    const size_t tile_bytes = align256((size_t)sets_piece * cdiv(rows_piece, 256) * 8 * row32);
    qrfs_status s = ensure_workspace(ctx, tile_bytes + 256 + scale_bytes);
    if (s) return s;
    double* ascale = (double*)((char*)ctx->ws + tile_bytes + 256);
    if (precision == QRFS_PREC_FP16X3) {
        hipError_t e = qrfs::launch_wide_scale(a.w, a.K, n_sets, ascale, st);
        if (e != hipSuccess) return hip_fail(e, "tile scale launch");
    }
    // accumulation ranges: whole K for split-BF16, else about
    // ctx->range_freqs frequencies (an even number of chunks)
    int64_t rch = precision == QRFS_PREC_SPLIT_BF16 ? nch : cdiv(ctx->range_freqs, KCH);
    rch += rch & 1;
    const double* fx0 = a.fx;
    const double* fy0 = a.fy;
    const double* w0 = a.w;
    qrfs::WideArgs wa{};
    wa.nkv = nkv;
    wa.cts = cts;
    wa.ctile = ctx->ws;
    wa.sink = (float*)((char*)ctx->ws + tile_bytes);
    for (int64_t s0 = 0; s0 < n_sets; s0 += sets_piece) {
        const int64_t s1 = s0 + sets_piece < n_sets ? s0 + sets_piece : n_sets;
        for (int64_t off = 0; off < a.R_block; off += rows_piece) {
            // the last set may end before this row range
            if (s1 - s0 == 1 && s0 * a.R_block + off >= a.R) break;
            wa.s = a;
            wa.s.set0 = s0;
            wa.s.set1 = s1;
            wa.s.fx = fx0 + s0 * a.K;
            wa.s.fy = fy0 + s0 * a.K;
            wa.s.w = w0 + s0 * a.K;
            wa.ascale = ascale + s0;
            wa.row_off = off;
            wa.rows = off + rows_piece < a.R_block ? rows_piece : a.R_block - off;
            wa.rts = cdiv(wa.rows, 256);
            wa.rt32 = wa.rts * 8;
            hipError_t e = qrfs::launch_wide_coef(precision, wa, st);
            if (e != hipSuccess) return hip_fail(e, "coefficient tile launch");
            wa.ch0 = 0;
            wa.ch1 = nch;
            wa.range_ch = rch;
            wa.accumulate = 0;
            e = qrfs::launch_wide_sum(precision, basis, wa, st);
            if (e != hipSuccess) return hip_fail(e, "two-phase contraction launch");
        }
    }
    return QRFS_OK;
}

qrfs_status sum_entry(qrfs_context* ctx, int basis, int64_t K, const double* fx,
                      const double* fy, const double* w, int64_t P, const double* px,
                      const double* py, const double* apD, const double* apd, int64_t R,
                      int64_t R_block, const qrfs_rng* rng, const double* coef,
                      int32_t precision, void* out, void* stream,
                      const double* grad_u = nullptr) {
    qrfs_status s = check_sum_common(K, P, R, R_block, rng, coef, precision);
    if (s) return s;
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(w);
    CHECK_PTR(px);
    CHECK_PTR(py);
    if (basis == qrfs::BASIS_PISTON) {
        CHECK_PTR(apD);
        CHECK_PTR(apd);
    }
    if (!out) return fail(QRFS_ERR_INVALID_ARG, "output is NULL");
    if (((uintptr_t)out & (precision == QRFS_PREC_FP64 ? 7u : 3u)) != 0)
        return fail(QRFS_ERR_INVALID_ARG, "output is misaligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    qrfs::SumArgs a{};
    a.K = K;
    a.fx = fx;
    a.fy = fy;
    a.w = w;
    a.P = P;
    a.px = px;
    a.py = py;
    a.apD = apD;
    a.apd = apd;
    a.R = R;
    a.R_block = R_block;
    a.seed = rng ? rng->seed : 0;
    a.counter = rng ? rng->counter : 0;
    a.mode = rng ? rng->mode : 0;
    a.coef = coef;
    a.out = out;
    a.partial = nullptr;
    a.ksplit = 1;
    a.kspan = K;
    a.phi_part = nullptr;
    if (grad_u) {
        a.grad = 1;
        a.gx = 2.0 * M_PI * grad_u[0];
        a.gy = 2.0 * M_PI * grad_u[1];
    }
    if (use_wide(ctx, precision, P, R, R_block, coef != nullptr))
        s = wide_sum(ctx, precision, basis, a, cdiv(R, R_block), (hipStream_t)stream);
    else
        s = run_sum(precision, basis, qrfs::EPI_STORE, a, cdiv(R, R_block), (hipStream_t)stream);
    if (s) return s;
    return ok();
}

}  // namespace

namespace qrfs {
// shared with the batch layer
qrfs_status api_fail(qrfs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_detail = buf;
    return s;
}
qrfs_status api_ok() { return ok(); }
int64_t api_context_range_freqs(const qrfs_context* ctx) { return ctx->range_freqs; }
int api_context_device(const qrfs_context* ctx) { return ctx->device; }
}  // namespace qrfs

extern "C" {

const char* qrfs_error_string(qrfs_status s) {
    switch (s) {
        case QRFS_OK: return "success";
        case QRFS_ERR_INVALID_ARG: return "invalid argument";
        case QRFS_ERR_OUT_OF_MEMORY: return "out of device memory";
        case QRFS_ERR_DEVICE: return "device (HIP runtime) error";
        case QRFS_ERR_UNSUPPORTED: return "unsupported";
        case QRFS_ERR_NOT_CONVERGED: return "not converged";
        default: return "unknown status";
    }
}

const char* qrfs_last_error_detail(void) { return g_detail.c_str(); }

int32_t qrfs_abi_version(void) { return QRFS_ABI_VERSION; }

qrfs_status qrfs_context_create(qrfs_context** out, int32_t device, size_t workspace_cap_bytes) {
    if (!out) return fail(QRFS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(QRFS_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, n);
    {
        DeviceGuard g(device);
        if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", device);
        e = scratch_setup(device);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
    }
    qrfs_context* c = new (std::nothrow) qrfs_context();
    if (!c) return fail(QRFS_ERR_OUT_OF_MEMORY, "host allocation of the context");
    c->device = device;
    c->ws_cap = workspace_cap_bytes;
    *out = c;
    return ok();
}

qrfs_status qrfs_context_set_tuning(qrfs_context* ctx, int32_t key, int64_t value) {
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    if (key == QRFS_TUNE_WIDE_PATH) {
        if (value < 0 || value > 2)
            return fail(QRFS_ERR_INVALID_ARG, "wide path must be 0, 1 or 2 (got %lld)", (long long)value);
        ctx->wide_path = (int)value;
    } else if (key == QRFS_TUNE_RANGE_FREQS) {
        if (value < 0 || value > ((int64_t)1 << 33))
            return fail(QRFS_ERR_INVALID_ARG, "range of %lld frequencies", (long long)value);
        ctx->range_freqs = value == 0 ? 2048 : value;
    } else if (key == QRFS_TUNE_TILE_BYTES) {
        if (value < 0) return fail(QRFS_ERR_INVALID_ARG, "tile cap of %lld bytes", (long long)value);
        ctx->tile_cap = value == 0 ? ((size_t)2 << 30) : (size_t)value;
    } else {
        return fail(QRFS_ERR_INVALID_ARG, "unknown tuning key %d", key);
    }
    return ok();
}

qrfs_status qrfs_context_destroy(qrfs_context* ctx) {
    if (!ctx) return ok();
    qrfs_status st = QRFS_OK;
    {
        DeviceGuard g(ctx->device);
        if (ctx->ws) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize in destroy");
            (void)hipFree(ctx->ws);
        }
    }
    delete ctx;
    return st ? st : ok();
}

qrfs_status qrfs_sample_frequencies(qrfs_context* ctx, qrfs_sampler* s, int64_t n_sets,
                                    int64_t K, double* fx, double* fy, double* area,
                                    void* stream) {
    qrfs_status st = check_sampler(s, K);
    if (st) return st;
    if (K <= 0 || n_sets <= 0)
        return fail(QRFS_ERR_INVALID_ARG, "K and n_sets must be > 0 (got %lld, %lld)",
                    (long long)K, (long long)n_sets);
    if (n_sets > INT64_MAX / K || n_sets * K > QRFS_MAX_POINTS_PER_CALL)
        return fail(QRFS_ERR_INVALID_ARG, "n_sets * K = %lld exceeds %lld points per call",
                    (long long)(n_sets > INT64_MAX / K ? INT64_MAX : n_sets * K),
                    (long long)QRFS_MAX_POINTS_PER_CALL);
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(area);
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    hipError_t e = sample_any(s, s->index, n_sets, K, fx, fy, area, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sampler launch");
    s->index += (uint64_t)(n_sets * K);
    return ok();
}

// The precision argument of the weight entry points: any known precision,
// FP64 for binary64 weights, the others for weights that feed FP32-class sums.
static qrfs_status check_weight_precision(int32_t precision) {
    if (precision < QRFS_PREC_FP64 || precision > QRFS_PREC_FP16X3)
        return fail(QRFS_ERR_INVALID_ARG, "unknown precision %d", precision);
    return QRFS_OK;
}

qrfs_status qrfs_weights(qrfs_context* ctx, const qrfs_psd* psd, const qrfs_aperture* ap,
                         int64_t n, const double* fx, const double* fy, const double* area,
                         int32_t precision, double* w, void* stream) {
    qrfs_status st = check_psd(psd);
    if (st) return st;
    if (ap && (st = check_ap(ap))) return st;
    if ((st = check_weight_precision(precision))) return st;
    if (n <= 0 || n > QRFS_MAX_POINTS_PER_CALL)
        return fail(QRFS_ERR_INVALID_ARG, "n must be in 1..%lld (got %lld)",
                    (long long)QRFS_MAX_POINTS_PER_CALL, (long long)n);
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(area);
    CHECK_PTR(w);
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    const double c = qrfs::psd_constant(psd->c, psd->wavelength);
    hipError_t e = qrfs::launch_weights(psd->model, c, psd->r0, psd->L0, ap ? 1 : 0,
                                        ap ? ap->D : 0.0, ap ? ap->d : 0.0,
                                        precision != QRFS_PREC_FP64, n, fx, fy, area, w,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "weights launch");
    return ok();
}

qrfs_status qrfs_sample_weights(qrfs_context* ctx, qrfs_sampler* s, int64_t n_sets, int64_t K,
                                const qrfs_psd* psd, const qrfs_aperture* ap, int32_t precision,
                                double* fx, double* fy, double* w, void* stream) {
    qrfs_status st = check_sampler(s, K);
    if (st) return st;
    if ((st = check_psd(psd))) return st;
    if (ap && (st = check_ap(ap))) return st;
    if ((st = check_weight_precision(precision))) return st;
    if (K <= 0 || n_sets <= 0)
        return fail(QRFS_ERR_INVALID_ARG, "K and n_sets must be > 0 (got %lld, %lld)",
                    (long long)K, (long long)n_sets);
    if (n_sets > INT64_MAX / K || n_sets * K > QRFS_MAX_POINTS_PER_CALL)
        return fail(QRFS_ERR_INVALID_ARG, "n_sets * K = %lld exceeds %lld points per call",
                    (long long)(n_sets > INT64_MAX / K ? INT64_MAX : n_sets * K),
                    (long long)QRFS_MAX_POINTS_PER_CALL);
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(w);
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    double* area = nullptr;
    if (s->scheme == QRFS_SAMPLER_LEARNED) {  // its cell areas go through the workspace
        if ((st = ensure_workspace(ctx, (size_t)(n_sets * K) * sizeof(double)))) return st;
        area = (double*)ctx->ws;
    }
    const double c = qrfs::psd_constant(psd->c, psd->wavelength);
    hipError_t e =
        sample_weights_any(s, s->index, n_sets, K, psd, c, ap, precision != QRFS_PREC_FP64, fx,
                           fy, area, w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sampler / weights launch");
    s->index += (uint64_t)(n_sets * K);
    return ok();
}

qrfs_status qrfs_synthesize_phase(qrfs_context* ctx, int64_t K, const double* fx,
                                  const double* fy, const double* w, int64_t P,
                                  const double* px, const double* py, int64_t R,
                                  int64_t R_block, const qrfs_rng* rng, const double* coef,
                                  int32_t precision, void* phase, void* stream) {
    return sum_entry(ctx, qrfs::BASIS_PHASE, K, fx, fy, w, P, px, py, nullptr, nullptr, R,
                     R_block, rng, coef, precision, phase, stream);
}

qrfs_status qrfs_piston(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                        const double* w, int64_t n_ap, const double* cx, const double* cy,
                        const double* apD, const double* apd, int64_t R, int64_t R_block,
                        const qrfs_rng* rng, const double* coef, int32_t precision,
                        void* piston, void* stream) {
    return sum_entry(ctx, qrfs::BASIS_PISTON, K, fx, fy, w, n_ap, cx, cy, apD, apd, R, R_block,
                     rng, coef, precision, piston, stream);
}

qrfs_status qrfs_tilt(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                      const double* w, int64_t n_ap, const double* cx, const double* cy,
                      const double* apD, const double* apd, double ux, double uy, int64_t R,
                      int64_t R_block, const qrfs_rng* rng, const double* coef,
                      int32_t precision, void* tilt, void* stream) {
    if (!std::isfinite(ux) || !std::isfinite(uy) || (ux == 0.0 && uy == 0.0))
        return fail(QRFS_ERR_INVALID_ARG, "direction (%g, %g) is zero or not finite", ux, uy);
    const double u[2] = {ux, uy};
    return sum_entry(ctx, qrfs::BASIS_PISTON, K, fx, fy, w, n_ap, cx, cy, apD, apd, R, R_block,
                     rng, coef, precision, tilt, stream, u);
}

qrfs_status qrfs_diff_piston(qrfs_context* ctx, int64_t K, const double* fx, const double* fy,
                             const double* w, int64_t nB, const double* bx, const double* by,
                             int64_t R, int64_t R_block, const qrfs_rng* rng, const double* coef,
                             int32_t precision, void* dp, void* stream) {
    return sum_entry(ctx, qrfs::BASIS_DIFF, K, fx, fy, w, nB, bx, by, nullptr, nullptr, R,
                     R_block, rng, coef, precision, dp, stream);
}

qrfs_status qrfs_diff_piston_structure(qrfs_context* ctx, const qrfs_psd* psd,
                                       const qrfs_aperture* ap, int64_t nB, const double* bx,
                                       const double* by, qrfs_sampler* s, int64_t K, int64_t R,
                                       int64_t R_block, const qrfs_rng* rng, int32_t precision,
                                       double* sf, double* sf_stderr, void* stream) {
    qrfs_status st = check_psd(psd);
    if (st) return st;
    if (!ap) return fail(QRFS_ERR_INVALID_ARG, "aperture is required");
    if ((st = check_ap(ap))) return st;
    if ((st = check_sampler(s, K))) return st;
    if ((st = check_sum_common(K, nB, R, R_block, rng, nullptr, precision))) return st;
    CHECK_PTR(bx);
    CHECK_PTR(by);
    CHECK_PTR(sf);
    if (sf_stderr && !aligned8(sf_stderr))
        return fail(QRFS_ERR_INVALID_ARG, "sf_stderr is not 8-byte aligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);

    const int64_t n_sets = cdiv(R, R_block);
    const int64_t rts = qrfs::sum_row_tiles_per_set(precision, qrfs::BASIS_DIFF, R_block, nB);
    const qrfs::SfPlan plan = qrfs::sf_plan(precision, K, R, R_block, nB);
    const size_t partial_bytes = align256((size_t)(plan.n_partial_tiles * nB) * 2 * sizeof(double));
    const size_t phi_bytes = align256(plan.phi_floats * sizeof(float));
    const size_t per_set = (size_t)K * 4 * sizeof(double);
    const size_t budget = (size_t)1 << 30;
    int64_t spb = (int64_t)(budget / per_set);
    if (spb < 1) spb = 1;
    if (spb > n_sets) spb = n_sets;
    const size_t arr = align256((size_t)spb * K * sizeof(double));
    if ((st = ensure_workspace(ctx, partial_bytes + phi_bytes + 4 * arr))) return st;
    char* base = (char*)ctx->ws;
    double* partial = (double*)base;
    float* phi = (float*)(base + partial_bytes);
    char* fbase = base + partial_bytes + phi_bytes;
    double* fx = (double*)(fbase);
    double* fy = (double*)(fbase + arr);
    double* area = (double*)(fbase + 2 * arr);
    double* w = (double*)(fbase + 3 * arr);
    hipStream_t stream_ = (hipStream_t)stream;
    const double c = qrfs::psd_constant(psd->c, psd->wavelength);

    for (int64_t s0 = 0; s0 < n_sets; s0 += spb) {
        int64_t s1 = s0 + spb < n_sets ? s0 + spb : n_sets;
        int64_t ns = s1 - s0;
        hipError_t e = sample_weights_any(s, s->index + (uint64_t)(s0 * K), ns, K, psd, c, ap, 0,
                                          fx, fy, area, w, stream_);
        if (e != hipSuccess) return hip_fail(e, "sampler / weights launch");
        qrfs::SumArgs a{};
        a.K = K;
        a.fx = fx;
        a.fy = fy;
        a.w = w;
        a.P = nB;
        a.px = bx;
        a.py = by;
        a.R = R;
        a.R_block = R_block;
        a.seed = rng->seed;
        a.counter = rng->counter;
        a.mode = rng->mode;
        a.coef = nullptr;
        a.out = nullptr;
        a.ksplit = plan.ksplit;
        a.kspan = plan.kspan;
        a.phi_part = phi;
        // absolute set bounds; the batch buffers hold exactly these sets
        a.set0 = s0;
        a.set1 = s1;
        a.partial = partial + s0 * rts * nB * 2;
        e = qrfs::launch_sum(precision, qrfs::BASIS_DIFF, qrfs::EPI_SFSUM, a, stream_);
        if (e != hipSuccess) return hip_fail(e, "structure-function launch");
    }
    if (plan.ksplit > 1) {
        hipError_t e = qrfs::launch_sfsum_rows(phi, plan.ksplit, R, nB, partial, stream_);
        if (e != hipSuccess) return hip_fail(e, "split-K square launch");
    }
    hipError_t e = qrfs::launch_reduce_sf(partial, plan.n_partial_tiles, nB, R, sf, sf_stderr,
                                          stream_);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    s->index += (uint64_t)(n_sets * K);
    return ok();
}

qrfs_status qrfs_point_set_measures(qrfs_context* ctx, int64_t n_sets, int64_t K,
                                    const double* fx, const double* fy, double x0, double y0,
                                    double Lx, double Ly, double r_clash, double* min_dist,
                                    int64_t* n_clash, double* l2_star, void* stream) {
    if (n_sets < 1 || K < 1)
        return fail(QRFS_ERR_INVALID_ARG, "n_sets and K must be >= 1 (got %lld, %lld)",
                    (long long)n_sets, (long long)K);
    if (K > ((int64_t)1 << 24))
        return fail(QRFS_ERR_INVALID_ARG, "K must be <= 2^24 (got %lld)", (long long)K);
    // one block of 256 threads per (set, 256-point tile): at most 2^24
    // blocks keep the launch within 2^32 work-items
    if (n_sets * qrfs::measure_tiles(K) >= ((int64_t)1 << 24))
        return fail(QRFS_ERR_INVALID_ARG, "n_sets * ceil(K/256) must be < 2^24");
    if (!(Lx > 0.0) || !(Ly > 0.0) || !std::isfinite(Lx) || !std::isfinite(Ly) ||
        !std::isfinite(x0) || !std::isfinite(y0))
        return fail(QRFS_ERR_INVALID_ARG, "the unit-square map needs finite x0, y0 and Lx, Ly > 0");
    if (!(r_clash >= 0.0) || !std::isfinite(r_clash))
        return fail(QRFS_ERR_INVALID_ARG, "r_clash must be finite and >= 0 (got %g)", r_clash);
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(min_dist);
    CHECK_PTR(n_clash);
    CHECK_PTR(l2_star);
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    const size_t part_bytes = align256((size_t)(n_sets * qrfs::measure_tiles(K)) * 4 * sizeof(double));
    qrfs_status st = ensure_workspace(ctx, part_bytes);
    if (st) return st;
    hipError_t e = qrfs::launch_point_set_measures(n_sets, K, fx, fy, x0, y0, Lx, Ly, r_clash,
                                                   (double*)ctx->ws, min_dist, n_clash, l2_star,
                                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "point-set measure launch");
    return ok();
}

qrfs_status qrfs_set_sf_expectation(qrfs_context* ctx, int64_t K, const double* fx,
                                    const double* fy, const double* w, int64_t n_sets, int64_t nB,
                                    const double* bx, const double* by, double* S, void* stream) {
    if (K < 1 || n_sets < 1 || nB < 1)
        return fail(QRFS_ERR_INVALID_ARG, "K, n_sets and nB must be >= 1");
    if (n_sets >= ((int64_t)1 << 24))  // one 256-thread block per set
        return fail(QRFS_ERR_INVALID_ARG, "n_sets must be < 2^24");
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(w);
    CHECK_PTR(bx);
    CHECK_PTR(by);
    CHECK_PTR(S);
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    hipError_t e = qrfs::launch_set_sf(n_sets, K, fx, fy, w, nB, bx, by, S, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "per-set structure function launch");
    return ok();
}

qrfs_status qrfs_temporal_sf(qrfs_context* ctx, int64_t R, int64_t M, int32_t precision,
                             const void* pistons, double* sf, double* sf_stderr, void* stream) {
    if (R < 1) return fail(QRFS_ERR_INVALID_ARG, "R must be >= 1 (got %lld)", (long long)R);
    if (M < 1 || M > qrfs::TEMPORAL_MAX_M)
        return fail(QRFS_ERR_INVALID_ARG, "M must be in [1, %d] (got %lld)", qrfs::TEMPORAL_MAX_M,
                    (long long)M);
    if (precision != QRFS_PREC_FP64 && precision != QRFS_PREC_FP32 &&
        precision != QRFS_PREC_SPLIT_BF16 && precision != QRFS_PREC_BF16X6 &&
        precision != QRFS_PREC_FP16X3)
        return fail(QRFS_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (!pistons) return fail(QRFS_ERR_INVALID_ARG, "pistons is NULL");
    if (((uintptr_t)pistons & (precision == QRFS_PREC_FP64 ? 7u : 3u)) != 0)
        return fail(QRFS_ERR_INVALID_ARG, "pistons is misaligned");
    CHECK_PTR(sf);
    if (sf_stderr && !aligned8(sf_stderr))
        return fail(QRFS_ERR_INVALID_ARG, "sf_stderr is not 8-byte aligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    const int64_t nb = qrfs::temporal_blocks(R);
    qrfs_status st = ensure_workspace(ctx, align256((size_t)nb * M * 2 * sizeof(double)));
    if (st) return st;
    double* part = (double*)ctx->ws;
    hipStream_t stream_ = (hipStream_t)stream;
    hipError_t e = qrfs::launch_temporal_rows(precision == QRFS_PREC_FP64, pistons, R, M, part,
                                              stream_);
    if (e != hipSuccess) return hip_fail(e, "temporal estimator launch");
    e = qrfs::launch_reduce_sf(part, nb, M, R, sf, sf_stderr, stream_);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    return ok();
}

qrfs_status qrfs_temporal_piston_structure(qrfs_context* ctx, const qrfs_psd* psd,
                                           const qrfs_aperture* ap, const double* c1,
                                           const double* c2, const double* v, double dt,
                                           int64_t M, qrfs_sampler* s, int64_t K, int64_t R,
                                           int64_t R_block, const qrfs_rng* rng,
                                           int32_t precision, double* sf, double* sf_stderr,
                                           void* stream) {
    qrfs_status st = check_psd(psd);
    if (st) return st;
    if (!ap) return fail(QRFS_ERR_INVALID_ARG, "aperture is required");
    if ((st = check_ap(ap))) return st;
    if ((st = check_sampler(s, K))) return st;
    if (M < 1 || M > qrfs::TEMPORAL_MAX_M)
        return fail(QRFS_ERR_INVALID_ARG, "M must be in [1, %d] (got %lld)", qrfs::TEMPORAL_MAX_M,
                    (long long)M);
    if ((st = check_sum_common(K, 2 * M, R, R_block, rng, nullptr, precision))) return st;
    if (!c1 || !c2 || !v) return fail(QRFS_ERR_INVALID_ARG, "c1, c2 and v are required");
    if (!(dt >= 0.0) || !std::isfinite(dt))
        return fail(QRFS_ERR_INVALID_ARG, "dt must be finite and >= 0");
    for (int i = 0; i < 2; ++i)
        if (!std::isfinite(c1[i]) || !std::isfinite(c2[i]) || !std::isfinite(v[i]))
            return fail(QRFS_ERR_INVALID_ARG, "c1, c2, v must be finite");
    CHECK_PTR(sf);
    if (sf_stderr && !aligned8(sf_stderr))
        return fail(QRFS_ERR_INVALID_ARG, "sf_stderr is not 8-byte aligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);

    const int64_t n_sets = cdiv(R, R_block);
    const int64_t P = 2 * M;
    const bool fp64 = precision == QRFS_PREC_FP64;
    const size_t esize = fp64 ? sizeof(double) : sizeof(float);
    // pieces of whole sets (at most ~1 GiB of frequencies and pistons) whose
    // first realisation is a multiple of the estimator's row blocks, so the
    // fixed-order reduction sees the same blocks however the sets are cut
    const int64_t q = qrfs::TEMPORAL_ROWS_PER_BLOCK / std::gcd(R_block,
                                                              (int64_t)qrfs::TEMPORAL_ROWS_PER_BLOCK);
    const size_t per_set = (size_t)K * 4 * sizeof(double) + (size_t)R_block * P * esize;
    int64_t spb = (int64_t)(((size_t)1 << 30) / per_set);
    spb = spb / q * q;
    if (spb < q) spb = q;
    if (spb > n_sets) spb = n_sets;
    const int64_t nb = qrfs::temporal_blocks(R);
    const size_t part_bytes = align256((size_t)nb * M * 2 * sizeof(double));
    const size_t pt_bytes = align256((size_t)P * sizeof(double));
    const size_t arr = align256((size_t)spb * K * sizeof(double));
    const size_t pist_bytes = align256((size_t)spb * R_block * P * esize);
    if ((st = ensure_workspace(ctx, part_bytes + 2 * pt_bytes + 4 * arr + pist_bytes))) return st;
    char* base = (char*)ctx->ws;
    double* part = (double*)base;
    double* px = (double*)(base + part_bytes);
    double* py = (double*)(base + part_bytes + pt_bytes);
    char* fbase = base + part_bytes + 2 * pt_bytes;
    double* fx = (double*)fbase;
    double* fy = (double*)(fbase + arr);
    double* area = (double*)(fbase + 2 * arr);
    double* w = (double*)(fbase + 3 * arr);
    void* pist = fbase + 4 * arr;
    hipStream_t stream_ = (hipStream_t)stream;
    const double c = qrfs::psd_constant(psd->c, psd->wavelength);

    hipError_t e = qrfs::launch_taylor_points(c1, c2, v, dt, M, px, py, stream_);
    if (e != hipSuccess) return hip_fail(e, "point launch");
    for (int64_t s0 = 0; s0 < n_sets; s0 += spb) {
        const int64_t s1 = s0 + spb < n_sets ? s0 + spb : n_sets;
        const int64_t ns = s1 - s0;
        const int64_t r0 = s0 * R_block;
        const int64_t rows = (s1 * R_block < R ? s1 * R_block : R) - r0;
        // equal apertures: the filter of Eq. 7 folds into the weight
        e = sample_weights_any(s, s->index + (uint64_t)(s0 * K), ns, K, psd, c, ap, 0, fx, fy,
                               area, w, stream_);
        if (e != hipSuccess) return hip_fail(e, "sampler / weights launch");
        // the piece as a problem of its own: realisations r0 .. r0 + rows
        qrfs::SumArgs a{};
        a.K = K;
        a.fx = fx;
        a.fy = fy;
        a.w = w;
        a.P = P;
        a.px = px;
        a.py = py;
        a.R = rows;
        a.R_block = R_block;
        a.seed = rng->seed;
        a.counter = rng->counter + (uint64_t)r0;
        a.mode = rng->mode;
        a.coef = nullptr;
        a.out = pist;
        a.partial = nullptr;
        a.ksplit = 1;
        a.kspan = K;
        a.phi_part = nullptr;
        if ((st = run_sum(precision, qrfs::BASIS_PHASE, qrfs::EPI_STORE, a, ns, stream_)))
            return st;
        e = qrfs::launch_temporal_rows(fp64, pist, rows, M,
                                       part + (r0 / qrfs::TEMPORAL_ROWS_PER_BLOCK) * M * 2,
                                       stream_);
        if (e != hipSuccess) return hip_fail(e, "temporal estimator launch");
    }
    e = qrfs::launch_reduce_sf(part, nb, M, R, sf, sf_stderr, stream_);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    s->index += (uint64_t)(n_sets * K);
    return ok();
}

qrfs_status qrfs_diff_piston_structure_sets(qrfs_context* ctx, int64_t K, const double* fx,
                                            const double* fy, const double* w, int64_t nB,
                                            const double* bx, const double* by, int64_t R,
                                            int64_t R_block, const qrfs_rng* rng,
                                            int32_t precision, double* sf, double* sf_stderr,
                                            void* stream) {
    qrfs_status st = check_sum_common(K, nB, R, R_block, rng, nullptr, precision);
    if (st) return st;
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(w);
    CHECK_PTR(bx);
    CHECK_PTR(by);
    CHECK_PTR(sf);
    if (sf_stderr && !aligned8(sf_stderr))
        return fail(QRFS_ERR_INVALID_ARG, "sf_stderr is not 8-byte aligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    const qrfs::SfPlan plan = qrfs::sf_plan(precision, K, R, R_block, nB);
    const size_t partial_bytes = align256((size_t)(plan.n_partial_tiles * nB) * 2 * sizeof(double));
    const size_t phi_bytes = align256(plan.phi_floats * sizeof(float));
    if ((st = ensure_workspace(ctx, partial_bytes + phi_bytes))) return st;
    st = sf_sets_enqueue(plan, (char*)ctx->ws, K, fx, fy, w, nB, bx, by, R, R_block, rng,
                         precision, sf, sf_stderr, (hipStream_t)stream);
    return st ? st : ok();
}

qrfs_status qrfs_diff_piston_structure_sets_noalloc(qrfs_context* ctx, int64_t K,
                                                    const double* fx, const double* fy,
                                                    const double* w, int64_t nB,
                                                    const double* bx, const double* by,
                                                    int64_t R, int64_t R_block,
                                                    const qrfs_rng* rng, int32_t precision,
                                                    double* sf, double* sf_stderr,
                                                    void* stream) {
    qrfs_status st = check_sum_common(K, nB, R, R_block, rng, nullptr, precision);
    if (st) return st;
    CHECK_PTR(fx);
    CHECK_PTR(fy);
    CHECK_PTR(w);
    CHECK_PTR(bx);
    CHECK_PTR(by);
    CHECK_PTR(sf);
    if (sf_stderr && !aligned8(sf_stderr))
        return fail(QRFS_ERR_INVALID_ARG, "sf_stderr is not 8-byte aligned");
    if (!ctx) return fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    DeviceGuard g(ctx->device);
    if (!g.okay) return fail(QRFS_ERR_DEVICE, "cannot select device %d", ctx->device);
    const qrfs::SfPlan plan = qrfs::sf_plan(precision, K, R, R_block, nB, kScratchBytes);
    const size_t need = qrfs::sf_plan_bytes(plan, nB);
    if (need > kScratchBytes)
        return fail(QRFS_ERR_INVALID_ARG,
                    "needs %zu bytes of scratch; the allocation-free entry point has %zu "
                    "(fewer sets, realisations or baselines per call)",
                    need, kScratchBytes);
    void* base = scratch_ptr(ctx->device);
    if (!base) return fail(QRFS_ERR_UNSUPPORTED, "no static scratch on device %d", ctx->device);
    st = sf_sets_enqueue(plan, (char*)base, K, fx, fy, w, nB, bx, by, R, R_block, rng, precision,
                         sf, sf_stderr, (hipStream_t)stream);
    return st ? st : ok();
}

}  // extern "C"

namespace {
// The sums of qrfs_diff_piston_structure_sets over caller frequency sets,
// with the plan's scratch at `base`: per-tile partials first, then the
// split-K partial sums (every element the later kernels read is written
// first, so the scratch needs no clearing).
qrfs_status sf_sets_enqueue(const qrfs::SfPlan& plan, char* base, int64_t K, const double* fx,
                            const double* fy, const double* w, int64_t nB, const double* bx,
                            const double* by, int64_t R, int64_t R_block, const qrfs_rng* rng,
                            int32_t precision, double* sf, double* sf_stderr, hipStream_t stream) {
    qrfs_status st;
    const int64_t n_sets = cdiv(R, R_block);
    const size_t partial_bytes = align256((size_t)(plan.n_partial_tiles * nB) * 2 * sizeof(double));
    double* partial = (double*)base;
    float* phi = (float*)(base + partial_bytes);
    qrfs::SumArgs a{};
    a.K = K;
    a.fx = fx;
    a.fy = fy;
    a.w = w;
    a.P = nB;
    a.px = bx;
    a.py = by;
    a.R = R;
    a.R_block = R_block;
    a.seed = rng->seed;
    a.counter = rng->counter;
    a.mode = rng->mode;
    a.partial = partial;
    a.ksplit = plan.ksplit;
    a.kspan = plan.kspan;
    a.phi_part = phi;
    if ((st = run_sum(precision, qrfs::BASIS_DIFF, qrfs::EPI_SFSUM, a, n_sets, stream))) return st;
    if (plan.ksplit > 1) {
        hipError_t e = qrfs::launch_sfsum_rows(phi, plan.ksplit, R, nB, partial, stream);
        if (e != hipSuccess) return hip_fail(e, "split-K square launch");
    }
    hipError_t e = qrfs::launch_reduce_sf(partial, plan.n_partial_tiles, nB, R, sf, sf_stderr,
                                          stream);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    return QRFS_OK;
}
}  // namespace
