// qrfs_batch.cpp -- batched persistent launches of uneven phase-field,
// piston and tilt instances: work list (longest items first), autotuned launch shape, and
// HIP graph capture of the whole sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qrfs.h"
#include "qrfs_internal.hpp"

namespace qrfs {
// defined in qrfs_api.cpp
qrfs_status api_fail(qrfs_status s, const char* fmt, ...);
qrfs_status api_ok();
int api_context_device(const qrfs_context* ctx);
int64_t api_context_range_freqs(const qrfs_context* ctx);
}  // namespace qrfs

// Coefficient tiles of a two-phase batch take at most this much device
// memory; larger batches are left to the fused shapes.
static constexpr size_t kBatchTileCap = (size_t)16 << 30;

struct qrfs_batch {
    int device = 0;
    int precision = 1;
    int n = 0;
    std::vector<qrfs_batch_instance> inst;
    std::vector<int64_t> n_sets;
    double terms = 0.0;
    // device buffers
    void* freq = nullptr;      // fx, fy, area, w of every instance
    qrfs::SumArgs* d_args = nullptr;
    qrfs::BatchItem* d_items = nullptr;
    unsigned* d_counter = nullptr;
    std::vector<qrfs::SumArgs> args;  // host copy (frequency pointers into `freq`)
    std::vector<double*> fx, fy, area, w;
    int n_items = 0;
    int shape = 0;
    bool has_ap = false;  // some instance computes pistons or tilts
    int n_cu = 256;
    // two-phase form: coefficient tiles of every instance and its launch
    // arguments (allocated on first use of the two-phase shape)
    int64_t range_freqs = 2048;
    size_t tile_bytes = 0;  // 0: the two-phase shape is not available
    void* tiles = nullptr;
    qrfs::WideArgs* d_wargs = nullptr;
    std::vector<qrfs::WideArgs> wargs;
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_shape = -1;
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

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

qrfs_status check_instance(const qrfs_batch_instance& in, int64_t i) {
    const qrfs_psd& p = in.psd;
    if (p.model != QRFS_PSD_KOLMOGOROV && p.model != QRFS_PSD_VON_KARMAN)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: unknown PSD model", (long long)i);
    if (!(p.r0 > 0.0) || (p.model == QRFS_PSD_VON_KARMAN && !(p.L0 > 0.0)))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: r0 and L0 must be > 0", (long long)i);
    if (!std::isfinite(p.c) || !(p.wavelength >= 0.0) || !std::isfinite(p.wavelength))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: PSD constant or wavelength invalid",
                        (long long)i);
    const qrfs_sampler& s = in.sampler;
    const int sc = s.scheme;
    if (sc == QRFS_SAMPLER_R2_CARTESIAN || sc == QRFS_SAMPLER_RANDOM_CARTESIAN ||
        sc == QRFS_SAMPLER_JITTER) {
        if (s.N <= 0 || !(s.df > 0.0))
            return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: Cartesian N, df must be > 0",
                            (long long)i);
        if (sc == QRFS_SAMPLER_JITTER && in.K != (int64_t)s.N * s.N)
            return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: jittered grid needs K = N^2",
                            (long long)i);
    } else if (sc == QRFS_SAMPLER_R2_LOGPOLAR || sc == QRFS_SAMPLER_RANDOM_LOGPOLAR) {
        if (!(s.fmin > 0.0) || !(s.fmax > s.fmin))
            return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: needs 0 < fmin < fmax",
                            (long long)i);
    } else if (sc == QRFS_SAMPLER_R2_DISC || sc == QRFS_SAMPLER_RANDOM_DISC) {
        if (!(s.fmax > 0.0))
            return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: needs fmax > 0", (long long)i);
    } else {
        return api_fail(QRFS_ERR_UNSUPPORTED, "instance %lld: sampler scheme %d not accepted",
                        (long long)i, s.scheme);
    }
    if (in.K <= 0 || in.P <= 0 || in.R <= 0)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: K, P, R must be > 0", (long long)i);
    if (in.R_block < 1 || in.R_block > in.R)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: R_block must be in [1, R]",
                        (long long)i);
    if (in.K > ((int64_t)1 << 33) || in.R > ((int64_t)1 << 31) || in.P > ((int64_t)1 << 31))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: sizes too large", (long long)i);
    if (!in.px || !in.py || !in.phase)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: NULL array", (long long)i);
    if (((uintptr_t)in.px & 7) || ((uintptr_t)in.py & 7) || ((uintptr_t)in.phase & 3))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: misaligned array", (long long)i);
    if (in.rng.mode != QRFS_COEF_GAUSS_CS && in.rng.mode != QRFS_COEF_EQ3)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: unknown coefficient mode",
                        (long long)i);
    if (!in.apD != !in.apd)
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: apD and apd go together",
                        (long long)i);
    if (((uintptr_t)in.apD & 7) || ((uintptr_t)in.apd & 7))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: misaligned array", (long long)i);
    if (!std::isfinite(in.ux) || !std::isfinite(in.uy))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: direction not finite",
                        (long long)i);
    if (!in.apD && (in.ux != 0.0 || in.uy != 0.0))
        return api_fail(QRFS_ERR_INVALID_ARG, "instance %lld: a tilt direction needs apertures",
                        (long long)i);
    return QRFS_OK;
}

// Coefficient-tile bytes of instance i in the two-phase form (all sets).
size_t wide_instance_bytes(const qrfs_batch* b, int i) {
    const qrfs_batch_instance& in = b->inst[i];
    const int KCH = qrfs::wide_chunk(b->precision);
    const int64_t nkv = cdiv(in.K, KCH) * 2 * KCH;
    const int64_t rt32 = cdiv(in.R_block, 256) * 8;
    size_t bytes = (size_t)b->n_sets[i] * rt32 * qrfs::wide_frag_bytes_per_row32(b->precision, nkv);
    return (bytes + 255) & ~(size_t)255;
}

// Allocates the coefficient tiles and the per-instance launch arguments of
// the two-phase form (once).
qrfs_status ensure_wide(qrfs_batch* b) {
    if (b->tiles) return QRFS_OK;
    if (!b->tile_bytes) return api_fail(QRFS_ERR_UNSUPPORTED, "two-phase shape unavailable");
    // FP16x3: after the tiles and the 256-byte sink, one power of two per
    // set of every instance (the scale of its coefficient tiles)
    size_t scale_bytes = 0;
    if (b->precision == QRFS_PREC_FP16X3)
        for (int i = 0; i < b->n; ++i) scale_bytes += (size_t)b->n_sets[i] * sizeof(double);
    hipError_t e = hipMalloc(&b->tiles, b->tile_bytes + 256 + scale_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_wargs, sizeof(qrfs::WideArgs) * b->n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (b->tiles) (void)hipFree(b->tiles);
        b->tiles = nullptr;
        return api_fail(QRFS_ERR_OUT_OF_MEMORY, "coefficient tiles: %s", hipGetErrorString(e));
    }
    const int KCH = qrfs::wide_chunk(b->precision);
    char* p = (char*)b->tiles;
    double* scales = (double*)((char*)b->tiles + b->tile_bytes + 256);
    b->wargs.clear();
    for (int i = 0; i < b->n; ++i) {
        const qrfs_batch_instance& in = b->inst[i];
        qrfs::WideArgs wa{};
        wa.s = b->args[i];
        const int64_t nch = cdiv(in.K, KCH);
        wa.row_off = 0;
        wa.rows = in.R_block;
        wa.rts = cdiv(in.R_block, 256);
        wa.rt32 = wa.rts * 8;
        wa.cts = cdiv(in.P, 256);
        wa.nkv = nch * 2 * KCH;
        wa.ch0 = 0;
        wa.ch1 = nch;
        int64_t rch = b->precision == QRFS_PREC_SPLIT_BF16 ? nch : cdiv(b->range_freqs, KCH);
        wa.range_ch = rch + (rch & 1);
        wa.accumulate = 0;
        wa.ctile = p;
        wa.sink = (float*)((char*)b->tiles + b->tile_bytes);
        if (b->precision == QRFS_PREC_FP16X3) {
            wa.ascale = scales;
            scales += b->n_sets[i];
        }
        p += wide_instance_bytes(b, i);
        b->wargs.push_back(wa);
    }
    e = hipMemcpy(b->d_wargs, b->wargs.data(), sizeof(qrfs::WideArgs) * b->n,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hfail(e, "two-phase instance upload");
    return QRFS_OK;
}

// A captured graph holds the device addresses of the work list and of the
// two-phase buffers as kernel arguments; it is dropped whenever those are
// rebuilt, so the next graph execution captures the new ones.
void drop_graph(qrfs_batch* b) {
    if (b->exec) {
        (void)hipDeviceSynchronize();  // a replay in flight still reads its arguments
        (void)hipGraphExecDestroy(b->exec);
    }
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_shape = -1;
}

// Work list for the current shape: every (instance, set, row tile, column
// tile), sorted by decreasing cost (rows x columns x K), stable.
qrfs_status build_items(qrfs_batch* b) {
    drop_graph(b);
    qrfs::BatchShape sh = qrfs::batch_shape(b->precision, b->shape);
    if (sh.wide) {
        qrfs_status s = ensure_wide(b);
        if (s) return s;
    }
    const int64_t MT = sh.wide ? 256 : 32 * sh.MW * 4, NT = sh.wide ? 256 : 32 * sh.NB;
    struct Rec {
        double cost;
        qrfs::BatchItem it;
    };
    std::vector<Rec> recs;
    for (int i = 0; i < b->n; ++i) {
        const qrfs_batch_instance& in = b->inst[i];
        const int64_t rts = cdiv(in.R_block, MT), cts = cdiv(in.P, NT);
        for (int64_t s = 0; s < b->n_sets[i]; ++s) {
            int64_t rows_set = std::min(in.R, (s + 1) * in.R_block) - s * in.R_block;
            for (int64_t rt = 0; rt < rts; ++rt) {
                int64_t rows = std::min<int64_t>(MT, rows_set - rt * MT);
                if (rows <= 0) continue;
                for (int64_t ct = 0; ct < cts; ++ct) {
                    Rec r;
                    r.cost = (double)in.K * (double)MT * (double)NT;
                    r.it = {i, (int32_t)s, (int32_t)rt, (int32_t)ct};
                    recs.push_back(r);
                }
            }
        }
    }
    if (recs.size() > (size_t)0x7fffffff)
        return api_fail(QRFS_ERR_INVALID_ARG, "batch has too many work items");
    std::stable_sort(recs.begin(), recs.end(),
                     [](const Rec& x, const Rec& y) { return x.cost > y.cost; });
    std::vector<qrfs::BatchItem> items(recs.size());
    for (size_t j = 0; j < recs.size(); ++j) items[j] = recs[j].it;
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    hipError_t e = hipMalloc(&b->d_items, sizeof(qrfs::BatchItem) * std::max<size_t>(1, items.size()));
    if (e != hipSuccess) return api_fail(QRFS_ERR_OUT_OF_MEMORY, "work list: %s", hipGetErrorString(e));
    e = hipMemcpy(b->d_items, items.data(), sizeof(qrfs::BatchItem) * items.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hfail(e, "work list upload");
    b->n_items = (int)items.size();
    return QRFS_OK;
}

// The whole sequence on one stream: per-instance sampler and weights, then
// the persistent kernel.
qrfs_status enqueue(qrfs_batch* b, hipStream_t st) {
    for (int i = 0; i < b->n; ++i) {
        const qrfs_batch_instance& in = b->inst[i];
        const qrfs_sampler& s = in.sampler;
        hipError_t e = qrfs::launch_sample(s.scheme, s.seed_x, s.seed_y, s.index, b->n_sets[i],
                                           in.K, s.N, s.df, s.fmin, s.fmax, b->fx[i], b->fy[i],
                                           b->area[i], st);
        if (e != hipSuccess) return hfail(e, "sampler launch");
        const double c = qrfs::psd_constant(in.psd.c, in.psd.wavelength);
        e = qrfs::launch_weights(in.psd.model, c, in.psd.r0, in.psd.L0, 0, 0.0, 0.0, 0,
                                 b->n_sets[i] * in.K, b->fx[i], b->fy[i], b->area[i], b->w[i], st);
        if (e != hipSuccess) return hfail(e, "weights launch");
    }
    qrfs::BatchShape sh = qrfs::batch_shape(b->precision, b->shape);
    int blocks = std::max(1, std::min(b->n_items, b->n_cu * sh.blocks_per_cu));
    hipError_t e;
    if (sh.wide) {
        for (int i = 0; i < b->n; ++i) {
            if (b->precision == QRFS_PREC_FP16X3) {
                e = qrfs::launch_wide_scale(b->w[i], b->inst[i].K, b->n_sets[i],
                                            (double*)b->wargs[i].ascale, st);
                if (e != hipSuccess) return hfail(e, "tile scale launch");
            }
            e = qrfs::launch_wide_coef(b->precision, b->wargs[i], st);
            if (e != hipSuccess) return hfail(e, "coefficient tile launch");
        }
        e = qrfs::launch_wide_batch(b->precision, b->has_ap, b->d_wargs, b->d_items, b->n_items,
                                    b->d_counter, blocks, st);
    } else {
        e = qrfs::launch_batch(b->precision, sh, b->has_ap, b->d_args, b->d_items, b->n_items,
                               b->d_counter, blocks, st);
    }
    if (e != hipSuccess) return hfail(e, "persistent launch");
    return QRFS_OK;
}

// Key of a batch in the autotune cache: FNV-1a (64-bit) over the device's
// architecture name and compute-unit count, the precision and each
// instance's sizes and basis flags -- what the launch shapes' timings
// depend on.
uint64_t tuning_key(const qrfs_batch* b) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    };
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess)
        mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    mix(&b->n_cu, sizeof(b->n_cu));
    mix(&b->precision, sizeof(b->precision));
    for (int i = 0; i < b->n; ++i) {
        const qrfs_batch_instance& in = b->inst[i];
        const int64_t v[6] = {in.K, in.P, in.R, in.R_block, in.apD ? 1 : 0,
                              (in.ux != 0.0 || in.uy != 0.0) ? 1 : 0};
        mix(v, sizeof(v));
    }
    return h;
}

// Last line of the cache file with this key; false when there is none (a
// missing or unreadable file is an empty cache).
bool cache_lookup(const char* path, uint64_t key, int* shape, double* ms) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        unsigned long long k = 0;
        int sh = -1;
        double t = 0.0;
        if (sscanf(line, "qrfs-autotune-1 %llx %d %lf", &k, &sh, &t) == 3 && k == key) {
            *shape = sh;
            *ms = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

bool cache_append(const char* path, uint64_t key, int shape, double ms) {
    FILE* f = fopen(path, "a");
    if (!f) return false;
    const bool okw = fprintf(f, "qrfs-autotune-1 %016llx %d %.6f\n", (unsigned long long)key,
                             shape, ms) > 0;
    return (fclose(f) == 0) && okw;
}

}  // namespace

extern "C" {

qrfs_status qrfs_batch_create(qrfs_context* ctx, int64_t n, const qrfs_batch_instance* inst,
                              int32_t precision, qrfs_batch** out) {
    if (!out) return api_fail(QRFS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n <= 0 || n > 65535) return api_fail(QRFS_ERR_INVALID_ARG, "n must be in [1, 65535]");
    if (!inst) return api_fail(QRFS_ERR_INVALID_ARG, "instances are NULL");
    if (precision == QRFS_PREC_FP64)
        return api_fail(QRFS_ERR_UNSUPPORTED, "batches run on the matrix cores (no FP64 path)");
    if (precision != QRFS_PREC_FP32 && precision != QRFS_PREC_SPLIT_BF16 &&
        precision != QRFS_PREC_BF16X6 && precision != QRFS_PREC_FP16X3)
        return api_fail(QRFS_ERR_INVALID_ARG, "unknown precision %d", precision);
    for (int64_t i = 0; i < n; ++i) {
        qrfs_status s = check_instance(inst[i], i);
        if (s) return s;
    }
    if (!ctx) return api_fail(QRFS_ERR_INVALID_ARG, "context is NULL");
    const int dev = qrfs::api_context_device(ctx);
    Guard g(dev);
    if (!g.okay) return api_fail(QRFS_ERR_DEVICE, "cannot select device %d", dev);
    qrfs_batch* b = new (std::nothrow) qrfs_batch();
    if (!b) return api_fail(QRFS_ERR_OUT_OF_MEMORY, "host allocation of the batch");
    b->device = dev;
    b->precision = precision;
    b->n = (int)n;
    b->inst.assign(inst, inst + n);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
        b->n_cu = ncu;
    size_t total = 0;
    for (int i = 0; i < b->n; ++i) {
        int64_t ns = cdiv(b->inst[i].R, b->inst[i].R_block);
        b->n_sets.push_back(ns);
        total += (size_t)(ns * b->inst[i].K) * 4;
        b->terms += (double)b->inst[i].R * (double)b->inst[i].K * (double)b->inst[i].P;
    }
    hipError_t e = hipMalloc(&b->freq, total * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->d_args, sizeof(qrfs::SumArgs) * b->n);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, 256);
    if (e != hipSuccess) {
        qrfs_batch_destroy(b);
        return api_fail(QRFS_ERR_OUT_OF_MEMORY, "batch buffers: %s", hipGetErrorString(e));
    }
    double* p = (double*)b->freq;
    for (int i = 0; i < b->n; ++i) {
        const qrfs_batch_instance& in = b->inst[i];
        const int64_t m = b->n_sets[i] * in.K;
        b->fx.push_back(p);
        b->fy.push_back(p + m);
        b->area.push_back(p + 2 * m);
        b->w.push_back(p + 3 * m);
        p += 4 * m;
        qrfs::SumArgs a{};
        a.K = in.K;
        a.fx = b->fx[i];
        a.fy = b->fy[i];
        a.w = b->w[i];
        a.P = in.P;
        a.px = in.px;
        a.py = in.py;
        a.R = in.R;
        a.R_block = in.R_block;
        a.set0 = 0;
        a.set1 = b->n_sets[i];
        a.seed = in.rng.seed;
        a.counter = in.rng.counter;
        a.mode = in.rng.mode;
        a.out = in.phase;
        a.ksplit = 1;
        a.kspan = in.K;
        if (in.apD) {
            a.apD = in.apD;
            a.apd = in.apd;
            b->has_ap = true;
            if (in.ux != 0.0 || in.uy != 0.0) {
                a.grad = 1;
                a.gx = 2.0 * M_PI * in.ux;
                a.gy = 2.0 * M_PI * in.uy;
            }
        }
        b->args.push_back(a);
    }
    e = hipMemcpy(b->d_args, b->args.data(), sizeof(qrfs::SumArgs) * b->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        qrfs_batch_destroy(b);
        return hfail(e, "instance upload");
    }
    // the two-phase shape is offered when its coefficient tiles fit the cap;
    // it is the starting shape then
    b->range_freqs = qrfs::api_context_range_freqs(ctx);
    size_t tb = 0;
    for (int i = 0; i < b->n; ++i) tb += wide_instance_bytes(b, i);
    b->tile_bytes = tb <= kBatchTileCap ? tb : 0;
    b->shape = b->tile_bytes ? qrfs::batch_shape_count(b->precision) - 1 : 0;
    qrfs_status s = build_items(b);
    if (s) {
        qrfs_batch_destroy(b);
        return s;
    }
    *out = b;
    return api_ok();
}

qrfs_status qrfs_batch_execute(qrfs_batch* b, int32_t use_graph, void* stream) {
    if (!b) return api_fail(QRFS_ERR_INVALID_ARG, "batch is NULL");
    Guard g(b->device);
    if (!g.okay) return api_fail(QRFS_ERR_DEVICE, "cannot select device %d", b->device);
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) {
        qrfs_status s = enqueue(b, st);
        return s ? s : api_ok();
    }
    if (!b->exec || b->graph_shape != b->shape) {
        drop_graph(b);
        hipError_t e = hipSuccess;
        if (!b->cap_stream) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hfail(e, "capture stream");
        e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hfail(e, "begin capture");
        qrfs_status s = enqueue(b, b->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
        if (s) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e2 != hipSuccess) return hfail(e2, "end capture");
        b->graph = graph;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hfail(e, "graph instantiate");
        }
        b->graph_shape = b->shape;
    }
    hipError_t e = hipGraphLaunch(b->exec, st);
    if (e != hipSuccess) return hfail(e, "graph launch");
    return api_ok();
}

qrfs_status qrfs_batch_autotune(qrfs_batch* b, void* stream, const char* cache_path,
                                double* best_ms) {
    if (!b) return api_fail(QRFS_ERR_INVALID_ARG, "batch is NULL");
    Guard g(b->device);
    if (!g.okay) return api_fail(QRFS_ERR_DEVICE, "cannot select device %d", b->device);
    hipStream_t st = (hipStream_t)stream;
    uint64_t key = 0;
    if (cache_path) {
        key = tuning_key(b);
        int shape = -1;
        double ms = 0.0;
        if (cache_lookup(cache_path, key, &shape, &ms) &&
            shape >= 0 && shape < qrfs::batch_shape_count(b->precision) &&
            !(qrfs::batch_shape(b->precision, shape).wide && !b->tile_bytes)) {
            b->shape = shape;
            qrfs_status s = build_items(b);
            if (s) return s;
            if (best_ms) *best_ms = ms;
            return api_ok();
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hfail(e, "event create");
    int best = b->shape;
    float best_t = 1e30f;
    qrfs_status s = QRFS_OK;
    for (int id = 0; id < qrfs::batch_shape_count(b->precision) && !s; ++id) {
        if (qrfs::batch_shape(b->precision, id).wide && !b->tile_bytes) continue;
        b->shape = id;
        if ((s = build_items(b))) break;
        if ((s = enqueue(b, st))) break;  // warm-up
        float t = 1e30f;
        for (int rep = 0; rep < 2 && !s; ++rep) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) s = enqueue(b, st);
            if (!s && e == hipSuccess) e = hipEventRecord(e1, st);
            if (!s && e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (!s && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) s = hfail(e, "autotune timing");
            if (!s) t = std::min(t, ms);
        }
        if (!s && t < best_t) {
            best_t = t;
            best = id;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    b->shape = best;
    if ((s = build_items(b))) return s;
    if (best_ms) *best_ms = best_t;
    if (cache_path && !cache_append(cache_path, key, best, best_t))
        return api_fail(QRFS_ERR_INVALID_ARG, "cannot append to the autotune cache %s", cache_path);
    return api_ok();
}

qrfs_status qrfs_batch_set_shape(qrfs_batch* b, int32_t shape) {
    if (!b) return api_fail(QRFS_ERR_INVALID_ARG, "batch is NULL");
    if (shape < 0 || shape >= qrfs::batch_shape_count(b->precision))
        return api_fail(QRFS_ERR_INVALID_ARG, "shape %d out of range", shape);
    if (qrfs::batch_shape(b->precision, shape).wide && !b->tile_bytes)
        return api_fail(QRFS_ERR_UNSUPPORTED, "two-phase shape: coefficient tiles exceed %zu bytes",
                        kBatchTileCap);
    Guard g(b->device);
    if (!g.okay) return api_fail(QRFS_ERR_DEVICE, "cannot select device %d", b->device);
    const int prev = b->shape;
    b->shape = shape;
    qrfs_status s = build_items(b);
    if (s) {
        b->shape = prev;
        (void)build_items(b);
        return s;
    }
    return api_ok();
}

qrfs_status qrfs_batch_info(const qrfs_batch* b, int64_t* n_items, int32_t* shape, double* terms) {
    if (!b) return api_fail(QRFS_ERR_INVALID_ARG, "batch is NULL");
    if (n_items) *n_items = b->n_items;
    if (shape) *shape = b->shape;
    if (terms) *terms = b->terms;
    return api_ok();
}

qrfs_status qrfs_batch_destroy(qrfs_batch* b) {
    if (!b) return api_ok();
    {
        Guard g(b->device);
        (void)hipDeviceSynchronize();
        drop_graph(b);
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
        if (b->freq) (void)hipFree(b->freq);
        if (b->d_args) (void)hipFree(b->d_args);
        if (b->d_items) (void)hipFree(b->d_items);
        if (b->d_counter) (void)hipFree(b->d_counter);
        if (b->tiles) (void)hipFree(b->tiles);
        if (b->d_wargs) (void)hipFree(b->d_wargs);
    }
    delete b;
    return api_ok();
}

}  // extern "C"
