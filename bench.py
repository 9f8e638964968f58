"""Benchmark of the differential-piston structure-function path on one MI355X.

Workload (all inputs synthetic and seeded): two D = 1.8 m apertures, 32
baselines log-spaced over 1-130 m, von Karman r0 = 0.1 m with L0 in
{10, 25, 100} m, log-polar R2 frequencies over [1e-3, 1e2] cycles/m,
K = 16384 frequencies per set, R = 100000 realisations per L0, R_block
realisations per frequency set (default 256).  The contraction runs in
FP16x3 by default (operands split into fp16 hi + lo, three products on the
matrix cores, FP32-class accuracy: it meets the FP32 parity tolerance); the
same workload with the FP32 MFMA contraction is timed as a reference.

One step = for each L0: draw the frequency sets (R2 sampler), weight them
(PSD x aperture filter), and run the fused coefficient x basis contraction
with the structure-function epilogue and its reduction.  Inputs are
resident in HBM; nothing is copied to or from the host inside the timed
region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 10] [--warmup 10] [--precision fp16x3]
  python bench.py --mode copy      (HBM counter calibration)
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "synthesized terms/s (R·K·P) and realisations/s at fixed error, plain vs chosen"
PEAKS = {"fp32": 157.3, "split_bf16": 2500.0, "bf16x6": 2500.0, "fp16x3": 2500.0, "fp64": 78.6}  # dense TFLOP/s
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane op per cycle
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
FP32_VECTOR_PEAK = 157.3  # TFLOP/s, MI355X fp32 vector
# the method's vector work: per coefficient Philox4x32-10 (10 rounds x
# (2 products + 2 three-input xors) per 4 words = 10), the uniform (2: one
# funnel shift and one subtraction) and Box-Muller (log, sqrt, sin, cos and
# 2 products per pair: 4 per coefficient); per (frequency, baseline, set)
# the FP64 product and range reduction (5), the difference basis sin,
# sin^2 (5) and the amplitude (2)
METHOD_OPS_PER_COEF = 16.0
METHOD_OPS_PER_BASIS = 12.0
PREC_IDS = {"fp64": 0, "fp32": 1, "split_bf16": 2, "bf16x6": 3, "fp16x3": 4}
# MFMA FLOPs executed per algorithmic flop (split-BF16 runs 3 products, BF16x6 six)
MFMA_PASSES = {"fp32": 1, "split_bf16": 3, "bf16x6": 6, "fp16x3": 3, "fp64": 1}
DTYPES = {"fp32": "f32", "split_bf16": "bf16x3", "bf16x6": "bf16x6", "fp16x3": "fp16x3", "fp64": "f64"}
# HBM bytes per launch of the timed kernel group (sum kernel, split-K row sums,
# final reduction) from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a 1 GiB copy
# (x2.0 / x1.0), valid only for the kernel source they were taken with
# sources the structure-function kernels are built from (hashed together)
KERNEL_SOURCES = ("qrfs_kernels.hip", "qrfs_mfma.hpp", "qrfs_device.hpp", "qrfs_internal.hpp")
TRAFFIC = {"sha256_prefix": "19671342cbee67df", "K": 16384, "R": 100000, "R_block": 256,
           "bytes": {"fp16x3": 5.240e8, "fp32": 6.477e8}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=list(PREC_IDS), default="fp16x3")
    ap.add_argument("--mode", choices=["bench", "copy", "peaks"], default="bench",
                    help="copy: only a 1 GiB device-to-device copy, the reference for the "
                         "HBM byte counters; peaks: the measured ceilings of MFMA, vector "
                         "FMA and HBM copy against the nominal peaks")
    ap.add_argument("--R", type=int, default=100000)
    ap.add_argument("--K", type=int, default=16384)
    ap.add_argument("--R-block", type=int, default=256)
    ap.add_argument("--range-freqs", type=int, default=0,
                    help="large_screen: frequencies per FP32-class accumulation range of the "
                         "two-phase kernel (0: the library's default, 2048)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle sample (0 disables it)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the realisations/s-at-fixed-error comparison (plain vs learned)")
    ap.add_argument("--workload", choices=["diffpiston", "phase", "large_screen", "batched",
                                           "temporal", "sampler_ablation"],
                    default="diffpiston",
                    help="diffpiston: the headline line; the others print their own report")
    return ap.parse_args()


def _time_call(fn, reps=3):
    """Median wall time in ms of fn() bracketed by device synchronisation."""
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def train_proposal(q, ctx, cfg, L0, n_ctx=1024, m=2048, steps=2000):
    """The learned proposal of the chosen configuration: trained on
    n_ctx * m = 2.1e6 per-frequency variance contributions the plain method
    generates (the contexts cover D, L0 and the baselines), then tabulated
    for the benchmark's aperture, outer scale and 32 baselines."""
    import numpy as np
    import torch
    import workloads
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    ctxs = torch.as_tensor(workloads.proposal_contexts(n_ctx, seed=0), device=dev)
    prop = q.Proposal(ctx, cfg["fmin"], cfg["fmax"], workloads.mlp_init(0).astype(np.float32))
    plain_rows = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=1 << 40)
    ell, theta, h = prop.rows(plain_rows, ctxs, m, cfg["r0"])
    loss = prop.train(ctxs, ell, theta, h, steps=steps, ctx_per_step=16, lr=2e-3, seed=1)
    prop.tabulate(cfg["D"], L0, cfg["bx"], np.zeros(cfg["bx"].size))
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    info = {"rows": n_ctx * m, "contexts": n_ctx, "steps": steps,
            "train_s": time.perf_counter() - t0,
            "loss_first_last": [float(np.mean(loss[:20])), float(np.mean(loss[-20:]))]}
    return prop, info


def fixed_error(q, ctx, cfg, L0=25.0, R=100000, targets=(0.01, 0.002)):
    """Realisations/s at a fixed error, plain vs chosen (the metric's second
    half).  The error that K controls is the sampling error of the frequency
    sets: given the sets, the coefficients make the estimate's expectation
    the mean over the sets used of S_s(B) = sum_k w_k^2 2 (1 - cos 2 pi f_k.B)
    (qrfs_set_sf_expectation), so E_S(K) = RMS over the 32 baselines of
    that mean against the band-limited analytic curve is the noise-free
    error.  For the plain sampler (log-polar R2) and the learned proposal,
    and for R_block = 256 (391 sets of the continuing sequence) and
    R_block = R (one static set, the case Sec. 2.3 warns about), the
    smallest K on a grid 2^8 .. 2^18 with E_S(K) <= target is found; the
    end-to-end structure function (sampling, weights, sums of R = 1e5
    realisations) is then timed at that K in FP64 and in FP16x3.  The total
    error of each timed run against the curve (noise included; the noise
    floor is sqrt(2/R) = 0.45 % per baseline) is reported beside it."""
    import numpy as np
    import torch
    from oracle import analytic
    dev = torch.device("cuda", 0)
    bx = torch.as_tensor(cfg["bx"], dtype=torch.float64, device=dev)
    by = torch.as_tensor(cfg["by"], dtype=torch.float64, device=dev)
    ap = q.Aperture(cfg["D"], 0.0)
    psd = q.psd(cfg["r0"], L0)
    an = analytic.sf_band(cfg["bx"], cfg["r0"], L0, cfg["fmin"], cfg["fmax"], D=cfg["D"])
    prop, train = train_proposal(q, ctx, cfg, L0)
    samplers = {"plain": lambda: q.logpolar_sampler(cfg["fmin"], cfg["fmax"]),
                "learned": lambda: q.learned_sampler(prop)}
    grid = [1 << e for e in range(8, 19)]
    out = {"L0": L0, "R": R, "training": train, "K_grid": grid, "targets": list(targets),
           "runs": {}}

    def e_s(name, K, Rb):
        n_sets = math.ceil(R / Rb)
        counts = np.full(n_sets, Rb, dtype=np.float64)
        counts[-1] = R - (n_sets - 1) * Rb
        fx, fy, w = ctx.sample_weights(samplers[name](), n_sets, K, psd, ap)
        S = ctx.set_sf_expectation(K, fx, fy, w, n_sets, bx, by).cpu().numpy()
        mean = counts @ S / R
        return float(np.sqrt(np.mean((mean / an - 1.0) ** 2)))

    for Rb in (256, R):
        tag = f"R_block={Rb}"
        curves = {n: [e_s(n, K, Rb) for K in grid] for n in samplers}
        block = {"E_S": curves, "by_target": {}}
        for tgt in targets:
            row = {}
            for n in samplers:
                ks = [K for K, e in zip(grid, curves[n]) if e <= tgt]
                if not ks:
                    row[n] = {"K": None}
                    continue
                K = ks[0]
                row[n] = {"K": K}
                for pname, prec in (("fp64", q.PREC_FP64), ("fp16x3", q.PREC_FP16X3)):
                    res = {}

                    def call():
                        res["sf"] = ctx.diff_piston_structure(
                            psd, ap, bx, by, samplers[n](), K, R, Rb,
                            rng=q.Rng(7, 0, q.COEF_GAUSS_CS), precision=prec)[0]
                    ms = _time_call(call)
                    rel = res["sf"].cpu().numpy() / an - 1.0
                    row[n][pname] = {"ms": ms, "realisations_per_s": R / (ms * 1e-3),
                                     "error_rms": float(np.sqrt(np.mean(rel ** 2))),
                                     "error_max": float(np.max(np.abs(rel)))}
            if row["plain"]["K"] and row["learned"]["K"]:
                base = row["plain"]["fp64"]["realisations_per_s"]
                row["speedup_learned_fp16x3_vs_plain_fp64"] = (
                    row["learned"]["fp16x3"]["realisations_per_s"] / base)
                row["speedup_learned_vs_plain_both_fp16x3"] = (
                    row["learned"]["fp16x3"]["realisations_per_s"] /
                    row["plain"]["fp16x3"]["realisations_per_s"])
                row["speedup_plain_fp16x3_vs_plain_fp64"] = (
                    row["plain"]["fp16x3"]["realisations_per_s"] / base)
            block["by_target"][f"{tgt:.3%}"] = row
        out["runs"][tag] = block
    prop.close()
    return out


def cpu_baseline(cfg, K, target_s):
    """Times the FP64 oracle on a bounded sample of the same workload
    (L0 = 25 m curve, first frequency set, the first R_s realisations)."""
    import numpy as np
    import oracle
    fx, fy, area = oracle.sample_logpolar(1, K, cfg["fmin"], cfg["fmax"])
    w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=25.0, D=cfg["D"])
    nB = cfg["bx"].size

    def run(R_s):
        t = time.perf_counter()
        oracle.diff_piston_sf(fx, fy, w, cfg["bx"], cfg["by"], R_s, R_s, K=K, seed=0)
        return time.perf_counter() - t

    R_s = 32
    dt = run(R_s)
    R_s = int(max(32, min(20000, R_s * target_s / max(dt, 1e-3))))
    dt = run(R_s)
    threads = int(os.environ.get("OMP_NUM_THREADS", 0) or len(os.sched_getaffinity(0)))
    return {"value": R_s * K * nB / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, L0=25 m curve, {R_s} realisations x K={K} x {nB} baselines "
                      f"({dt:.1f} s); realisations/s = {R_s / dt:.1f}",
            "realisations_per_s": R_s / dt, "host": host_cpu()}


def host_cpu():
    """CPU model and the logical CPUs this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def traffic_bytes(args, K, R, Rb):
    """Measured HBM bytes per launch, or None when the kernel source or the
    problem differs from the one the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2404_02978_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()[:16]
    t = TRAFFIC
    if sha != t["sha256_prefix"] or (K, R, Rb) != (t["K"], t["R"], t["R_block"]):
        return None
    return t["bytes"].get(args.precision)


def workload_phase(args):
    """Phase screen, FP64: K = 1024 log-polar frequencies, 32 x 32 points over
    1 m, R = 128; R_block = 1 (paper usage) and 128; empirical structure
    function at the grid separations against the von Karman curve."""
    import numpy as np
    import torch
    import paper_2404_02978_amd as q
    import workloads
    import oracle
    from oracle import analytic
    cfg = workloads.phase_fp64()
    K, R = cfg["K"], cfg["R"]
    ctx = q.Context(0)
    px = torch.as_tensor(cfg["px"], device="cuda")
    py = torch.as_tensor(cfg["py"], device="cuda")
    out = {"workload": "phase screen FP64, K=1024, 32x32 points over 1 m, R=128", "runs": {}}
    for Rb in (1, R):
        n_sets = math.ceil(R / Rb)
        res = {}

        def call():
            s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
            fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
            w = ctx.weights(q.psd(cfg["r0"], cfg["L0"]), fx, fy, area)
            res["out"] = ctx.synthesize_phase(K, fx, fy, w, px, py, R, Rb,
                                              rng=q.Rng(cfg["seed"], 0, 0), precision=q.PREC_FP64)
            res["f"] = (fx, fy, w)
        ms = _time_call(call)
        ph = res["out"].cpu().numpy()
        fx, fy, w = (t.cpu().numpy() for t in res["f"])
        t = time.perf_counter()
        ref = oracle.synthesize(fx, fy, w, cfg["px"], cfg["py"], R, Rb, K=K, seed=cfg["seed"])
        oracle_s = time.perf_counter() - t
        err = float(np.max(np.abs(ph - ref)) / np.sqrt(np.mean(ref ** 2)))
        # empirical SF along x at separations of 1..31 pitches
        g = ph.reshape(R, 32, 32)
        seps = np.arange(1, 32)
        emp = np.array([np.mean((g[:, :, s:] - g[:, :, :-s]) ** 2) for s in seps])
        an = analytic.sf_band(seps / 31.0, cfg["r0"], cfg["L0"], cfg["fmin"], cfg["fmax"])
        res_rel = emp / an - 1
        out["runs"][f"R_block={Rb}"] = {
            "ms": ms, "terms_per_s": R * K * 1024 / (ms * 1e-3), "max_err_vs_oracle": err,
            "oracle_s": oracle_s, "oracle_terms_per_s": R * K * 1024 / oracle_s,
            "sf_rel_err_rms": float(np.sqrt(np.mean(res_rel ** 2))),
            "sf_rel_err_at": {f"{s / 31:.3f} m": float(r) for s, r in zip(seps[::6], res_rel[::6])}}
    print(json.dumps(out), flush=True)


def workload_large_screen(args):
    """Large screen: K = 65536, 256 x 256 points over an 8 m square,
    R = 4096, one frequency set, for r0 = 0.05, 0.1 and 0.2 m; the
    contraction in split-BF16, FP16x3, BF16x6 and FP32 (two-phase kernel:
    coefficient tiles, then 256 x 256 MFMA tiles), each checked against the
    FP64 oracle on realisations 0..63 at 1024
    sampled points (max and RMS phase error in rad), also reported for the
    sampled points inside the circular pupil |x| <= 4 m; the pupil's own
    point set (51 040 points) is timed too.  With --steps >= 2 the fused
    kernel is timed for comparison at r0 = 0.1 m.  The MFMA ceilings the
    device sustains on varied operands (libqrfs_peaks) are measured after
    the runs, and each run's executed MFMA rate is also given against them."""
    import numpy as np
    import torch
    import paper_2404_02978_amd as q
    import workloads
    import oracle
    base = workloads.large_screen()
    K, R = base["K"], base["R"]
    P = base["px"].size
    ctx = q.Context(0)
    px = torch.as_tensor(base["px"], device="cuda")
    py = torch.as_tensor(base["py"], device="cuda")
    s = q.logpolar_sampler(base["fmin"], base["fmax"])
    fx, fy, area = ctx.sample_frequencies(s, 1, K)
    hfx, hfy = fx.cpu().numpy(), fy.cpu().numpy()
    cols = np.random.default_rng(0).choice(P, 1024, replace=False)
    inside = np.hypot(base["px"][cols], base["py"][cols]) <= 4.0
    mask = np.hypot(base["px"], base["py"]) <= 4.0
    mpx = torch.as_tensor(base["px"][mask], device="cuda")
    mpy = torch.as_tensor(base["py"][mask], device="cuda")
    cols_t = torch.as_tensor(cols, device="cuda")
    out = {"workload": "large screen, K=65536, 256x256 points over 8 m, R=4096, "
                       "r0 in {0.05, 0.1, 0.2} m, L0=25 m",
           "flops": 4.0 * R * K * P, "pupil_points": int(mask.sum()),
           "range_freqs": args.range_freqs or 2048, "runs": {}}
    phase = torch.empty((R, P), dtype=torch.float32, device="cuda")
    mphase = torch.empty((R, int(mask.sum())), dtype=torch.float32, device="cuda")
    for r0 in base["r0_list"]:
        w = ctx.weights(q.psd(r0, base["L0"]), fx, fy, area)
        hw = w.cpu().numpy()
        t = time.perf_counter()
        ref = oracle.synthesize(hfx, hfy, hw, base["px"][cols], base["py"][cols], 64, 64, K=K,
                                seed=base["seed"])
        oracle_s = time.perf_counter() - t
        runs = {"oracle_subset_s": oracle_s, "phase_rms_rad": float(np.sqrt(np.mean(ref ** 2)))}
        cases = [("split_bf16", q.PREC_SPLIT_BF16, 3, 2500.0, 2, "mfma_bf16"),
                 ("fp16x3", q.PREC_FP16X3, 3, 2500.0, 2, "mfma_fp16"),
                 ("bf16x6", q.PREC_BF16X6, 6, 2500.0, 2, "mfma_bf16"),
                 ("fp32", q.PREC_FP32, 1, 157.3, 2, "mfma_f32")]
        if r0 == 0.1 and args.steps >= 2:
            cases += [("split_bf16_fused", q.PREC_SPLIT_BF16, 3, 2500.0, 1, "mfma_bf16"),
                      ("fp16x3_fused", q.PREC_FP16X3, 3, 2500.0, 1, "mfma_fp16"),
                      ("bf16x6_fused", q.PREC_BF16X6, 6, 2500.0, 1, "mfma_bf16"),
                      ("fp32_fused", q.PREC_FP32, 1, 157.3, 1, "mfma_f32")]
        for name, prec, passes, peak, path, probe in cases:
            ctx.set_tuning(q.TUNE_WIDE_PATH, path)
            if args.range_freqs:
                ctx.set_tuning(q.TUNE_RANGE_FREQS, args.range_freqs)

            def call():
                ctx.synthesize_phase(K, fx, fy, w, px, py, R, R, rng=q.Rng(base["seed"], 0, 0),
                                     precision=prec, out=phase)
            ms = _time_call(call, reps=3)
            got = phase[:64][:, cols_t].double().cpu().numpy()
            d = got - ref
            alg = 4.0 * R * K * P / (ms * 1e-3) / 1e12
            runs[name] = {"ms": ms, "terms_per_s": R * K * P / (ms * 1e-3),
                          "algorithmic_tflops": alg, "mfma_frac": alg / peak,
                          "executed_mfma_frac": alg * passes / peak,
                          "executed_tflops": alg * passes, "ceiling_probe": probe,
                          "max_abs_err_rad": float(np.max(np.abs(d))),
                          "rms_abs_err_rad": float(np.sqrt(np.mean(d * d))),
                          "pupil_max_abs_err_rad": float(np.max(np.abs(d[:, inside]))),
                          "pupil_rms_abs_err_rad": float(np.sqrt(np.mean(d[:, inside] ** 2)))}
        # the circular pupil alone (split-BF16, two-phase kernel)
        ctx.set_tuning(q.TUNE_WIDE_PATH, 2)

        def call_mask():
            ctx.synthesize_phase(K, fx, fy, w, mpx, mpy, R, R, rng=q.Rng(base["seed"], 0, 0),
                                 precision=q.PREC_SPLIT_BF16, out=mphase)
        ms = _time_call(call_mask, reps=3)
        sel = np.flatnonzero(mask)
        pos = np.searchsorted(sel, cols[inside])
        got = mphase[:64][:, torch.as_tensor(pos, device="cuda")].double().cpu().numpy()
        d = got - ref[:, inside]
        runs["split_bf16_pupil_only"] = {
            "ms": ms, "points": int(mask.sum()),
            "terms_per_s": R * K * mask.sum() / (ms * 1e-3),
            "max_abs_err_rad": float(np.max(np.abs(d))),
            "rms_abs_err_rad": float(np.sqrt(np.mean(d * d)))}
        out["runs"][f"r0={r0}"] = runs
        print(json.dumps({f"r0={r0}": runs}), file=sys.stderr, flush=True)
    ctx.set_tuning(q.TUNE_WIDE_PATH, 0)
    del phase, mphase
    try:
        ceil = {k: probe_ceiling(k, repeats=3) for k in ("mfma_bf16", "mfma_fp16", "mfma_f32")}
        out["measured_ceilings_tflops"] = {k: v["achieved"] for k, v in ceil.items()}
        for runs in out["runs"].values():
            for rec in runs.values():
                if isinstance(rec, dict) and "ceiling_probe" in rec:
                    rec["executed_frac_of_measured"] = (rec["executed_tflops"] /
                                                        ceil[rec["ceiling_probe"]]["achieved"])
    except Exception as exc:  # context only: never lose the measured runs to a probe
        out["measured_ceilings_tflops"] = {"error": f"{type(exc).__name__}: {exc}"}
    print(json.dumps(out), flush=True)


def workload_batched(args):
    """64 uneven instances (D ~ U[0.5, 39] m, grids 32^2..512^2 masked to the
    disk, K = 2^11..2^16, L0 ~ U[10, 100] m, R = 256) in one persistent,
    autotuned launch captured in a HIP graph; one instance checked against
    the FP64 oracle on sampled outputs."""
    import numpy as np
    import torch
    import paper_2404_02978_amd as q
    import workloads
    import oracle
    ctx = q.Context(0)
    inst = []
    specs = workloads.batched()
    for i, d in enumerate(specs):
        inst.append(dict(psd=q.psd(d["r0"], d["L0"]),
                         sampler=q.logpolar_sampler(workloads.FMIN, workloads.FMAX,
                                                    index=i * (1 << 20)),
                         K=d["K"], px=torch.as_tensor(d["px"], device="cuda"),
                         py=torch.as_tensor(d["py"], device="cuda"), R=d["R"], R_block=d["R"],
                         rng=q.Rng(d["seed"], d["counter"], 0)))
    out = {"workload": "64 uneven phase-field instances, R=256 each", "runs": {}}
    for name, prec in (("fp16x3", q.PREC_FP16X3), ("bf16x6", q.PREC_BF16X6),
                       ("split_bf16", q.PREC_SPLIT_BF16)):
        b = q.Batch(ctx, inst, precision=prec)
        terms = b.info()["terms"]
        first_ms = _time_call(lambda: b.execute(), reps=1)
        tuned_ms = b.autotune()
        eager_ms = _time_call(lambda: b.execute())
        graph_ms = _time_call(lambda: b.execute(use_graph=True))
        info = b.info()
        out["runs"][name] = {"terms": terms, "n_items": info["n_items"], "shape": info["shape"],
                             "first_call_ms": first_ms, "autotune_best_ms": tuned_ms,
                             "eager_ms": eager_ms, "graph_ms": graph_ms,
                             "terms_per_s_graph": terms / (graph_ms * 1e-3)}
        if name in ("fp16x3", "bf16x6"):
            j = int(np.argmax([d["K"] for d in specs]))
            d = specs[j]
            fxo, fyo, ao = oracle.sample_logpolar(1, d["K"], workloads.FMIN, workloads.FMAX,
                                                  index=j * (1 << 20))
            wo = oracle.weights(fxo, fyo, ao, r0=d["r0"], L0=d["L0"])
            cols = np.random.default_rng(1).choice(d["px"].size, min(256, d["px"].size),
                                                   replace=False)
            ref = oracle.synthesize(fxo, fyo, wo, d["px"][cols], d["py"][cols], 8, 8, K=d["K"],
                                    seed=d["seed"], counter=d["counter"])
            got = b.outputs[j][:8][:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
            out["runs"][name]["check_instance"] = j
            out["runs"][name]["max_err_vs_oracle"] = float(
                np.max(np.abs(got - ref)) / np.sqrt(np.mean(ref * ref)))
        b.close()
    print(json.dumps(out), flush=True)


def workload_temporal(args):
    """The statistical test of the worked example (Sec. 4.4, Fig. 5): two
    UTs (D = 8 m, d = 1.1 m) 56.5 m apart, frozen flow at 10.2 m/s along the
    baseline, L0 = 22 m, r0 = 0.1 m at 0.5 um, Cartesian R2 with
    df = 0.25/22 and fmax = 0.25 (N = 44, K = 1936) drawn afresh for every
    realisation (R_block = 1), 2000 realisations, 1024 samples 1 ms apart;
    the temporal structure function of the differential piston in FP64,
    FP32 and BF16x6 against the exact expectation over the sampling square
    and the untruncated analytic curve, as OPD (lambda / 2 pi)^2 D in um^2."""
    import numpy as np
    import torch
    import paper_2404_02978_amd as q
    from oracle import analytic as A
    N, df = 44, 0.25 / 22
    K, R, M, dt = N * N, 2000, 1024, 1e-3
    D, d, L0, r0, lam = 8.0, 1.1, 22.0, 0.1, 0.5e-6
    B, v = np.array([56.5, 0.0]), np.array([10.2, 0.0])
    ctx = q.Context(0)
    opd = (lam / (2 * np.pi)) ** 2 * 1e12  # analytic curves: rad^2 -> um^2
    lags = np.array([1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 1023])
    ex = A.temporal_sf_square(lags * dt, B, v, r0, L0, D, d, half_width=0.25, n=200)
    iso = A.temporal_sf(lags * dt, B, v, r0, L0, D, d)
    out = {"workload": "frozen-flow differential piston, UTs 56.5 m apart, 10.2 m/s, L0=22 m, "
                       "Cartesian R2 N=44 (K=1936), R_block=1, R=2000, 1024 samples at 1 ms",
           "terms": float(R) * K * 2 * M, "lags_ms": (lags * dt * 1e3).tolist(),
           "expected_opd_um2_square": (ex * opd).tolist(),
           "analytic_opd_um2_untruncated": (iso * opd).tolist(), "runs": {}}
    for name, prec in (("fp64", q.PREC_FP64), ("fp32", q.PREC_FP32), ("bf16x6", q.PREC_BF16X6)):
        holder = {}

        def call():
            s = q.cartesian_sampler(N, df)
            holder["r"] = ctx.temporal_piston_structure(
                q.psd(r0, L0, wavelength=lam), q.Aperture(D, d), (0.0, 0.0), tuple(-B), tuple(v),
                dt, M, s, K, R,
                1, rng=q.Rng(0, 0, 0), precision=prec)
        ms = _time_call(call, reps=3)
        sf, se = (t.cpu().numpy() for t in holder["r"])
        out["runs"][name] = {"ms": ms, "realisations_per_s": R / (ms * 1e-3),
                             "terms_per_s": R * K * 2 * M / (ms * 1e-3),
                             "opd_um2": (sf[lags] * 1e12).tolist(),  # library gives m^2
                             "z_vs_expected": ((sf[lags] * 1e12 - ex * opd)
                                               / (se[lags] * 1e12)).round(2).tolist()}
    print(json.dumps(out), flush=True)


# FP64 vector ops per unordered pair in k_pair_measures, with 1 - x and
# 1 - y formed once per point: Warnock term (2 minima, product, sum),
# squared distance (2 differences, 2 squares, sum), running minimum (1),
# clash count (compare, add)
PAIR_OPS = 12


def workload_sampler_ablation(args):
    """The samplers Sec. 3.1-3.2 compares (R2 against the jittered grid of
    Eq. 4 and fully random frequencies), on the worked example's Cartesian
    geometry: UTs (D = 8 m, d = 1.1 m), L0 = 22 m, r0 = 0.1 m, df = 0.25/22,
    N = 44 (K = 1936), 2000 fresh sets each (one per realisation, as the
    paper draws them).  Per scheme: minimum pairwise distance (in cells),
    clashes closer than a tenth of a cell, L2 star discrepancy, and the
    per-set sampling error E_S = RMS over 32 baselines (1-130 m) of the
    noise-free structure function against its expectation over the square.
    The pair kernel is timed with events and rated against the FP64 vector
    peak."""
    import numpy as np
    import torch
    import paper_2404_02978_amd as q
    from oracle import analytic as A
    N, df, n_sets = 44, 0.25 / 22, 2000
    K = N * N
    D, d, L0, r0 = 8.0, 1.1, 22.0, 0.1
    B = 10.0 ** np.linspace(0.0, math.log10(130.0), 32)
    ex = A.diff_piston_sf_square(B, 0.0 * B, r0, L0, D, d, half_width=0.25, n=200)
    ctx = q.Context(0)
    dev = torch.device("cuda", 0)
    bx = torch.as_tensor(B, device=dev)
    by = torch.zeros_like(bx)
    L = N * df
    r_clash = 0.1 / N
    pair_ops = n_sets * (K * (K - 1) / 2) * PAIR_OPS
    out = {"workload": "sampler ablation: UTs D=8 m d=1.1 m, L0=22 m, Cartesian N=44 "
                       "(K=1936), 2000 sets per scheme, 32 baselines 1-130 m",
           "clash_radius_cells": 0.1, "schemes": {}}
    samplers = {"r2": lambda: q.cartesian_sampler(N, df),
                "jitter": lambda: q.jitter_sampler(N, df),
                "random": lambda: q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df)}
    for name, mk in samplers.items():
        fx, fy, area = ctx.sample_frequencies(mk(), n_sets, K)
        w = ctx.weights(q.psd(r0, L0), fx, fy, area, q.Aperture(D, d))
        t_meas, t_sf = [], []
        for _ in range(3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            md, nc, T = ctx.point_set_measures(fx, fy, n_sets, K, -L / 2, -L / 2, L, L, r_clash)
            e[1].record()
            S = ctx.set_sf_expectation(K, fx, fy, w, n_sets, bx, by)
            e[2].record()
            torch.cuda.synchronize()
            t_meas.append(e[0].elapsed_time(e[1]))
            t_sf.append(e[1].elapsed_time(e[2]))
        ms_m, ms_s = sorted(t_meas)[1], sorted(t_sf)[1]
        S = S.cpu().numpy()
        es = np.sqrt(np.mean((S / ex[None, :] - 1.0) ** 2, axis=1))
        out["schemes"][name] = {
            "min_dist_cells_mean": float(md.mean().item() * N),
            "min_dist_cells_min": float(md.min().item() * N),
            "clashes_per_set": float(nc.double().mean().item()),
            "l2_star_mean": float(T.mean().item()),
            "E_S_mean": float(es.mean()), "E_S_p95": float(np.percentile(es, 95)),
            "measures_ms": ms_m, "set_sf_ms": ms_s,
            "pair_kernel_alu": {"bound": "alu", "achieved": pair_ops / (ms_m * 1e-3) / 1e12,
                                "peak": VALU_PEAK_TOPS, "unit": "T FP64 ops/s",
                                "frac": pair_ops / (ms_m * 1e-3) / 1e12 / VALU_PEAK_TOPS}}
    print(json.dumps(out), flush=True)


def copy_calibration():
    """A plain 1 GiB device copy: FETCH_SIZE / WRITE_SIZE of this dispatch
    calibrate the HBM byte counters against a known traffic."""
    import torch
    n = (1 << 30) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n}), flush=True)


_X_MFMA, _X_FMA, _Y_FMA = 2.0 ** -6, 1.0, 2.0 ** -10


def _probe_table():
    """(kind, name, operand x (0: varied data), nominal flop/s or B/s, closed
    form of the per-lane sums after `it` rounds, or None: linear in `it`)."""
    from paper_2404_02978_amd import peaks as pk
    x = _X_MFMA
    return [
        (pk.PEAK_MFMA_BF16, "mfma_bf16", 0.0, 2500e12, None),
        (pk.PEAK_MFMA_FP16, "mfma_fp16", 0.0, 2500e12, None),
        (pk.PEAK_MFMA_F32, "mfma_f32", 0.0, 157.3e12, None),
        (pk.PEAK_MFMA_BF16, "mfma_bf16_const", x, 2500e12, lambda it: 64 * it * 16 * x * x),
        (pk.PEAK_MFMA_FP16, "mfma_fp16_const", x, 2500e12, lambda it: 64 * it * 16 * x * x),
        (pk.PEAK_MFMA_F32, "mfma_f32_const", x, 157.3e12, lambda it: 64 * it * 2 * x * x),
        (pk.PEAK_VALU_F32, "valu_fma_f32", _X_FMA, 78.6e12, lambda it: 8 * it * _Y_FMA),
        (pk.PEAK_VALU_F64, "valu_fma_f64", _X_FMA, 78.6e12, lambda it: 8 * it * _Y_FMA),
        (pk.PEAK_HBM_COPY, "hbm_copy", 0.0, 8e12, None),
    ]


def probe_ceiling(name, repeats=5):
    """Runs one probe of libqrfs_peaks: first checked against its expected
    sums on a short run, then timed on one round of resident blocks (about
    50 ms of nominal work), best of `repeats` launches timed with events on
    the stream they run on.  Returns the probe's record (achieved and nominal
    in TFLOP/s or TB/s)."""
    import torch
    from paper_2404_02978_amd import peaks as pk
    kind, _, x, nominal, closed = next(p for p in _probe_table() if p[1] == name)
    st = torch.cuda.current_stream()
    blocks = pk.peak_blocks(kind)
    y = _Y_FMA
    if kind == pk.PEAK_HBM_COPY:
        n = 1 << 28
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.zeros_like(src)
        out, iters, args_ = None, 0, (src, dst, n)
        pk.peak_launch(kind, blocks, 0, x, y, None, src, dst, n, st)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), "copy probe moved the wrong data"
    else:
        out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
        if closed is None:  # varied operands: the sums are linear in the rounds
            pk.peak_launch(kind, blocks, 1, x, y, out, None, None, 0, st)
            ref = 16 * out.clone()
        w16 = pk.peak_launch(kind, blocks, 16, x, y, out, None, None, 0, st)
        torch.cuda.synchronize()
        expect = ref if closed is None else closed(16)
        bad = int((out != expect).sum())
        assert bad == 0, f"{name}: {bad} lanes differ from the expected sums"
        if closed is None:
            assert bool((ref != 0).any()), f"{name}: all sums are zero"
        iters = max(16, int(0.05 * nominal / (w16 / 16)))
        args_ = (None, None, 0)
    work = pk.peak_launch(kind, blocks, iters, x, y, out, *args_, st)  # warm-up
    best = 0.0
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        pk.peak_launch(kind, blocks, iters, x, y, out, *args_, st)
        e1.record(st)
        torch.cuda.synchronize()
        best = max(best, work / (e0.elapsed_time(e1) * 1e-3))
    return {"achieved": best / 1e12, "nominal": nominal / 1e12,
            "unit": "TB/s" if kind == pk.PEAK_HBM_COPY else "TFLOP/s",
            "operands": ("varied" if x == 0.0 else "constant")
            if kind <= pk.PEAK_MFMA_F32 else None,
            "frac": best / nominal, "blocks": blocks, "iters": iters}


def measure_peaks():
    """Throughput the device sustains per instruction class (libqrfs_peaks):
    dense MFMA in bf16, fp16 and FP32 on varied and on constant operands,
    unpacked vector FMA in FP32 and FP64, and a streaming copy, each against
    MI355X's nominal peak."""
    import torch
    out_json = {"mode": "peaks", "device": torch.cuda.get_device_name(0), "probes": {}}
    for p in _probe_table():
        out_json["probes"][p[1]] = probe_ceiling(p[1])
    # matrix-core clock implied by the bf16 probes (2.4 GHz nominal)
    out_json["implied_mfma_clock_ghz"] = {
        k: 2.4 * out_json["probes"][k]["frac"] for k in ("mfma_bf16", "mfma_bf16_const")}
    print(json.dumps(out_json), flush=True)


def main():
    args = parse()
    if args.mode == "copy":
        copy_calibration()
        return
    if args.mode == "peaks":
        measure_peaks()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              "data-parallel over realisation blocks and is measured on a single MI355X.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "diffpiston":
        {"phase": workload_phase, "large_screen": workload_large_screen,
         "batched": workload_batched, "temporal": workload_temporal,
         "sampler_ablation": workload_sampler_ablation}[args.workload](args)
        return
    import numpy as np
    import torch

    import paper_2404_02978_amd as q
    import workloads
    from oracle import analytic

    cfg = workloads.diffpiston(R=args.R, K=args.K)
    K, R, Rb = cfg["K"], cfg["R"], args.R_block
    prec = PREC_IDS[args.precision]
    n_sets = math.ceil(R / Rb)
    cur = {"prec": prec}
    nB = cfg["bx"].size
    L0s = cfg["L0_list"]
    dev = torch.device("cuda", 0)
    bx = torch.as_tensor(cfg["bx"], dtype=torch.float64, device=dev)
    by = torch.as_tensor(cfg["by"], dtype=torch.float64, device=dev)
    ap = q.Aperture(cfg["D"], 0.0)
    ctx = q.Context(0)
    sampler = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
    counter = [0]
    kernel_ms = []
    last_sf = {}
    events = []

    def step(record):
        for L0 in L0s:
            # frequencies and weights in one pass (the cell areas are not needed),
            # the weights for sums in the precision of the step
            fx, fy, w = ctx.sample_weights(sampler, n_sets, K, q.psd(cfg["r0"], L0), ap,
                                           precision=cur["prec"])
            rng = q.Rng(cfg["seed"], counter[0], q.COEF_GAUSS_CS)
            counter[0] += R
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sf, se = ctx.diff_piston_structure_sets(K, fx, fy, w, bx, by, R, Rb, rng=rng,
                                                    precision=cur["prec"])
            e1.record()
            if record:
                events.append((e0, e1))
            last_sf[L0] = (sf, se)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = [a.elapsed_time(b) for a, b in events]

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    terms_per_step = len(L0s) * R * K * nB
    terms_per_s = terms_per_step / (ms_per_step * 1e-3)
    real_per_s = len(L0s) * R / (ms_per_step * 1e-3)

    # error of the estimate against the band-limited analytic curve (RMS over baselines)
    errors = {}
    for L0 in L0s:
        sf, se = last_sf[L0]
        an = analytic.sf_band(cfg["bx"], cfg["r0"], L0, cfg["fmin"], cfg["fmax"], D=cfg["D"])
        rel = sf.cpu().numpy() / an - 1.0
        errors[str(int(L0))] = {"rms": float(np.sqrt(np.mean(rel ** 2))),
                                "max": float(np.max(np.abs(rel)))}

    avg_kernel_ms = float(np.mean(kernel_ms))
    # the method's work per launch: the contraction's 4 flops per term
    # (2 MACs, cos and sin, per (r, k, b)), and, beside it, the vector work
    # of its generator and basis (METHOD_OPS_*), without what the
    # implementation adds (operand splits, basis rebuilt per row tile)
    flops = 4.0 * R * K * nB
    achieved = flops / (avg_kernel_ms * 1e-3) / 1e12
    method_ops = (R * 2.0 * K * METHOD_OPS_PER_COEF
                  + n_sets * K * nB * METHOD_OPS_PER_BASIS)
    alu_view = {"achieved": method_ops / (avg_kernel_ms * 1e-3) / 1e12,
                "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                "frac": method_ops / (avg_kernel_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                "ops_per_launch": method_ops,
                "ops": f"{METHOD_OPS_PER_COEF} per coefficient (Philox4x32-10 10, uniform 2, "
                       f"Box-Muller 4) + {METHOD_OPS_PER_BASIS} per (frequency, baseline, set)"}
    kern = ("k_sum_mfma<diff, sfsum> + k_sfsum_rows + k_reduce_sf (event-timed per launch on "
            "the stream they run on)")
    one_real = Rb == 1 and nB <= 64 and args.precision != "fp64"
    if one_real:
        # one realisation per set: k_sf_one, binary32 FMAs on the vector ALU
        # whatever the FP32-class precision (no operand split, no MFMA)
        kern = "k_sf_one + k_reduce_sf (event-timed per launch on the stream they run on)"
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": None,
                "flops_per_launch": flops, "kernel": kern, "kernel_ms": avg_kernel_ms,
                "alu_view": alu_view}
    elif args.precision == "fp64":
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAKS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAKS["fp64"], "traffic": None,
                "flops_per_launch": flops, "kernel": "k_sum_f64 + k_reduce_sf",
                "kernel_ms": avg_kernel_ms, "alu_view": alu_view}
    else:
        # the contraction on the matrix cores against the dense peak of its
        # operand type; the generator on the vector ALU bounds the kernel
        passes = MFMA_PASSES[args.precision]
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAKS[args.precision],
                "unit": "TFLOP/s", "frac": achieved / PEAKS[args.precision],
                "traffic": traffic_bytes(args, K, R, Rb), "flops_per_launch": flops,
                "kernel": kern, "kernel_ms": avg_kernel_ms,
                "executed_mfma": {"passes": passes, "tflops": achieved * passes,
                                  "frac": achieved * passes / PEAKS[args.precision]},
                "alu_view": alu_view}

    # the same instruction classes measured on this device (libqrfs_peaks),
    # outside the timed region: a busy MI355X holds a clock below 2.4 GHz,
    # and lower still when the matrix cores see changing data
    meas = {}
    mfma_probe = {"fp16x3": "mfma_fp16", "split_bf16": "mfma_bf16", "bf16x6": "mfma_bf16",
                  "fp32": "mfma_f32"}.get(args.precision)
    try:
        if mfma_probe and "executed_mfma" in roof:
            m = probe_ceiling(mfma_probe, repeats=3)
            meas["mfma"] = {"probe": mfma_probe + " (varied operands)", "achieved": m["achieved"],
                            "unit": "TFLOP/s",
                            "executed_frac": roof["executed_mfma"]["tflops"] / m["achieved"]}
        v = probe_ceiling("valu_fma_f32", repeats=3)
        meas["valu"] = {"probe": "valu_fma_f32", "achieved": v["achieved"] / 2,
                        "unit": "T lane-ops/s",
                        "alu_view_frac": alu_view["achieved"] / (v["achieved"] / 2)}
    except Exception as exc:  # context only: never lose the measured line to a probe
        meas["error"] = f"{type(exc).__name__}: {exc}"
    roof["measured_ceilings"] = meas

    # the same workload with the FP32 MFMA contraction, for reference
    fp32_ref = None
    if args.precision != "fp32":
        events.clear()
        cur["prec"] = PREC_IDS["fp32"]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(max(1, args.steps // 2)):
            step(True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        cur["prec"] = prec
        k32 = float(np.mean([a.elapsed_time(b) for a, b in events]))
        ms32 = (t3 - t2) * 1e3 / max(1, args.steps // 2)
        fp32_ref = {"value": terms_per_step / (ms32 * 1e-3), "ms_per_step": ms32,
                    "kernel_ms": k32, "mfma_frac": flops / (k32 * 1e-3) / 1e12 / PEAKS["fp32"]}

    compare = None
    if not args.no_compare:
        compare = fixed_error(q, ctx, cfg)

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(cfg, K, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": terms_per_s, "unit": "terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # the arithmetic the sums run in: binary32 FMAs in k_sf_one
        "dtype": "f32" if one_real else DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": "diff-piston structure function, D=1.8 m, 32 baselines 1-130 m, "
                               "L0 in {10,25,100} m, r0=0.1 m, log-polar R2 K=16384, R=1e5",
                   "K": K, "R": R, "R_block": Rb, "baselines": nB, "L0": list(L0s),
                   "precision": args.precision, "realisations_per_step": len(L0s) * R},
        "realisations_per_s": real_per_s,
        "error_vs_analytic": errors,
        "noise_floor_rms": math.sqrt(2.0 / R),
        "roofline": roof,
        "fp32_mfma_reference": fp32_ref,
        "fixed_error": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
