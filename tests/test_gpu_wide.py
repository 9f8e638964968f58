"""Two-phase contraction (coefficient tiles, then 256 x 256 MFMA tiles) for
wide point sets, against the FP64 oracle through the C ABI.

The two-phase kernel is forced with the context's tuning knob at sizes the
oracle finishes in seconds: ragged rows (sets of 300 and 100 rows), ragged
columns (520 = 2 x 256 + 8), ragged frequency chunks (K = 203), several
frequency ranges added into the output, and coefficient tiles cut into
pieces of sets or of 256-row blocks.  Tolerances as for the fused kernel:
max error relative to the RMS of the oracle output, 1e-5 (FP32, BF16x6),
1e-3 (split-BF16).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {1: 1e-5, 2: 1e-3, 3: 1e-5, 4: 1e-5}
PRECS = [1, 2, 3, 4]


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    q.load_library()
    return q


@pytest.fixture()
def ctx(q):
    c = q.Context(0)
    c.set_tuning(q.TUNE_WIDE_PATH, 2)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def report(name, got, ref, tol):
    d = got - ref
    rms = math.sqrt(np.mean(ref * ref))
    e_rms, e_max = math.sqrt(np.mean(d * d)) / rms, np.max(np.abs(d)) / rms
    print(f"{name}: eps_rms={e_rms:.3e} eps_max={e_max:.3e} tol={tol:g}", flush=True)
    assert e_max <= tol, (name, e_rms, e_max)


def _freqs(ctx, q, n_sets, K, L0=25.0, ap=None, index=0):
    s = q.logpolar_sampler(1e-3, 1e2, index=index)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(0.1, L0), fx, fy, area, None if ap is None else q.Aperture(*ap))
    return fx, fy, w


def _points(P, seed, half=2.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-half, half, P), rng.uniform(-half, half, P)


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("R,R_block", [(300, 300), (700, 300), (256, 256)])
def test_wide_synthesize(q, ctx, precision, R, R_block):
    K, P = 203, 520
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K)
    px, py = _points(P, R)
    print(f"wide synth p{precision} R{R} Rb{R_block} K{K} P{P}", flush=True)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block,
                               rng=q.Rng(3, 500, 0), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=3,
                            counter=500)
    report(f"wide synth p{precision} R{R} Rb{R_block}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("range_freqs", [16, 48, 100])
def test_wide_frequency_ranges(q, ctx, precision, range_freqs):
    """Several launches over frequency ranges, each adding into the output
    (split-BF16 always contracts one range)."""
    ctx.set_tuning(q.TUNE_RANGE_FREQS, range_freqs)
    K, P, R = 203, 300, 280
    fx, fy, w = _freqs(ctx, q, 1, K)
    px, py = _points(P, 5)
    print(f"wide ranges p{precision} range {range_freqs}", flush=True)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R,
                               rng=q.Rng(4, 0, 0), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R, K=K, seed=4)
    report(f"wide ranges p{precision} r{range_freqs}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("cap", [1, 1_000_000, 2_000_000])
def test_wide_pieces(q, ctx, precision, cap):
    """Coefficient tiles cut into pieces: one 256-row block at a time (cap 1),
    or groups of whole sets."""
    ctx.set_tuning(q.TUNE_TILE_BYTES, cap)
    K, P, R, R_block = 150, 260, 1300, 600
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, index=77)
    px, py = _points(P, 6)
    print(f"wide pieces p{precision} cap {cap}", flush=True)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block,
                               rng=q.Rng(8, 9, 0), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=8,
                            counter=9)
    report(f"wide pieces p{precision} cap{cap}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_wide_given_coefficients(q, ctx, precision):
    K, P, R, R_block = 70, 300, 400, 260
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K)
    rng = np.random.default_rng(4)
    coef = rng.normal(size=(R, 2 * K))
    px, py = _points(P, 7)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block, coef=dev(coef),
                               precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, coef=coef)
    report(f"wide given coef p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_wide_eq3_mode(q, ctx, precision):
    K, P, R = 123, 270, 300
    fx, fy, w = _freqs(ctx, q, 1, K)
    px, py = _points(P, 8)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R,
                               rng=q.Rng(5, 3, q.COEF_EQ3), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R, K=K, seed=5, counter=3,
                            mode=1)
    report(f"wide eq3 p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_wide_piston(q, ctx, precision):
    K, R, R_block, n_ap = 97, 300, 300, 300
    fx, fy, w = _freqs(ctx, q, 1, K)
    rng = np.random.default_rng(9)
    cx, cy = rng.uniform(-60, 60, n_ap), rng.uniform(-60, 60, n_ap)
    D = rng.uniform(0.5, 10.0, n_ap)
    d = D * rng.uniform(0.0, 0.3, n_ap)
    out = ctx.piston(K, fx, fy, w, dev(cx), dev(cy), dev(D), dev(d), R, R_block,
                     rng=q.Rng(2, 77, 0), precision=precision)
    ref = oracle.piston(host(fx), host(fy), host(w), cx, cy, D, d, R, R_block, K=K, seed=2,
                        counter=77)
    report(f"wide piston p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_wide_diff_piston(q, ctx, precision):
    K, R, nB = 111, 280, 300
    fx, fy, w = _freqs(ctx, q, 1, K, ap=(1.8, 0.0))
    bx = np.logspace(0, np.log10(130), nB)
    by = np.linspace(-3, 3, nB)
    out = ctx.diff_piston(K, fx, fy, w, dev(bx), dev(by), R, R, rng=q.Rng(0, 5, 0),
                          precision=precision)
    px = np.concatenate([[0.0], bx])
    py = np.concatenate([[0.0], by])
    pist = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R, K=K, seed=0, counter=5)
    ref = pist[:, 1:] - pist[:, :1]
    report(f"wide diff piston p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_wide_matches_fused(q, ctx, precision):
    """Same inputs through both kernels (no oracle): they agree to the
    precision's tolerance."""
    K, P, R, R_block = 1000, 1100, 600, 600
    fx, fy, w = _freqs(ctx, q, 1, K)
    px, py = _points(P, 10, half=4.0)
    args = (K, fx, fy, w, dev(px), dev(py), R, R_block)
    a = host(ctx.synthesize_phase(*args, rng=q.Rng(1, 0, 0), precision=precision))
    ctx.set_tuning(q.TUNE_WIDE_PATH, 1)
    b = host(ctx.synthesize_phase(*args, rng=q.Rng(1, 0, 0), precision=precision))
    report(f"wide vs fused p{precision}", a, b, 2 * TOL[precision])


def test_wide_policy(q):
    """The default policy takes the two-phase kernel for a wide screen and
    the fused kernel for a narrow one; both agree with the oracle."""
    c = q.Context(0)
    try:
        K, R = 64, 512
        fx, fy, w = _freqs(c, q, 1, K)
        for P in (40, 4096):
            px, py = _points(P, P)
            out = c.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R, rng=q.Rng(2, 0, 0),
                                     precision=3)
            ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R, K=K, seed=2)
            report(f"policy P{P}", host(out), ref, TOL[3])
    finally:
        c.close()


@pytest.mark.parametrize("r0", [0.05, 0.1, 0.2])
@pytest.mark.parametrize("precision", PRECS)
def test_wide_large_screen_sampled(q, precision, r0):
    """The 256 x 256-point, 8 m, K = 65536, R = 4096 screen in the launch
    configuration the benchmark times (default policy), for each r0 of the
    workload: sampled realisations and points against the oracle, including
    rows past the first coefficient-tile piece; then the circular pupil
    |x| <= 4 m alone as the point set, at sampled points."""
    cfg = workloads.large_screen()
    c = q.Context(0)
    try:
        K, R = cfg["K"], cfg["R"]
        s = q.logpolar_sampler(1e-3, 1e2)
        fx, fy, area = c.sample_frequencies(s, 1, K)
        w = c.weights(q.psd(r0, cfg["L0"]), fx, fy, area)
        print(f"large screen p{precision} r0 {r0}", flush=True)
        out = c.synthesize_phase(K, fx, fy, w, dev(cfg["px"]), dev(cfg["py"]), R, R,
                                 rng=q.Rng(cfg["seed"], 0, 0), precision=precision)
        torch.cuda.synchronize()
        rows = np.array([0, 1, 255, 256, 2047, 2048, 3000, R - 1])
        cols = np.random.default_rng(0).choice(cfg["px"].size, 96, replace=False)
        got = out[torch.as_tensor(rows).cuda()][:, torch.as_tensor(cols).cuda()]
        got = host(got)
        del out
        hfx, hfy, hw = host(fx), host(fy), host(w)
        ref = np.empty_like(got)
        for i, r in enumerate(rows):
            ref[i] = oracle.synthesize(hfx, hfy, hw, cfg["px"][cols], cfg["py"][cols], 1, 1,
                                       K=K, seed=cfg["seed"], counter=int(r))[0]
        report(f"large screen p{precision} r0 {r0}", got, ref, TOL[precision])
        # the circular pupil as the point set
        mask = np.hypot(cfg["px"], cfg["py"]) <= 4.0
        mx, my = cfg["px"][mask], cfg["py"][mask]
        out = c.synthesize_phase(K, fx, fy, w, dev(mx), dev(my), R, R,
                                 rng=q.Rng(cfg["seed"], 0, 0), precision=precision)
        torch.cuda.synchronize()
        mcols = np.random.default_rng(1).choice(mx.size, 64, replace=False)
        got = host(out[torch.as_tensor(rows[:4]).cuda()][:, torch.as_tensor(mcols).cuda()])
        del out
        ref = np.empty_like(got)
        for i, r in enumerate(rows[:4]):
            ref[i] = oracle.synthesize(hfx, hfy, hw, mx[mcols], my[mcols], 1, 1, K=K,
                                       seed=cfg["seed"], counter=int(r))[0]
        report(f"pupil p{precision} r0 {r0}", got, ref, TOL[precision])
    finally:
        c.close()
