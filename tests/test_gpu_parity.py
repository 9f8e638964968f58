"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (normwise over the compared block, error relative to the RMS of
the oracle; per-element relative error is meaningless at zero crossings):
  FP64        1e-11
  FP32        1e-5   (max error) -- FP32 MFMA, FP32 transcendentals
  SPLIT_BF16  1e-3   (max error) -- bf16 hi+lo operands, FP32 accumulation
  BF16X6      1e-5   (max error) -- bf16 hi+mid+lo operands: FP32-class
Integer work (R2 sequence) is compared bit for bit.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {0: 1e-11, 1: 1e-5, 2: 1e-3, 3: 1e-5, 4: 1e-5}
PRECS = [0, 1, 2, 3, 4]


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    q.load_library()
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def errs(got, ref):
    d = got - ref
    rms = math.sqrt(np.mean(ref * ref))
    return math.sqrt(np.mean(d * d)) / rms, np.max(np.abs(d)) / rms


def report(name, got, ref, tol):
    e_rms, e_max = errs(got, ref)
    print(f"{name}: eps_rms={e_rms:.3e} eps_max={e_max:.3e} tol={tol:g}", flush=True)
    assert e_max <= tol, (name, e_rms, e_max)


# ------------------------------------------------------------- sampler ----

@pytest.mark.parametrize("index", [0, 12345, (1 << 40) + 7, (1 << 64) - 1500])
def test_sampler_cartesian_bit_exact(q, ctx, index):
    """Points bit for bit; the last index runs the 64-bit state across its
    wrap (the exact Weyl sequence is periodic mod 2^64), on both sides."""
    n_sets, K, N, df = 3, 1000, 44, 0.25 / 22
    s = q.cartesian_sampler(N, df, index=index)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    assert s.index == (index + n_sets * K) % (1 << 64)
    rx, ry, ra = oracle.sample_cartesian(n_sets, K, N, df, index=index)
    assert np.array_equal(host(fx), rx) and np.array_equal(host(fy), ry)
    assert np.array_equal(host(area), ra)


def test_synthesize_split_launches(q, ctx):
    """5e6 realisations with fresh frequencies each (R_block = 1): more sets
    than one launch takes (2^22 blocks), so the contraction runs in several
    launches; realisations on both sides of each cut and the last one match
    the oracle."""
    K, R = 8, 5_000_000
    gx, gy = np.meshgrid(np.linspace(-0.5, 0.5, 8), np.linspace(-0.5, 0.5, 8))
    px, py = gx.ravel(), gy.ravel()
    s = q.logpolar_sampler(1e-3, 1e2)
    fx, fy, area = ctx.sample_frequencies(s, R, K)
    w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, 1, rng=q.Rng(7, 0, 0),
                               precision=q.PREC_FP32)
    for r in (0, (1 << 21) - 1, 1 << 21, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, R - 1):
        sl = slice(r * K, (r + 1) * K)
        ref = oracle.synthesize(host(fx[sl]), host(fy[sl]), host(w[sl]), px, py, 1, 1, K=K,
                                seed=7, counter=r)
        report(f"split launches, realisation {r}", host(out[r:r + 1]), ref, 1e-5)
    del out, fx, fy, area, w


def test_sampler_logpolar(q, ctx):
    n_sets, K = 2, 777
    s = q.logpolar_sampler(1e-3, 1e2, index=99, seed_x=3 << 60, seed_y=5 << 59)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    rx, ry, ra = oracle.sample_logpolar(n_sets, K, 1e-3, 1e2, index=99, s0x=3 << 60, s0y=5 << 59)
    f = np.hypot(rx, ry)
    assert np.max(np.abs(host(fx) - rx) / f) < 1e-14
    assert np.max(np.abs(host(fy) - ry) / f) < 1e-14
    assert np.max(np.abs(host(area) / ra - 1)) < 1e-14


def test_sampler_disc(q, ctx):
    """Polar quasi-random frequencies (square-to-disc map): points to 1e-14
    of the radius, equal cell areas pi fmax^2 / K."""
    n_sets, K, fmax = 3, 999, 0.25
    s = q.disc_sampler(fmax, index=12345)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    assert s.index == 12345 + n_sets * K
    rx, ry, ra = oracle.sample_disc(n_sets, K, fmax, index=12345)
    assert np.max(np.abs(host(fx) - rx)) < 1e-14 * fmax
    assert np.max(np.abs(host(fy) - ry)) < 1e-14 * fmax
    assert np.max(np.abs(host(area) / ra - 1)) < 1e-15


@pytest.mark.parametrize("precision", [0, 3, 4])
def test_structure_function_disc_sampler(q, ctx, precision):
    cfg = workloads.diffpiston()
    K, R, R_block, fmax = 600, 300, 100, 0.5
    s = q.disc_sampler(fmax, index=77)
    sf, se = ctx.diff_piston_structure(q.psd(0.1, 25.0), q.Aperture(cfg["D"], 0.0),
                                       dev(cfg["bx"]), dev(cfg["by"]), s, K, R, R_block,
                                       rng=q.Rng(6, 0, 0), precision=precision)
    fx, fy, area = oracle.sample_disc(3, K, fmax, index=77)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0, D=cfg["D"])
    rsf, _ = oracle.diff_piston_sf(fx, fy, w, cfg["bx"], cfg["by"], R, R_block, K=K, seed=6)
    assert np.max(np.abs(host(sf) / rsf - 1)) < (1e-10 if precision == 0 else 2e-5)


def test_sampler_continuation(q, ctx):
    """Two calls continue one sequence (Sec. 3.2: never reinitialised)."""
    s = q.logpolar_sampler(1e-3, 1e2)
    a = ctx.sample_frequencies(s, 1, 500)[0]
    b = ctx.sample_frequencies(s, 1, 300)[0]
    t = q.logpolar_sampler(1e-3, 1e2)
    c = ctx.sample_frequencies(t, 1, 800)[0]
    assert torch.equal(torch.cat([a, b]), c)


# ------------------------------------------------------------- weights ----

@pytest.mark.parametrize("model,L0,ap", [(1, 25.0, None), (1, 10.0, (1.8, 0.0)),
                                         (0, None, (8.0, 1.1))])
def test_weights(q, ctx, model, L0, ap):
    n_sets, K = 2, 1500
    s = q.logpolar_sampler(1e-3, 1e2)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    p = q.psd(0.1, L0, model=model)
    w = ctx.weights(p, fx, fy, area, None if ap is None else q.Aperture(*ap))
    ref = oracle.weights(host(fx), host(fy), host(area), model=model, r0=0.1,
                         L0=L0 or 0.0, D=None if ap is None else ap[0],
                         d=0.0 if ap is None else ap[1])
    g = host(w)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(g - ref)) / scale < 1e-13
    # each weight to 1e-11 relative, except that the aperture filter is held
    # to an absolute 1e-13: a weight w0 F enters the sums of Eq. 3 linearly,
    # so near the zeros of F its error counts against w0, not against w
    w0 = ref if ap is None else oracle.weights(host(fx), host(fy), host(area), model=model,
                                               r0=0.1, L0=L0 or 0.0)
    tol = np.maximum(1e-11 * np.abs(ref), 1e-13 * np.abs(w0)) + 1e-300 + scale * 1e-23
    assert np.all(np.abs(g - ref) <= tol)


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("model,L0,ap", [(1, 25.0, None), (1, 10.0, (1.8, 0.0)),
                                         (0, None, (8.0, 1.1))])
def test_weights_fp32_class(q, ctx, precision, model, L0, ap):
    """Weights for FP32-class sums, every factor to binary32 accuracy: phase
    weights within 3e-7 relative (the PSD power's binary32 Newton step), the
    filter from the shorter J1 with a binary32 Hankel branch within 1e-7 of
    the unfiltered weight on top (a binary32 rounding of a weight is 6e-8 of
    it)."""
    n_sets, K = 2, 1500
    s = q.logpolar_sampler(1e-3, 1e2)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    p = q.psd(0.1, L0, model=model)
    w = ctx.weights(p, fx, fy, area, None if ap is None else q.Aperture(*ap),
                    precision=precision)
    ref = oracle.weights(host(fx), host(fy), host(area), model=model, r0=0.1,
                         L0=L0 or 0.0, D=None if ap is None else ap[0],
                         d=0.0 if ap is None else ap[1])
    g = host(w)
    w0 = oracle.weights(host(fx), host(fy), host(area), model=model, r0=0.1, L0=L0 or 0.0)
    err = np.abs(g - ref) / np.abs(w0)
    print(f"p{precision} ap={ap}: max |dw| / w0 = {err.max():.2e}")
    assert np.all(err <= (3e-7 if ap is None else 4e-7))


@pytest.mark.parametrize("D,d", [(1.8, 0.0), (8.0, 1.1), (39.0, 0.0)])
def test_weights_fp32_class_filter_range(q, ctx, D, d):
    """The FP32-class filter against the binary64 one over arguments pi D f
    from 1e-3 to 1e6 (log-spaced, both sides of the x = 8 switch), with
    w0 = sqrt(W) (unit cell areas)."""
    f = np.exp(np.linspace(np.log(1e-3 / (np.pi * D)), np.log(1e6 / (np.pi * D)), 200003))
    fx, fy, area = dev(f), dev(np.zeros_like(f)), dev(np.ones_like(f))
    p, a = q.psd(0.1, 25.0), q.Aperture(D, d)
    w64 = host(ctx.weights(p, fx, fy, area, a))
    w32 = host(ctx.weights(p, fx, fy, area, a, precision=q.PREC_FP16X3))
    w0 = host(ctx.weights(p, fx, fy, area))
    # the filter's own error, the common PSD factor's (<= 3e-7 relative) aside
    f32, f64 = w32 / host(ctx.weights(p, fx, fy, area, precision=q.PREC_FP16X3)), w64 / w0
    err = np.abs(f32 - f64)
    print(f"D={D} d={d}: max |dF| = {err.max():.2e}")
    assert np.all(err <= 1e-7)


def test_weights_kolmogorov_zero_frequency(q, ctx):
    fx = dev([0.0, 0.5])
    w = ctx.weights(q.psd(0.1), fx, dev([0.0, 0.0]), dev([1.0, 1.0]))
    g = host(w)
    assert g[0] == 0.0 and g[1] > 0.0


# ----------------------------------------------------------- synthesis ----

def _freqs(ctx, q, n_sets, K, L0=25.0, ap=None, fmin=1e-3, fmax=1e2, index=0):
    s = q.logpolar_sampler(fmin, fmax, index=index)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(0.1, L0), fx, fy, area, None if ap is None else q.Aperture(*ap))
    return fx, fy, w


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("R,R_block", [(300, 300), (300, 97), (40, 1), (133, 64)])
def test_synthesize_parity(q, ctx, precision, R, R_block):
    K, P = 301, 150
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K)
    rng = np.random.default_rng(R + R_block)
    px, py = rng.uniform(-1.5, 1.5, P), rng.uniform(-1.5, 1.5, P)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block,
                               rng=q.Rng(11, 1000, 0), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=11,
                            counter=1000)
    report(f"synth p{precision} R{R} Rb{R_block}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_synthesize_phase_workload(q, ctx, precision):
    """The 32x32-point, K = 1024, R = 128 phase workload, whole output."""
    cfg = workloads.phase_fp64()
    K, R = cfg["K"], cfg["R"]
    for R_block in (R, 1):
        n_sets = math.ceil(R / R_block)
        fx, fy, w = _freqs(ctx, q, n_sets, K, L0=cfg["L0"])
        out = ctx.synthesize_phase(K, fx, fy, w, dev(cfg["px"]), dev(cfg["py"]), R, R_block,
                                   rng=q.Rng(cfg["seed"], 0, 0), precision=precision)
        ref = oracle.synthesize(host(fx), host(fy), host(w), cfg["px"], cfg["py"], R, R_block,
                                K=K, seed=cfg["seed"])
        report(f"phase workload p{precision} Rb{R_block}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_synthesize_given_coefficients(q, ctx, precision):
    K, P, R, R_block = 70, 45, 90, 33
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K)
    rng = np.random.default_rng(4)
    coef = rng.normal(size=(R, 2 * K))
    px, py = rng.uniform(-1, 1, P), rng.uniform(-1, 1, P)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block, coef=dev(coef),
                               precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, coef=coef)
    report(f"given coef p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", [0, 1, 3, 4])
def test_synthesize_eq3_mode(q, ctx, precision):
    K, P, R = 123, 37, 70
    fx, fy, w = _freqs(ctx, q, 1, K)
    rng = np.random.default_rng(8)
    px, py = rng.uniform(-1, 1, P), rng.uniform(-1, 1, P)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R,
                               rng=q.Rng(5, 3, q.COEF_EQ3), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R, K=K, seed=5, counter=3,
                            mode=1)
    report(f"eq3 p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
def test_synthesize_degenerate_sizes(q, ctx, precision):
    for K, P, R in ((1, 1, 1), (1, 33, 2), (17, 1, 65)):
        fx, fy, w = _freqs(ctx, q, R, K)
        px, py = np.array([0.3] * P), np.linspace(-1, 1, P)
        out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, 1,
                                   rng=q.Rng(1, 0, 0), precision=precision)
        ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, 1, K=K, seed=1)
        report(f"degenerate K{K} P{P} R{R} p{precision}", host(out), ref, TOL[precision])


# -------------------------------------------------------------- piston ----

@pytest.mark.parametrize("precision", PRECS)
def test_piston_parity(q, ctx, precision):
    K, R, R_block = 257, 200, 64
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K)
    cx = np.array([0.0, 56.5, 10.0, -3.0, 120.0])
    cy = np.array([0.0, 0.0, 20.0, 4.0, -7.0])
    D = np.array([8.0, 8.0, 1.8, 1.8, 0.5])
    d = np.array([1.1, 1.1, 0.0, 0.3, 0.0])
    out = ctx.piston(K, fx, fy, w, dev(cx), dev(cy), dev(D), dev(d), R, R_block,
                     rng=q.Rng(2, 77, 0), precision=precision)
    ref = oracle.piston(host(fx), host(fy), host(w), cx, cy, D, d, R, R_block, K=K, seed=2,
                        counter=77)
    report(f"piston p{precision}", host(out), ref, TOL[precision])


# -------------------------------------------------- differential piston ----

@pytest.mark.parametrize("precision", PRECS)
def test_diff_piston_parity(q, ctx, precision):
    cfg = workloads.diffpiston()
    K, R, R_block = 333, 150, 70
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, ap=(cfg["D"], 0.0))
    out = ctx.diff_piston(K, fx, fy, w, dev(cfg["bx"]), dev(cfg["by"]), R, R_block,
                          rng=q.Rng(0, 5, 0), precision=precision)
    px = np.concatenate([[0.0], cfg["bx"]])
    py = np.concatenate([[0.0], cfg["by"]])
    pist = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=0,
                             counter=5)
    ref = pist[:, 1:] - pist[:, :1]
    report(f"diff piston p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("R,R_block", [(500, 500), (500, 64), (60, 1)])
def test_diff_piston_structure_parity(q, ctx, precision, R, R_block):
    cfg = workloads.diffpiston()
    K = 700
    n_sets = math.ceil(R / R_block)
    s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=1234)
    sf, se = ctx.diff_piston_structure(q.psd(0.1, 25.0), q.Aperture(cfg["D"], 0.0),
                                       dev(cfg["bx"]), dev(cfg["by"]), s, K, R, R_block,
                                       rng=q.Rng(9, 0, 0), precision=precision)
    assert s.index == 1234 + n_sets * K
    fx, fy, area = oracle.sample_logpolar(n_sets, K, cfg["fmin"], cfg["fmax"], index=1234)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0, D=cfg["D"])
    rsf, rse = oracle.diff_piston_sf(fx, fy, w, cfg["bx"], cfg["by"], R, R_block, K=K, seed=9)
    tol = {0: 1e-10, 1: 2e-5, 2: 2e-3, 3: 2e-5, 4: 2e-5}[precision]
    g, gs = host(sf), host(se)
    print(f"sf p{precision} R{R} Rb{R_block}: max rel {np.max(np.abs(g / rsf - 1)):.3e}")
    assert np.max(np.abs(g / rsf - 1)) < tol
    assert np.max(np.abs(gs / rse - 1)) < 20 * tol


def test_diff_piston_structure_deterministic(q, ctx):
    cfg = workloads.diffpiston()
    outs = []
    for _ in range(2):
        s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
        sf, _ = ctx.diff_piston_structure(q.psd(0.1, 25.0), q.Aperture(1.8, 0.0), dev(cfg["bx"]),
                                          dev(cfg["by"]), s, 2048, 3000, 256,
                                          rng=q.Rng(0, 0, 0), precision=1)
        outs.append(host(sf))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("R_block", [256, 1])
def test_diff_piston_structure_full_size(q, ctx, R_block):
    """The 1e5-realisation, K = 16384 differential-piston workload in the
    launch configuration the benchmark times (R_block = 256), and with fresh
    frequencies for every realisation (R_block = 1, the paper's usage: 1e5
    sets, 52 GB of frequency arrays on the device): (a) the fused
    structure-function sums equal the squares of the stored differential
    pistons; (b) sampled realisations of those pistons equal the oracle's;
    (c) the estimate agrees with the analytic curve within its statistical
    error."""
    from oracle import analytic as A
    cfg = workloads.diffpiston()
    K, R = cfg["K"], cfg["R"]
    n_sets = math.ceil(R / R_block)
    p = q.psd(cfg["r0"], 25.0)
    ap = q.Aperture(cfg["D"], 0.0)
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
    sf, se = ctx.diff_piston_structure(p, ap, bx, by, s, K, R, R_block, rng=q.Rng(0, 0, 0),
                                       precision=1)
    # same frequency sets and coefficients through the storing kernel
    s2 = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
    fx, fy, area = ctx.sample_frequencies(s2, n_sets, K)
    w = ctx.weights(p, fx, fy, area, ap)
    dp = ctx.diff_piston(K, fx, fy, w, bx, by, R, R_block, rng=q.Rng(0, 0, 0), precision=1)
    dph = host(dp)
    mean_sq = np.mean(dph * dph, axis=0)
    assert np.max(np.abs(host(sf) / mean_sq - 1)) < 1e-6
    # sampled realisations against the oracle (their sets copied to the host)
    for r in (0, 255, 256, 54321, R - 1):
        sidx = r // R_block
        sl = slice(sidx * K, (sidx + 1) * K)
        px = np.concatenate([[0.0], cfg["bx"]])
        py = np.concatenate([[0.0], cfg["by"]])
        pist = oracle.synthesize(host(fx[sl]), host(fy[sl]), host(w[sl]), px, py, 1, 1, K=K,
                                 seed=0, counter=r)
        ref = pist[0, 1:] - pist[0, 0]
        e = np.max(np.abs(dph[r] - ref)) / math.sqrt(np.mean(ref * ref))
        print(f"row {r}: eps_max {e:.3e}")
        assert e < 1e-5
    # statistics: agreement with the band-limited analytic curve
    an = A.sf_band(cfg["bx"], cfg["r0"], 25.0, cfg["fmin"], cfg["fmax"], D=cfg["D"])
    z = (host(sf) - an) / host(se)
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)


@pytest.mark.parametrize("precision", [3, 4])
def test_diff_piston_structure_sets_full_size(q, ctx, precision):
    """The benchmark's own launch sequence at full size: 1e5 realisations,
    K = 16384, 32 baselines, R_block = 256, BF16x6 and FP16x3, the frequency
    sets and weights drawn in one pass and the sums taken from those sets.
    (a) The fused structure-function sums equal the mean squares of the
    stored differential pistons of the same sets and coefficients; (b) 16
    sampled realisations of those pistons equal the oracle's within the
    FP32-class tolerance; (c) the structure function of two-set subsets (512
    realisations at the start, the middle and the end, the same sets and
    coefficient counters) equals the oracle's baseline by baseline; (d) the
    estimate agrees with the analytic curve within its statistical error."""
    from oracle import analytic as A
    cfg = workloads.diffpiston()
    K, R, R_block = cfg["K"], cfg["R"], 256
    n_sets = math.ceil(R / R_block)
    p = q.psd(cfg["r0"], 25.0)
    ap = q.Aperture(cfg["D"], 0.0)
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
    fx, fy, w = ctx.sample_weights(s, n_sets, K, p, ap)
    assert s.index == n_sets * K
    rng = q.Rng(0, 0, q.COEF_GAUSS_CS)
    sf, se = ctx.diff_piston_structure_sets(K, fx, fy, w, bx, by, R, R_block, rng=rng,
                                            precision=precision)
    dp = ctx.diff_piston(K, fx, fy, w, bx, by, R, R_block, rng=rng, precision=precision)
    dph = host(dp)
    mean_sq = np.mean(dph * dph, axis=0)
    assert np.max(np.abs(host(sf) / mean_sq - 1)) < 1e-6
    px = np.concatenate([[0.0], cfg["bx"]])
    py = np.concatenate([[0.0], cfg["by"]])
    rows = [0, 255, 256, R - 1] + list(np.random.default_rng(precision).integers(0, R, 12))
    for r in rows:
        sl = slice((r // R_block) * K, (r // R_block + 1) * K)
        pist = oracle.synthesize(host(fx[sl]), host(fy[sl]), host(w[sl]), px, py, 1, 1, K=K,
                                 seed=0, counter=int(r))
        ref = pist[0, 1:] - pist[0, 0]
        e = np.max(np.abs(dph[r] - ref)) / math.sqrt(np.mean(ref * ref))
        print(f"row {r}: eps_max {e:.3e}")
        assert e < TOL[precision]
    for s0 in (0, n_sets // 2, n_sets - 3):
        sl = slice(s0 * K, (s0 + 2) * K)
        sub, _ = ctx.diff_piston_structure_sets(K, fx[sl], fy[sl], w[sl], bx, by, 2 * R_block,
                                                R_block, rng=q.Rng(0, s0 * R_block, 0),
                                                precision=precision)
        ref, _ = oracle.diff_piston_sf(host(fx[sl]), host(fy[sl]), host(w[sl]), cfg["bx"],
                                       cfg["by"], 2 * R_block, R_block, K=K, seed=0,
                                       counter=s0 * R_block)
        e = np.max(np.abs(host(sub) / ref - 1))
        print(f"sets {s0}, {s0 + 1}: structure function max rel {e:.3e}")
        assert e < 2e-5
    an = A.sf_band(cfg["bx"], cfg["r0"], 25.0, cfg["fmin"], cfg["fmax"], D=cfg["D"])
    z = (host(sf) - an) / host(se)
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)


# -------------------------------------------------------------- errors ----

def test_invalid_arguments_raise(q, ctx):
    fx = dev(np.zeros(10))
    with pytest.raises(q.QrfsError) as e:
        ctx.synthesize_phase(10, fx, fx, fx, fx, fx, 5, 6)  # R_block > R
    assert e.value.status == q.ERR_INVALID_ARG
    with pytest.raises(q.QrfsError) as e:
        ctx.weights(q.psd(-0.1, 25.0), fx, fx, fx)
    assert e.value.status == q.ERR_INVALID_ARG
    with pytest.raises(q.QrfsError) as e:
        ctx.sample_frequencies(q.logpolar_sampler(1.0, 0.5), 1, 10)
    assert e.value.status == q.ERR_INVALID_ARG
    s = q.logpolar_sampler(1e-3, 1e2)
    s.scheme = q.SAMPLER_LEARNED  # no proposal attached
    with pytest.raises(q.QrfsError) as e:
        ctx.sample_frequencies(s, 1, 10)
    assert e.value.status == q.ERR_INVALID_ARG


@pytest.mark.parametrize("scheme", ["cartesian", "disc", "jitter", "random_logpolar",
                                    "random_cartesian", "random_disc"])
def test_end_to_end_sampler_and_weights_equal_separate_calls(q, ctx, scheme):
    """The end-to-end structure function draws frequencies and weights in one
    fused kernel; with the same sets drawn by qrfs_sample_frequencies and
    weighted by qrfs_weights, the set-level entry gives bit-identical
    results, for every sampler the fused kernel serves."""
    cfg = workloads.diffpiston()
    N, df = 44, 0.25 / 22
    K, R, R_block = N * N, 300, 64
    n_sets = math.ceil(R / R_block)
    make = {
        "cartesian": lambda: q.cartesian_sampler(N, df, index=11),
        "disc": lambda: q.disc_sampler(0.25, index=11),
        "jitter": lambda: q.jitter_sampler(N, df, index=11),
        "random_logpolar": lambda: q.random_sampler(q.SAMPLER_RANDOM_LOGPOLAR, fmin=1e-3,
                                                    fmax=1e2, index=11),
        "random_cartesian": lambda: q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df,
                                                     index=11),
        "random_disc": lambda: q.random_sampler(q.SAMPLER_RANDOM_DISC, fmax=0.25, index=11),
    }[scheme]
    p, ap = q.psd(0.1, 22.0), q.Aperture(8.0, 1.1)
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    sf, se = ctx.diff_piston_structure(p, ap, bx, by, make(), K, R, R_block,
                                       rng=q.Rng(5, 2, 0), precision=1)
    fx, fy, area = ctx.sample_frequencies(make(), n_sets, K)
    w = ctx.weights(p, fx, fy, area, ap)
    sf2, se2 = ctx.diff_piston_structure_sets(K, fx, fy, w, bx, by, R, R_block,
                                              rng=q.Rng(5, 2, 0), precision=1)
    assert torch.equal(sf, sf2) and torch.equal(se, se2)


@pytest.mark.parametrize("precision", PRECS)
def test_diff_piston_structure_sets_equals_end_to_end(q, ctx, precision):
    """The set-level entry gives bit-identical results to the end-to-end one
    when handed the same frequency sets."""
    cfg = workloads.diffpiston()
    K, R, R_block = 1000, 700, 128
    n_sets = math.ceil(R / R_block)
    p, ap = q.psd(0.1, 10.0), q.Aperture(cfg["D"], 0.0)
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=77)
    sf, se = ctx.diff_piston_structure(p, ap, bx, by, s, K, R, R_block, rng=q.Rng(3, 9, 0),
                                       precision=precision)
    s2 = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=77)
    fx, fy, area = ctx.sample_frequencies(s2, n_sets, K)
    w = ctx.weights(p, fx, fy, area, ap)
    sf2, se2 = ctx.diff_piston_structure_sets(K, fx, fy, w, bx, by, R, R_block,
                                              rng=q.Rng(3, 9, 0), precision=precision)
    assert torch.equal(sf, sf2) and torch.equal(se, se2)
