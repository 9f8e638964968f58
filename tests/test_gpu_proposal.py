"""Learned proposal on the GPU against the FP64 oracle, and what it gains.

Parity (seeded parameters, never trained ones, feed both sides):
  network forward          FP32 vs FP64, 1e-5 of the output scale
  loss and gradient        1e-5 (loss), 1e-5 normwise (gradient)
  training rows            ell, theta to 1e-14, h to 1e-12
  sampling table           p to 1e-5 relative, alpha to 2e-5
  learned sampler          the oracle's table fed to both sides: 1e-12
  structure function       learned sampler end to end, FP32-class
Gain: after training, the per-set error of the conditional expectation
sum_k w_k^2 2(1 - cos 2 pi f_k.B) against the band-limited analytic curve
is smaller with the learned K = 4096 sets than with plain K = 4096 sets.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
import workloads

pytestmark = pytest.mark.gpu

FMIN, FMAX = workloads.FMIN, workloads.FMAX
LMIN, LW = math.log(FMIN), math.log(FMAX / FMIN)


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


def steep_params(H=128, slope=4.0, tilt=1.5, seed=11):
    rng = np.random.default_rng(seed)
    prm = workloads.mlp_init(seed, H=H, scale=1.0) * 0.3
    prm[0] += 1.5
    prm[6 * H] += 1.5
    o = 6 * H + H * H + H
    prm[o] += slope
    prm[o + H] += tilt
    return prm + rng.normal(0, 1e-3, prm.size)


def test_forward_parity(q, ctx):
    prm = steep_params()
    p = q.Proposal(ctx, FMIN, FMAX, prm.astype(np.float32))
    rng = np.random.default_rng(1)
    n = 1000
    ell = rng.uniform(LMIN, LMIN + LW, n)
    ctx4 = np.stack([rng.uniform(0.5, 10, n), rng.uniform(10, 100, n), rng.uniform(1, 130, n),
                     rng.uniform(0, np.pi, n)], 1)
    out = host(p.forward(dev(ell), dev(ctx4)))
    ref = oracle.mlp_forward(prm.astype(np.float32).astype(np.float64), ell, ctx4, LMIN, LW)
    scale = np.max(np.abs(ref))
    print("forward max err / scale", np.max(np.abs(out - ref)) / scale)
    assert np.max(np.abs(out - ref)) / scale < 1e-5
    p.close()


def test_rows_parity(q, ctx):
    p = q.Proposal(ctx, FMIN, FMAX, np.zeros(q.PROPOSAL_NPARAM, dtype=np.float32))
    c4 = workloads.proposal_contexts(6, seed=3)
    s = q.logpolar_sampler(FMIN, FMAX, index=500)
    ell, theta, h = p.rows(s, dev(c4), 777, 0.1)
    assert s.index == 500 + 6 * 777
    rl, rt, rh = oracle.proposal_rows(c4, 777, 0.1, FMIN, FMAX, index=500)
    assert np.max(np.abs(host(ell) - rl)) < 1e-13
    assert np.max(np.abs(host(theta) - rt)) < 1e-13
    gh = host(h)
    assert np.max(np.abs(gh - rh)) <= 1e-11 * np.max(np.abs(rh))
    p.close()


@pytest.mark.parametrize("G", [64, 100])
def test_loss_gradient_parity(q, ctx, G):
    prm = steep_params(seed=5)
    p = q.Proposal(ctx, FMIN, FMAX, prm.astype(np.float32))
    c4 = workloads.proposal_contexts(5, seed=4)
    ell, theta, h = oracle.proposal_rows(c4, 300, 0.1, FMIN, FMAX, index=9)
    loss, grad = p.loss_grad(dev(c4), dev(ell), dev(theta), dev(h), G=G)
    rl, rg = oracle.mlp_loss_grad(prm.astype(np.float32).astype(np.float64), c4, ell, theta, h,
                                  LMIN, LW, G=G)
    g = host(grad)
    e = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"loss {loss:.8f} vs {rl:.8f}; gradient normwise rel err {e:.2e}")
    assert loss == pytest.approx(rl, rel=1e-5, abs=1e-6)
    assert e < 1e-5
    p.close()


def test_table_parity(q, ctx):
    prm = steep_params(seed=7)
    p = q.Proposal(ctx, FMIN, FMAX, prm.astype(np.float32))
    bl = np.logspace(0, np.log10(130), 9)
    bth = np.linspace(0.0, 2.5, 9)
    p.tabulate(3.0, 40.0, bl, bth, n_cells=200, beta=0.2)
    tp, ta, tphi, tcdf = (host(x) for x in p.get_table())
    rp, ra, rphi, rcdf = oracle.proposal_table(prm.astype(np.float32).astype(np.float64), 3.0,
                                               40.0, bl, bth, FMIN, FMAX, n_cells=200, beta=0.2)
    assert np.max(np.abs(tp / rp - 1)) < 1e-5
    assert np.max(np.abs(ta - ra)) < 2e-5
    assert np.max(np.abs(tcdf - rcdf)) < 1e-5
    big = ra > 0.05
    assert np.max(np.abs(np.angle(np.exp(2j * (tphi[big] - rphi[big]))))) < 1e-3
    p.close()


def _oracle_table(seed=7, n_cells=256):
    bx, _ = workloads.baselines()
    return oracle.proposal_table(steep_params(seed=seed), 1.8, 25.0, bx, np.zeros(bx.size), FMIN,
                                 FMAX, n_cells=n_cells)


def test_learned_sampler_parity(q, ctx):
    tab = _oracle_table()
    p = q.Proposal(ctx, FMIN, FMAX, np.zeros(q.PROPOSAL_NPARAM, dtype=np.float32))
    p.set_table(*[dev(x) for x in tab])
    s = q.learned_sampler(p, index=321)
    fx, fy, area = ctx.sample_frequencies(s, 3, 1001)
    assert s.index == 321 + 3 * 1001
    rx, ry, ra = oracle.sample_learned(tab, 3, 1001, FMIN, FMAX, index=321)
    f = np.hypot(rx, ry)
    assert np.max(np.abs(host(fx) - rx) / f) < 1e-12
    assert np.max(np.abs(host(fy) - ry) / f) < 1e-12
    assert np.max(np.abs(host(area) / ra - 1)) < 1e-12
    p.close()


def test_learned_sample_weights_equal_two_calls(q, ctx):
    """The learned sampler through qrfs_sample_weights (cell areas in the
    context's workspace) gives the values of the two separate calls."""
    tab = _oracle_table()
    p = q.Proposal(ctx, FMIN, FMAX, np.zeros(q.PROPOSAL_NPARAM, dtype=np.float32))
    p.set_table(*[dev(x) for x in tab])
    psd, ap = q.psd(0.1, 25.0), q.Aperture(1.8, 0.0)
    fx, fy, w = ctx.sample_weights(q.learned_sampler(p, index=5), 2, 777, psd, ap)
    fx2, fy2, area = ctx.sample_frequencies(q.learned_sampler(p, index=5), 2, 777)
    w2 = ctx.weights(psd, fx2, fy2, area, ap)
    torch.cuda.synchronize()
    assert torch.equal(fx, fx2) and torch.equal(fy, fy2) and torch.equal(w, w2)
    p.close()


@pytest.mark.parametrize("precision", [0, 3])
def test_learned_structure_function_parity(q, ctx, precision):
    cfg = workloads.diffpiston()
    tab = _oracle_table()
    p = q.Proposal(ctx, FMIN, FMAX, np.zeros(q.PROPOSAL_NPARAM, dtype=np.float32))
    p.set_table(*[dev(x) for x in tab])
    K, R, R_block = 512, 400, 100
    s = q.learned_sampler(p, index=42)
    sf, se = ctx.diff_piston_structure(q.psd(0.1, 25.0), q.Aperture(cfg["D"], 0.0),
                                       dev(cfg["bx"]), dev(cfg["by"]), s, K, R, R_block,
                                       rng=q.Rng(4, 0, 0), precision=precision)
    fx, fy, area = oracle.sample_learned(tab, 4, K, FMIN, FMAX, index=42)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0, D=cfg["D"])
    rsf, _ = oracle.diff_piston_sf(fx, fy, w, cfg["bx"], cfg["by"], R, R_block, K=K, seed=4)
    err = np.max(np.abs(host(sf) / rsf - 1))
    print(f"learned SF p{precision}: max rel err {err:.2e}")
    assert err < (1e-10 if precision == 0 else 2e-5)
    p.close()


def _per_set_error(ctx, q, sampler, n_sets, K, cfg, L0):
    fx, fy, area = ctx.sample_frequencies(sampler, n_sets, K)
    w = ctx.weights(q.psd(cfg["r0"], L0), fx, fy, area, q.Aperture(cfg["D"], 0.0))
    fx, fy, w = host(fx), host(fy), host(w)
    an = A.sf_band(cfg["bx"], cfg["r0"], L0, FMIN, FMAX, D=cfg["D"])
    errs = []
    for s in range(n_sets):
        sl = slice(s * K, (s + 1) * K)
        S = np.array([np.sum(w[sl] ** 2 * 2 * (1 - np.cos(2 * np.pi * fx[sl] * b)))
                      for b in cfg["bx"]])
        errs.append(np.sqrt(np.mean((S / an - 1) ** 2)))
    return float(np.mean(errs))


def test_training_gain(q, ctx, tmp_path):
    """Train on the plain method's contributions, then compare the per-set
    error of learned and plain frequency sets of equal size."""
    cfg = workloads.diffpiston()
    L0 = 25.0
    c4 = workloads.proposal_contexts(128, seed=0)
    prm0 = workloads.mlp_init(0)
    p = q.Proposal(ctx, FMIN, FMAX, prm0.astype(np.float32))
    plain = q.logpolar_sampler(FMIN, FMAX, index=10_000_000)
    ell, theta, h = p.rows(plain, dev(c4), 2048, cfg["r0"])
    log = host(p.train(dev(c4), ell, theta, h, steps=600, ctx_per_step=16, lr=2e-3, seed=1))
    first, last = np.mean(log[:20]), np.mean(log[-20:])
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert np.all(np.isfinite(log)) and last < first - 0.05
    # save / load round trip
    path = tmp_path / "proposal.bin"
    p.save(path)
    before = host(p.params())
    p.set_params(np.zeros(q.PROPOSAL_NPARAM, dtype=np.float32))
    p.load(path)
    assert np.array_equal(host(p.params()), before)
    # per-set error at equal K for the benchmark geometry
    p.tabulate(cfg["D"], L0, cfg["bx"], np.zeros(cfg["bx"].size))
    K, n_sets = 4096, 8
    e_learned = _per_set_error(ctx, q, q.learned_sampler(p, index=77), n_sets, K, cfg, L0)
    e_plain = _per_set_error(ctx, q, q.logpolar_sampler(FMIN, FMAX, index=77), n_sets, K, cfg, L0)
    print(f"per-set RMS error, K = {K}: plain {e_plain:.4%}, learned {e_learned:.4%}")
    assert e_learned < e_plain
    p.close()


def _block_sf(ctx, q, sampler, K, cfg, L0, R, block, precision):
    """One static frequency set (R_block = R) and the structure function of
    each block of `block` realisations (coefficient counters r = 0 .. R-1,
    the same for every sampler): [R / block][nB]."""
    fx, fy, w = ctx.sample_weights(sampler, 1, K, q.psd(cfg["r0"], L0),
                                   q.Aperture(cfg["D"], 0.0))
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    out = []
    for b in range(R // block):
        sf, _ = ctx.diff_piston_structure_sets(K, fx, fy, w, bx, by, block, block,
                                               rng=q.Rng(7, b * block, 0), precision=precision)
        out.append(sf)
    return torch.stack(out).cpu().numpy()


def test_learned_not_worse_at_99_percent(q, ctx):
    """The learned-proposal criterion on the learned-proposal workload (D = 1.8 m, 32
    baselines 1-130 m, L0 = 25 m, R = 1e5, one static set, FP16x3): the
    error E = RMS over the baselines of sf / band-limited curve - 1 of
    learned K = 4096 satisfies E_learned <= max(1 %, E_plain) against plain
    K = 65536, and is not worse at 99 % confidence: over 2000 bootstrap
    resamples of the 100 blocks of 1000 realisations (paired: the blocks
    share coefficient counters), the 1st percentile of E_learned - E_plain
    is <= 0.  Plain K = 4096 (equal K) is reported beside it: at R = 1e5
    the coefficient noise (0.45 % per baseline) spreads the bootstrap
    difference over several tenths of a per cent, so the equal-K gain is
    tested noise-free instead (test_training_gain)."""
    cfg = workloads.diffpiston()
    L0, R, block = 25.0, 100000, 1000
    c4 = workloads.proposal_contexts(256, seed=0)
    p = q.Proposal(ctx, FMIN, FMAX, workloads.mlp_init(0).astype(np.float32))
    ell, theta, h = p.rows(q.logpolar_sampler(FMIN, FMAX, index=10_000_000), dev(c4), 2048,
                           cfg["r0"])
    p.train(dev(c4), ell, theta, h, steps=1000, ctx_per_step=16, lr=2e-3, seed=1)
    p.tabulate(cfg["D"], L0, cfg["bx"], np.zeros(cfg["bx"].size))
    an = A.sf_band(cfg["bx"], cfg["r0"], L0, FMIN, FMAX, D=cfg["D"])
    prec = q.PREC_FP16X3
    learned = _block_sf(ctx, q, q.learned_sampler(p, index=5), 4096, cfg, L0, R, block, prec)
    plain64 = _block_sf(ctx, q, q.logpolar_sampler(FMIN, FMAX, index=5), 65536, cfg, L0, R,
                        block, prec)
    plain4 = _block_sf(ctx, q, q.logpolar_sampler(FMIN, FMAX, index=5), 4096, cfg, L0, R,
                       block, prec)
    p.close()

    def err(blocks):
        return np.sqrt(np.mean((blocks.mean(axis=-2) / an - 1.0) ** 2, axis=-1))

    idx = np.random.default_rng(0).integers(0, R // block, size=(2000, R // block))
    e_l, e_64, e_4 = err(learned), err(plain64), err(plain4)
    d64 = err(learned[idx]) - err(plain64[idx])
    d4 = err(learned[idx]) - err(plain4[idx])
    print(f"E: learned K=4096 {e_l:.3%}, plain K=65536 {e_64:.3%}, plain K=4096 {e_4:.3%}; "
          f"bootstrap 1st/99th percentiles of learned - plain65536 {np.percentile(d64, 1):.3%} / "
          f"{np.percentile(d64, 99):.3%}, of learned - plain4096 {np.percentile(d4, 1):.3%} / "
          f"{np.percentile(d4, 99):.3%}")
    assert e_l <= max(0.01, e_64)
    assert np.percentile(d64, 1) <= 0.0
