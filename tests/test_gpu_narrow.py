"""Sets of at most 8 realisations (the narrow kernels, one point per thread)
against the FP64 oracle: R_block 2, 3, 5, 8 (the 2-, 4- and 8-row kernels,
with idle rows and a ragged last set), K ragged against the 64-frequency
chunk, point counts that pick 64-, 128- and 256-thread blocks, every basis
(phase, piston, G-tilt, differential piston), every coefficient source.

Tolerances as the other parity tests: max error relative to the RMS of the
oracle output, 1e-11 (FP64), 1e-5 (FP32 class: sets this narrow are summed
in FP32 for every FP32-class precision).
"""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

TOL = {0: 1e-11, 1: 1e-5, 2: 1e-5, 3: 1e-5, 4: 1e-5}


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


def report(name, got, ref, tol):
    d = got - ref
    rms = math.sqrt(np.mean(ref * ref))
    e = np.max(np.abs(d)) / rms
    print(f"{name}: eps_max={e:.3e} tol={tol:g}", flush=True)
    assert e <= tol, (name, e)


def _freqs(ctx, q, n_sets, K, index):
    s = q.logpolar_sampler(1e-3, 1e2, index=index)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area, None)
    return fx, fy, w


@pytest.mark.parametrize("precision", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("R_block", [2, 3, 5, 8])
@pytest.mark.parametrize("P", [37, 130, 300])
def test_narrow_phase(q, ctx, precision, R_block, P):
    K = 133
    R = 2 * R_block + 1  # the last set holds one realisation
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, index=P + R_block)
    rng = np.random.default_rng(P * 10 + R_block)
    px, py = rng.uniform(-3, 3, P), rng.uniform(-3, 3, P)
    print(f"narrow phase p{precision} Rb{R_block} P{P}", flush=True)
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block,
                               rng=q.Rng(7, 50, 0), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=7,
                            counter=50)
    report(f"narrow phase p{precision} Rb{R_block} P{P}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", [0, 1, 3, 4])
@pytest.mark.parametrize("R_block", [1, 4, 6])
def test_narrow_piston_and_tilt(q, ctx, precision, R_block):
    K, R = 150, 13
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, index=900 + R_block)
    rng = np.random.default_rng(R_block)
    n_ap = 70
    cx, cy = rng.uniform(-50, 50, n_ap), rng.uniform(-50, 50, n_ap)
    D = rng.choice([8.0, 1.8], n_ap)
    d = np.where(D > 3.0, 1.1, 0.0)
    args = (K, fx, fy, w, dev(cx), dev(cy), dev(D), dev(d))
    hargs = (host(fx), host(fy), host(w), cx, cy, D, d, R, R_block)
    print(f"narrow piston/tilt p{precision} Rb{R_block}", flush=True)
    pist = ctx.piston(*args, R, R_block, rng=q.Rng(3, 9, 0), precision=precision)
    ref = oracle.piston(*hargs, K=K, seed=3, counter=9)
    report(f"narrow piston p{precision} Rb{R_block}", host(pist), ref, TOL[precision])
    tilt = ctx.tilt(*args, (0.0, 1.0), R, R_block, rng=q.Rng(3, 9, 0), precision=precision)
    ref = oracle.tilt(*hargs, axis=1, K=K, seed=3, counter=9)
    report(f"narrow tilt p{precision} Rb{R_block}", host(tilt), ref, TOL[precision])


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_narrow_diff_piston(q, ctx, precision):
    K, R, R_block = 200, 17, 4
    n_sets = math.ceil(R / R_block)
    s = q.logpolar_sampler(1e-3, 1e2, index=77)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area, q.Aperture(1.8, 0.0))
    bx = 10.0 ** np.linspace(0, math.log10(130.0), 32)
    by = np.zeros(32)
    out = ctx.diff_piston(K, fx, fy, w, dev(bx), dev(by), R, R_block, rng=q.Rng(0, 3, 0),
                          precision=precision)
    px, py = np.concatenate([[0.0], bx]), np.concatenate([[0.0], by])
    pist = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=0,
                             counter=3)
    report(f"narrow diff p{precision}", host(out), pist[:, 1:] - pist[:, :1], TOL[precision])


@pytest.mark.parametrize("precision", [0, 1, 3])
def test_narrow_coefficient_sources(q, ctx, precision):
    """Caller-supplied coefficients and the literal Eq. 3 mode."""
    K, R, R_block, P = 90, 11, 3, 64
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, index=5)
    rng = np.random.default_rng(2)
    px, py = rng.uniform(-1, 1, P), rng.uniform(-1, 1, P)
    coef = rng.normal(size=(R, 2 * K))
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block, coef=dev(coef),
                               precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, coef=coef)
    report(f"narrow given coef p{precision}", host(out), ref, TOL[precision])
    out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R_block,
                               rng=q.Rng(5, 1, q.COEF_EQ3), precision=precision)
    ref = oracle.synthesize(host(fx), host(fy), host(w), px, py, R, R_block, K=K, seed=5,
                            counter=1, mode=1)
    report(f"narrow eq3 p{precision}", host(out), ref, TOL[precision])
