"""Angle of arrival (aperture-averaged phase gradient, G-tilt) through the C
ABI, against the FP64 oracle and the variance integral.

The oracle forms the gradient along the x and y axes; the gradient along
any u is u_x t_x + u_y t_y (linearity), formed here in FP64.  Tolerances as
for pistons: max error relative to the RMS of the oracle output, 1e-11
(FP64), 1e-5 (FP32, BF16x6), 1e-3 (split-BF16).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A

pytestmark = pytest.mark.gpu

TOL = {0: 1e-11, 1: 1e-5, 2: 1e-3, 3: 1e-5, 4: 1e-5}
DIRS = [(1.0, 0.0), (0.0, 1.0), (0.6, -0.8)]


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
    e_rms, e_max = math.sqrt(np.mean(d * d)) / rms, np.max(np.abs(d)) / rms
    print(f"{name}: eps_rms={e_rms:.3e} eps_max={e_max:.3e} tol={tol:g}", flush=True)
    assert e_max <= tol, (name, e_rms, e_max)


def _freqs(ctx, q, n_sets, K, index=0):
    s = q.logpolar_sampler(1e-3, 1e2, index=index)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area, None)
    return fx, fy, w


def _oracle_dir(u, fx, fy, w, cx, cy, D, d, R, R_block, K, seed, counter):
    out = 0.0
    for axis in (0, 1):
        if u[axis] != 0.0:
            out = out + u[axis] * oracle.tilt(fx, fy, w, cx, cy, D, d, R, R_block, axis=axis,
                                              K=K, seed=seed, counter=counter)
    return out


@pytest.mark.parametrize("precision", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("u", DIRS)
@pytest.mark.parametrize("R,R_block", [(200, 64), (37, 1)])
def test_tilt_parity_fused(q, ctx, precision, u, R, R_block):
    K = 257
    n_sets = math.ceil(R / R_block)
    fx, fy, w = _freqs(ctx, q, n_sets, K, index=R)
    cx = np.array([0.0, 56.5, 10.0, -3.0, 120.0])
    cy = np.array([0.0, 0.0, 20.0, 4.0, -7.0])
    D = np.array([8.0, 8.0, 1.8, 1.8, 0.5])
    d = np.array([1.1, 1.1, 0.0, 0.3, 0.0])
    print(f"tilt fused p{precision} u{u} R{R} Rb{R_block}", flush=True)
    out = ctx.tilt(K, fx, fy, w, dev(cx), dev(cy), dev(D), dev(d), u, R, R_block,
                   rng=q.Rng(2, 77, 0), precision=precision)
    ref = _oracle_dir(u, host(fx), host(fy), host(w), cx, cy, D, d, R, R_block, K, 2, 77)
    report(f"tilt p{precision}", host(out), ref, TOL[precision])


@pytest.mark.parametrize("precision", [1, 2, 3])
@pytest.mark.parametrize("u", [(1.0, 0.0), (0.6, -0.8)])
def test_tilt_parity_two_phase(q, precision, u):
    """Ragged apertures (300 = 256 + 44 columns), two sets of 150 rows."""
    c = q.Context(0)
    c.set_tuning(q.TUNE_WIDE_PATH, 2)
    try:
        K, R, R_block, n_ap = 203, 300, 150, 300
        fx, fy, w = _freqs(c, q, 2, K, index=99)
        rng = np.random.default_rng(5)
        cx, cy = rng.uniform(-60, 60, n_ap), rng.uniform(-60, 60, n_ap)
        D = rng.choice([8.0, 1.8, 4.0], n_ap)
        d = np.where(D > 3.0, 1.1, 0.0)
        print(f"tilt two-phase p{precision} u{u}", flush=True)
        out = c.tilt(K, fx, fy, w, dev(cx), dev(cy), dev(D), dev(d), u, R, R_block,
                     rng=q.Rng(9, 3, 0), precision=precision)
        ref = _oracle_dir(u, host(fx), host(fy), host(w), cx, cy, D, d, R, R_block, K, 9, 3)
        report(f"tilt two-phase p{precision}", host(out), ref, TOL[precision])
    finally:
        c.close()


def test_tilt_caller_coefficients(q, ctx):
    """Caller-supplied coefficients give the same result as drawing them."""
    K, R = 100, 16
    fx, fy, w = _freqs(ctx, q, 1, K, index=7)
    coef = dev(np.stack([oracle.coefficients(3, 40 + r, K) for r in range(R)]))
    cx, cy, D, d = (dev([0.0, 5.0]), dev([0.0, -2.0]), dev([1.8, 8.0]), dev([0.0, 1.1]))
    a = ctx.tilt(K, fx, fy, w, cx, cy, D, d, (0.0, 1.0), R, R, coef=coef, precision=0)
    b = ctx.tilt(K, fx, fy, w, cx, cy, D, d, (0.0, 1.0), R, R, rng=q.Rng(3, 40, 0), precision=0)
    assert np.allclose(host(a), host(b), rtol=1e-12, atol=1e-12 * np.abs(host(b)).max())


def test_tilt_variance_statistics(q, ctx):
    """Fresh log-polar frequency sets for every realisation: the mean square
    tilt along x agrees with the band-limited variance integral
    int W F^2 (2 pi f_x)^2 d^2f within its standard error."""
    K, R, D = 1000, 20000, 1.8
    fx, fy, w = _freqs(ctx, q, R, K, index=1)
    out = ctx.tilt(K, fx, fy, w, dev([0.0]), dev([0.0]), dev([D]), dev([0.0]), (1.0, 0.0), R, 1,
                   rng=q.Rng(11, 0, 0), precision=1)
    t2 = host(out)[:, 0] ** 2
    m, se = t2.mean(), t2.std(ddof=1) / math.sqrt(R)
    v = A.tilt_variance(0.1, 25.0, D, fmin=1e-3, fmax=1e2)
    print(f"<t^2> {m:.6e} +- {se:.2e}, integral {v:.6e}, z {(m - v) / se:.2f}")
    assert abs(m - v) < 4.5 * se
