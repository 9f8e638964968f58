"""Pins of the oracle's learned-proposal functions.

  loss gradient        -- central finite differences of the loss itself
  forward              -- explicit numpy evaluation of the layer equations
  table                -- normalisation; a constant network gives the plain
                          (uniform in ln f and angle) density; closed forms
                          of one-baseline and two-baseline tables built from
                          networks with exactly known piecewise-constant
                          outputs, and the mixture as a function of angle
                          (tests/proposal_pins.py)
  loss value           -- ln Lw for a constant network; closed-form log Z of
                          a step network on the normaliser grid; the angular
                          term at angles where its factor is 1 +- alpha or 1
                          (tests/proposal_pins.py)
  learned sampler      -- reduces to the plain log-polar sampler for the
                          uniform table; with a trained-like table its 1/q
                          cell areas keep sum W dA unbiased (closed-form band
                          variance) and the density of the draws is q
  training rows        -- their mean integrand is the analytic band SF
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic as A
import proposal_pins as PP
import workloads

FMIN, FMAX = workloads.FMIN, workloads.FMAX
LMIN, LW = math.log(FMIN), math.log(FMAX / FMIN)


def test_loss_gradient_finite_differences():
    H = 8
    rng = np.random.default_rng(0)
    prm = workloads.mlp_init(1, H=H, scale=2.0) + rng.normal(0, 0.1, oracle.mlp_param_count(H))
    ctx = workloads.proposal_contexts(3, seed=2)
    ell, theta, h = oracle.proposal_rows(ctx, 20, 0.1, FMIN, FMAX)
    loss, grad = oracle.mlp_loss_grad(prm, ctx, ell, theta, h, LMIN, LW, G=16, H=H)
    assert np.isfinite(loss)
    eps = 1e-6
    idx = rng.choice(prm.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(prm)
        e[i] = eps
        lp, _ = oracle.mlp_loss_grad(prm + e, ctx, ell, theta, h, LMIN, LW, G=16, H=H)
        lm, _ = oracle.mlp_loss_grad(prm - e, ctx, ell, theta, h, LMIN, LW, G=16, H=H)
        fd = (lp - lm) / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_forward_layer_equations():
    H = 16
    prm = workloads.mlp_init(3, H=H, scale=1.5)
    ctx = np.array([1.8, 25.0, 40.0, 0.3])
    ell = np.linspace(LMIN, LMIN + LW, 7)
    out = oracle.mlp_forward(prm, ell, ctx, LMIN, LW, H=H)
    W1 = prm[:5 * H].reshape(H, 5); b1 = prm[5 * H:6 * H]
    o = 6 * H
    W2 = prm[o:o + H * H].reshape(H, H); b2 = prm[o + H * H:o + H * H + H]
    o += H * H + H
    W3 = prm[o:o + 2 * H].reshape(2, H); b3 = prm[o + 2 * H:]
    for i, l in enumerate(ell):
        x = np.array([2 * (l - LMIN) / LW - 1, 2 * ctx[3] / np.pi - 1, np.log(ctx[0]) / 4,
                      np.log(ctx[1]) / 4 - 1, np.log(ctx[2]) / 4 - 0.5])
        ref = W3 @ np.tanh(W2 @ np.tanh(W1 @ x + b1) + b2) + b3
        assert np.allclose(out[i], ref, rtol=1e-13, atol=1e-14)


def steep_params(H=128, slope=4.0, tilt=1.5):
    """A network whose log-density rises steeply with ln f (and whose angle
    factor changes with it): g ~ slope tanh(1.5 tanh(1.5 x0))."""
    prm = np.zeros(oracle.mlp_param_count(H))
    prm[0] = 1.5                      # W1[0][0]
    o = 6 * H
    prm[o] = 1.5                      # W2[0][0]
    o += H * H + H
    prm[o] = slope                    # W3[0][0]
    prm[o + H] = tilt                 # W3[1][0]
    return prm


def _uniform_params(H=128):
    prm = workloads.mlp_init(0, H=H)
    prm[-(2 * H + 2):] = 0.0  # output layer zero -> o = (0, 0): flat density, alpha = 0
    return prm


def test_table_normalised_and_uniform_limit():
    prm = workloads.mlp_init(5, scale=3.0)
    bx, _ = workloads.baselines()
    p, al, ph, cdf = oracle.proposal_table(prm, 1.8, 25.0, bx, np.zeros(bx.size), FMIN, FMAX)
    dl = LW / p.size
    assert np.sum(p) * dl == pytest.approx(1.0, rel=1e-12)
    assert np.all(p > 0) and np.all(np.abs(al) < 1) and cdf[0] == 0.0
    assert np.all(np.diff(cdf) > 0)
    p, al, ph, cdf = oracle.proposal_table(_uniform_params(), 1.8, 25.0, bx, np.zeros(bx.size),
                                           FMIN, FMAX)
    assert np.allclose(p, 1.0 / LW, rtol=1e-12) and np.allclose(al, 0.0, atol=1e-15)


def test_learned_sampler_reduces_to_plain():
    bx, _ = workloads.baselines()
    tab = oracle.proposal_table(_uniform_params(), 1.8, 25.0, bx, np.zeros(bx.size), FMIN, FMAX)
    fx, fy, area = oracle.sample_learned(tab, 2, 1000, FMIN, FMAX, index=77)
    rx, ry, ra = oracle.sample_logpolar(2, 1000, FMIN, FMAX, index=77)
    f = np.hypot(rx, ry)
    assert np.max(np.abs(fx - rx) / f) < 1e-12 and np.max(np.abs(fy - ry) / f) < 1e-12
    assert np.max(np.abs(area / ra - 1)) < 1e-11


def test_learned_sampler_unbiased_weights():
    """sum_k W(f_k) area_k estimates the band integral of W for any
    proposal (the areas are 1/(K q)); checked with a strongly non-uniform
    table against the closed-form band variance."""
    bx, _ = workloads.baselines()
    tab = oracle.proposal_table(steep_params(), 1.8, 25.0, bx, np.zeros(bx.size), FMIN, FMAX)
    assert np.max(tab[0]) / np.min(tab[0]) > 3.0 and np.max(np.abs(tab[1])) > 0.3
    K = 65536
    fx, fy, area = oracle.sample_learned(tab, 1, K, FMIN, FMAX)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0)
    exact = A.variance_truncated(0.1, 25.0, FMIN, FMAX)
    assert np.sum(w * w) == pytest.approx(exact, rel=5e-3)


def test_learned_sampler_density():
    """The draws have density q: the histogram of ln f follows p, the
    angles within a cell follow 1 + alpha cos 2(theta - phi)."""
    bth = np.linspace(0.1, 1.2, 5)
    tab = oracle.proposal_table(steep_params(), 3.0, 40.0, np.full(5, 20.0), bth, FMIN, FMAX,
                                n_cells=16)
    p, al, ph, cdf = tab
    n = 200000
    fx, fy, area = oracle.sample_learned(tab, 1, n, FMIN, FMAX)
    ell = np.log(np.hypot(fx, fy))
    cells = np.minimum(((ell - LMIN) / (LW / 16)).astype(int), 15)
    frac = np.bincount(cells, minlength=16) / n
    assert np.allclose(frac, p * LW / 16, atol=2e-3)
    j = int(np.argmax(np.abs(al)))
    th = np.mod(np.arctan2(fy, fx)[cells == j] - ph[j], np.pi)
    # E[cos 2 t] under (1 + a cos 2t)/(2 pi) is a/2
    assert np.mean(np.cos(2 * th)) == pytest.approx(al[j] / 2, abs=0.02)


def test_training_rows_integrand():
    """Mean of h over uniform (ln f, theta) times the box measure is the
    band-limited differential-piston structure function."""
    ctx = np.array([[1.8, 25.0, 10.0, 0.0], [1.8, 60.0, 80.0, 0.7]])
    m = 1 << 17
    ell, theta, h = oracle.proposal_rows(ctx, m, 0.1, FMIN, FMAX)
    for c in range(2):
        est = np.mean(h[c * m:(c + 1) * m]) * LW * 2 * np.pi
        an = A.sf_band([ctx[c, 2]], 0.1, ctx[c, 1], FMIN, FMAX, D=ctx[c, 0])[0]
        assert est == pytest.approx(an, rel=5e-3)


@pytest.mark.parametrize("pin", PP.TABLE_PINS, ids=lambda f: f.__name__)
def test_table_closed_forms(pin):
    pin()


@pytest.mark.parametrize("pin", PP.LOSS_PINS, ids=lambda f: f.__name__)
def test_loss_value_closed_forms(pin):
    pin()
