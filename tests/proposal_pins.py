"""Closed-form pins of the oracle's learned-proposal table and loss value.

Shared by ``test_oracle_proposal.py`` (which runs them on the oracle) and
``test_oracle_mutations.py`` (which runs them on copies of the oracle with a
planted mistake and expects them to fail).  Every expected value below comes
from a closed form, not from the oracle's own formulas:

  * "staircase" networks: hidden units with very steep first-layer weights
    saturate tanh to exactly +-1 in binary64 away from their thresholds, so
    the network output is a known piecewise-constant function of the
    features and the normaliser on a grid is a finite sum of known terms;
  * the mixture of two angular factors with equal shapes and equal alpha,
    by the sum-to-product identity
        cos 2(t - a) + cos 2(t - b) = 2 cos(a - b) cos 2(t - (a + b)/2);
  * the mixture as a function of the angle, sampled at many angles, against
    the per-baseline densities (the definition of a mixture), which does not
    go through the amplitude/phase form the table stores.

The density model is the one the sampler uses (a learned PSD-aware mapping
of the frequency samples, which the paper's closing section suggests):
q(ell, theta) = p(ell) (1 + alpha(ell) cos 2(theta - theta_B)) / (2 pi),
p proportional to exp(o0), alpha = 0.9 tanh(o1).
"""
import math

import numpy as np

import oracle
import workloads

FMIN, FMAX = workloads.FMIN, workloads.FMAX
LMIN, LW = math.log(FMIN), math.log(FMAX / FMIN)
H = 128
SHARP = 1e5   # tanh(SHARP * d) == +-1 exactly in binary64 for |d| > 1.91e-4
SAT = 40.0    # tanh(+-40) == +-1 exactly


def staircase(units, b0=0.0, b1=0.0):
    """Network parameters whose outputs are piecewise constant.

    units: list of (out, coeffs, thr, height): hidden unit i computes
    sign(sum_f coeffs[f] x_f - thr) (exactly +-1 away from the threshold)
    and adds height * that sign to output `out` (0: o0, 1: o1).
    """
    prm = np.zeros(oracle.mlp_param_count(H))
    W1 = prm[:5 * H].reshape(H, 5)
    b1v = prm[5 * H:6 * H]
    o = 6 * H
    W2 = prm[o:o + H * H].reshape(H, H)
    o += H * H + H
    W3 = prm[o:o + 2 * H].reshape(2, H)
    b3 = prm[o + 2 * H:]
    for i, (out, coeffs, thr, height) in enumerate(units):
        for f, cf in coeffs.items():
            W1[i, f] = SHARP * cf
        b1v[i] = -SHARP * thr
        W2[i, i] = SAT
        W3[out, i] = height
    b3[0], b3[1] = b0, b1
    return prm


def features(ell, D, L0, B, thB):
    return np.array([2 * (ell - LMIN) / LW - 1, 2 * thB / math.pi - 1, math.log(D) / 4,
                     math.log(L0) / 4 - 1, math.log(B) / 4 - 0.5])


def staircase_out(units, b0, b1, x):
    """Exact outputs (o0, o1) of `staircase(units, b0, b1)` at features x,
    asserting that x keeps clear of every threshold."""
    o = [b0, b1]
    for out, coeffs, thr, height in units:
        a = sum(cf * x[f] for f, cf in coeffs.items()) - thr
        assert abs(a) > 5e-4, "feature too close to a step"
        o[out] += height * (1.0 if a > 0 else -1.0)
    return o


def angular_factor(alpha, phi, th):
    return 1.0 + alpha * np.cos(2.0 * (th - phi))


# ---------------------------------------------------------------- table pins
def check_table_one_baseline():
    """One baseline: p = (1 - beta) exp(o0)/Z + beta/Lw with Z the cell sum,
    alpha = (1 - beta) (exp(o0)/Z) 0.9 tanh(o1) / p, angle = theta_B."""
    units = [(0, {0: 1.0}, -0.5, 1.0), (0, {0: 1.0}, 0.25, 0.5), (1, {0: 1.0}, 0.0, 0.4)]
    b0, b1 = 0.3, 0.7
    D, L0, B, thB, beta, n = 1.8, 25.0, 40.0, 0.4, 0.1, 64
    prm = staircase(units, b0, b1)
    p, al, ph, cdf = oracle.proposal_table(prm, D, L0, [B], [thB], FMIN, FMAX, n_cells=n,
                                           beta=beta)
    dl = LW / n
    mids = LMIN + (np.arange(n) + 0.5) * dl
    o = np.array([staircase_out(units, b0, b1, features(m, D, L0, B, thB)) for m in mids])
    e = np.exp(o[:, 0])
    pb = e / (e.sum() * dl)
    p_ref = (1 - beta) * pb + beta / LW
    a_ref = (1 - beta) * pb * 0.9 * np.tanh(o[:, 1]) / p_ref
    assert np.allclose(p, p_ref, rtol=1e-12, atol=0)
    th = np.linspace(0, 2 * np.pi, 13)[:, None]
    assert np.allclose(angular_factor(al, ph, th), angular_factor(a_ref, thB, th), rtol=0,
                       atol=1e-12)
    assert np.allclose(cdf, np.concatenate([[0.0], np.cumsum(p_ref * dl)[:-1]]), rtol=0,
                       atol=1e-13)


def check_table_two_baselines_equal_shape():
    """Two baselines, equal normalised shape and equal alpha = a: the mixture
    is p_bar (1 + a cos(t1 - t2) cos 2(theta - (t1 + t2)/2)); the long
    baseline carries an extra constant in o0 that only the per-baseline
    normaliser removes."""
    units = [(0, {0: 1.0}, -0.2, 1.25), (0, {4: 1.0}, 0.25, 1.5)]
    b0, b1 = -0.4, 0.8
    a = 0.9 * math.tanh(b1)
    D, L0, beta, n = 1.8, 25.0, 0.1, 50
    bl, bth = [5.0, 80.0], [0.2, 0.9]
    prm = staircase(units, b0, b1)
    p, al, ph, cdf = oracle.proposal_table(prm, D, L0, bl, bth, FMIN, FMAX, n_cells=n, beta=beta)
    dl = LW / n
    mids = LMIN + (np.arange(n) + 0.5) * dl
    o = np.array([staircase_out(units, b0, b1, features(m, D, L0, bl[0], bth[0]))
                  for m in mids])
    e = np.exp(o[:, 0])
    pbar = e / (e.sum() * dl)
    p_ref = (1 - beta) * pbar + beta / LW
    amp = (1 - beta) * pbar * a * math.cos(bth[0] - bth[1]) / p_ref
    assert np.allclose(p, p_ref, rtol=1e-12, atol=0)
    assert np.allclose(al, amp, rtol=1e-12, atol=0)
    assert np.allclose(np.mod(ph - 0.5 * (bth[0] + bth[1]) + np.pi / 2, np.pi) - np.pi / 2, 0.0,
                       atol=1e-12)


def check_table_mixture_function():
    """Baselines with different shapes, normalisers and alphas: the table's
    angular density sum_b p_b (1 + alpha_b cos 2(theta - theta_b)) / nB,
    mixed with beta of the plain density, as a function of theta."""
    # step in ell whose position moves with |B|: x0 + 2 x4 > 0.3
    units = [(0, {0: 1.0, 4: 2.0}, 0.3, 1.0), (0, {4: 1.0}, 0.1, 0.75),
             (1, {0: 1.0, 4: -1.0}, -0.1, 0.6), (1, {1: 1.0}, 0.0, 0.3)]
    b0, b1 = 0.1, 0.2
    D, L0, beta, n = 3.0, 40.0, 0.25, 40
    bl = np.array([2.0, 11.0, 60.0])
    bth = np.array([0.15, 1.1, 2.6])
    prm = staircase(units, b0, b1)
    p, al, ph, cdf = oracle.proposal_table(prm, D, L0, bl, bth, FMIN, FMAX, n_cells=n, beta=beta)
    dl = LW / n
    mids = LMIN + (np.arange(n) + 0.5) * dl
    th = np.linspace(0, np.pi, 17)[:, None]
    mix = np.zeros((th.size, n))
    for B, tB in zip(bl, bth):
        o = np.array([staircase_out(units, b0, b1, features(m, D, L0, B, tB)) for m in mids])
        e = np.exp(o[:, 0])
        pb = e / (e.sum() * dl)
        mix += pb * angular_factor(0.9 * np.tanh(o[:, 1]), tB, th) / len(bl)
    ref = (1 - beta) * mix + beta / LW
    got = p * angular_factor(al, ph, th)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------- loss pins
def _rows(ctx, ells, thetas, hs):
    n_ctx = len(ctx)
    return (np.asarray(ctx, float).ravel(), np.tile(ells, n_ctx), np.tile(thetas, n_ctx),
            np.tile(hs, n_ctx))


def check_loss_constant_network():
    """A network with constant o0 and o1 = 0 is the plain density 1/Lw in
    ell: the cross-entropy (without the constant ln 2 pi of the angle) is
    ln Lw for any rows, and its gradient with respect to b3[0] vanishes."""
    prm = staircase([], b0=1.7, b1=0.0)
    rng = np.random.default_rng(11)
    ctx = [[1.8, 25.0, 7.0, 0.3], [8.0, 60.0, 100.0, 1.2]]
    ell = LMIN + LW * rng.random(37)
    c4, e, t, h = _rows(ctx, ell, 2 * np.pi * rng.random(37), rng.random(37) + 0.1)
    for G in (16, 64, 100):
        loss, grad = oracle.mlp_loss_grad(prm, c4, e, t, h, LMIN, LW, G=G)
        assert abs(loss - math.log(LW)) < 1e-13
        assert abs(grad[-2]) < 1e-13


def check_loss_step_network():
    """o0 piecewise constant in ell (levels known exactly), o1 = 0: the
    normaliser is the G-point midpoint sum (Lw/G) sum_j exp(o0(ell_j)), so
    the loss is -sum_i h_i (o0(ell_i) - log Z_c(i)) / sum_i h_i in closed
    form; the long-baseline context has its step elsewhere."""
    units = [(0, {0: 1.0, 4: 1.5}, 0.2, 1.5), (0, {0: 1.0}, -0.6, -0.75)]
    b0 = 0.25
    prm = staircase(units, b0, 0.0)
    ctx = [[1.8, 25.0, 3.0, 0.0], [1.8, 25.0, 90.0, 0.0]]
    rng = np.random.default_rng(5)
    m = 41
    ell = LMIN + LW * rng.random(m)
    th = 2 * np.pi * rng.random(m)
    h = rng.random(m) + 0.05
    c4, e, t, hh = _rows(ctx, ell, th, h)
    for G in (32, 100):
        loss, _ = oracle.mlp_loss_grad(prm, c4, e, t, hh, LMIN, LW, G=G)
        grid = LMIN + (np.arange(G) + 0.5) * LW / G
        tot, Htot = 0.0, 2 * h.sum()
        for cc in ctx:
            lev = lambda l: staircase_out(units, b0, 0.0, features(l, *cc))[0]  # noqa: E731
            Z = LW / G * sum(math.exp(lev(g)) for g in grid)
            tot += sum(hi * (lev(li) - math.log(Z)) for li, hi in zip(ell, h))
        assert abs(loss - (-tot / Htot)) < 1e-12


def check_loss_angular_term():
    """Constant o0, alpha = 0.9 tanh(o1) constant: rows along the baseline
    (theta - theta_B = 0 or pi) have angular factor 1 + alpha, rows across
    it (pi/2) 1 - alpha, rows at pi/4 exactly 1, so the loss is
    ln Lw - (h_along ln(1 + alpha) + h_across ln(1 - alpha)) / sum h."""
    b1 = 0.55
    alpha = 0.9 * math.tanh(b1)
    prm = staircase([], b0=-0.3, b1=b1)
    thB = 0.35
    ctx = [[1.8, 25.0, 30.0, thB]]
    rng = np.random.default_rng(2)
    offs = np.array([0.0, np.pi, np.pi / 2, -np.pi / 2, np.pi / 4, 3 * np.pi / 4] * 5)
    h = rng.random(offs.size) + 0.1
    ell = LMIN + LW * rng.random(offs.size)
    c4, e, t, hh = _rows(ctx, ell, thB + offs, h)
    loss, _ = oracle.mlp_loss_grad(prm, c4, e, t, hh, LMIN, LW, G=64)
    along = np.isclose(np.cos(2 * offs), 1.0)
    across = np.isclose(np.cos(2 * offs), -1.0)
    ref = math.log(LW) - (h[along].sum() * math.log1p(alpha) +
                          h[across].sum() * math.log1p(-alpha)) / h.sum()
    assert abs(loss - ref) < 1e-12


TABLE_PINS = [check_table_one_baseline, check_table_two_baselines_equal_shape,
              check_table_mixture_function]
LOSS_PINS = [check_loss_constant_network, check_loss_step_network, check_loss_angular_term]
