"""Pins of the angle-of-arrival measurable (aperture-averaged phase
gradient, G-tilt): the oracle's tilt against finite differences of its own
piston, its variance formula against the textbook Kolmogorov coefficient,
and its noise-free expectation per frequency set."""
import math

import numpy as np

import oracle
from oracle import analytic as A


def _set(K=300, index=5):
    fx, fy, area = oracle.sample_logpolar(1, K, 1e-3, 1e2, index=index)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0)
    return fx, fy, w


def test_tilt_is_gradient_of_piston():
    """d/dc of the piston of Eq. 3 (filter of Eq. 7) by central differences
    equals the tilt, for both axes and annular apertures."""
    fx, fy, w = _set()
    cx, cy = np.array([0.0, 3.0, -7.5]), np.array([0.0, 1.0, 20.0])
    D, d = np.array([8.0, 1.8, 4.0]), np.array([1.1, 0.0, 0.5])
    R, h = 5, 1e-4
    for axis, (ex, ey) in enumerate(((h, 0.0), (0.0, h))):
        t = oracle.tilt(fx, fy, w, cx, cy, D, d, R, R, axis=axis, seed=2)
        pp = oracle.piston(fx, fy, w, cx + ex, cy + ey, D, d, R, R, seed=2)
        pm = oracle.piston(fx, fy, w, cx - ex, cy - ey, D, d, R, R, seed=2)
        fd = (pp - pm) / (2 * h)
        err = np.max(np.abs(t - fd)) / math.sqrt(np.mean(t * t))
        print(axis, err)
        assert err < 1e-6


def test_tilt_variance_textbook_coefficient():
    """Kolmogorov G-tilt, one axis: (lambda/2 pi)^2 <t^2> = 0.170 (lambda/D)^2
    (D/r0)^(5/3), i.e. <t^2> D^2 / (4 pi^2 (D/r0)^(5/3)) = 0.170, for any D."""
    for D in (1.0, 8.0, 39.0):
        v = A.tilt_variance(0.1, 1e9, D, model=0)
        coef = v * D * D / (4 * math.pi ** 2) / (D / 0.1) ** (5.0 / 3.0)
        assert abs(coef - 0.170) < 1e-3, (D, coef)


def test_tilt_noise_free_expectation():
    """Given one frequency set, <t_x^2> over the coefficients is exactly
    sum_k w_k^2 F_k^2 (2 pi f_x,k)^2; the band-limited sum approaches the
    variance integral."""
    K = 2000
    fx, fy, area = oracle.sample_logpolar(1, K, 1e-3, 10.0, index=9)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0)
    D, d = 1.8, 0.0
    R = 20000
    t = oracle.tilt(fx, fy, w, [0.0], [0.0], [D], [d], R, R, axis=0, seed=4)[:, 0]
    F = oracle.aperture_filter(np.hypot(fx, fy), D, d)
    S = np.sum(w ** 2 * F ** 2 * (2 * math.pi * fx) ** 2)
    m = np.mean(t * t)
    se = np.std(t * t, ddof=1) / math.sqrt(R)
    print("z", (m - S) / se)
    assert abs(m - S) < 5 * se
    band = A.tilt_variance(0.1, 25.0, D, fmin=1e-3, fmax=10.0)
    assert abs(S / band - 1) < 0.02, S / band
