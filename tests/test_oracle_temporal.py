"""Pins of the temporal (frozen-flow) differential-piston structure function
of the worked example (Sec. 4.4): the oracle's estimator, its noise-free
expectation, and the analytic curve, each against something other than
itself."""
import math

import numpy as np

import oracle
from oracle import analytic as A


def test_estimator_brute_force():
    rng = np.random.default_rng(3)
    R, M = 4, 9
    p = rng.normal(size=(R, 2, M))
    sf, se = oracle.temporal_sf(p)
    dp = p[:, 0, :] - p[:, 1, :]
    per = np.zeros((R, M))
    for r in range(R):
        for j in range(1, M):
            per[r, j] = np.mean([(dp[r, m + j] - dp[r, m]) ** 2 for m in range(M - j)])
    assert np.allclose(sf, per.mean(0), rtol=1e-14, atol=0)
    assert np.allclose(se, per.std(0, ddof=1) / math.sqrt(R), rtol=1e-12, atol=1e-300)
    assert sf[0] == 0.0


def _cartesian_set(K_side, seed_index=0):
    N, df = K_side, 0.25 / 22 * 44 / K_side
    fx, fy, area = oracle.sample_cartesian(1, N * N, N, df, index=seed_index)
    return fx, fy, area


def test_noise_free_expectation():
    """Given one frequency set, the coefficients make dp(t + tau) - dp(t)
    exactly normal with variance S(tau) = sum_k w_k^2 16 sin^2(pi f.B)
    sin^2(pi f.v tau) (every pair, so also its time average): the estimate
    over many realisations agrees with S within its standard error."""
    fx, fy, area = _cartesian_set(12, seed_index=77)
    w = oracle.weights(fx, fy, area, r0=0.1, L0=22.0, D=8.0, d=1.1)
    c1, c2, v = (0.0, 0.0), (56.5, 0.0), (10.2, 3.0)
    dt, M, R = 0.05, 24, 6000
    sf, se = oracle.temporal_experiment(fx, fy, w, c1, c2, v, dt, M, R, R, seed=5)
    B = np.subtract(c1, c2)
    tau = np.arange(M) * dt
    S = np.array([np.sum(w ** 2 * 16.0 * np.sin(np.pi * (fx * B[0] + fy * B[1])) ** 2
                         * np.sin(np.pi * (fx * v[0] + fy * v[1]) * t) ** 2) for t in tau])
    z = (sf[1:] - S[1:]) / se[1:]
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 5.0)
    assert sf[0] == 0.0 and S[0] == 0.0


def test_analytic_covariance_form_matches_square_quadrature():
    """The four-covariance form (1-D Bessel integrals of the piston
    covariance) equals the 2-D integral of W F^2 16 sin^2 sin^2 over a square
    wide enough that the aperture filter has cut the PSD off."""
    B, v = (10.0, 0.0), (10.2, 4.0)
    tau = np.array([0.02, 0.3, 1.0, 4.0])
    iso = A.temporal_sf(tau, B, v, r0=0.1, L0=22.0, D=8.0, d=1.1)
    sq = A.temporal_sf_square(tau, B, v, r0=0.1, L0=22.0, D=8.0, d=1.1, half_width=1.5, n=300)
    print(iso, sq)
    assert np.allclose(sq, iso, rtol=2e-3)


def test_analytic_limits():
    """D(0) = 0, and for lags long enough that the screen has moved far past
    both apertures, D -> 4 (C(0) - C(B)) = twice the spatial differential-
    piston structure function at B."""
    B, v = (56.5, 0.0), (10.2, 0.0)
    D0, Dlong = A.temporal_sf([0.0, 600.0], B, v, r0=0.1, L0=22.0, D=8.0, d=1.1)
    two_dp = 2.0 * A.diff_piston_sf(56.5, 0.1, 22.0, 8.0, d=1.1)[0]
    assert abs(D0) < 1e-9 * two_dp
    assert abs(Dlong / two_dp - 1.0) < 2e-3
