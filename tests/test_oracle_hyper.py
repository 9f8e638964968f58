"""Pins of the sampling hyper-parameter tools of Secs. 3.2 and 4.3: the
square-to-disc (concentric) map for polar quasi-random frequencies, the disc
sampler, and the stopping rule that picks N."""
import math

import numpy as np

import oracle
from oracle import analytic as A


def test_concentric_map_points():
    """Centre, edge midpoints and corner of the square go to the centre, the
    axis points and the 45-degree point of the unit circle."""
    cases = {(0.5, 0.5): (0.0, 0.0), (1.0, 0.5): (1.0, 0.0), (0.0, 0.5): (-1.0, 0.0),
             (0.5, 1.0): (0.0, 1.0), (0.5, 0.0): (0.0, -1.0),
             (1.0, 1.0): (math.sqrt(0.5), math.sqrt(0.5)), (0.75, 0.5): (0.5, 0.0),
             (0.0, 0.0): (-math.sqrt(0.5), -math.sqrt(0.5))}
    for (ux, uy), (x, y) in cases.items():
        gx, gy = oracle.concentric_map(ux, uy)
        assert abs(gx - x) < 1e-15 and abs(gy - y) < 1e-15, (ux, uy, gx, gy)


def test_concentric_map_radius_and_area():
    """The radius is the concentric square's half-width max(|a|, |b|), and the
    map preserves area: on a fine grid of the square, the fraction of points
    inside radius rho is rho^2."""
    n = 400
    u = (np.arange(n) + 0.5) / n
    xs = np.empty((n, n))
    ys = np.empty((n, n))
    for i, ux in enumerate(u):
        for j, uy in enumerate(u):
            xs[i, j], ys[i, j] = oracle.concentric_map(ux, uy)
    a = 2 * u[:, None] - 1
    b = 2 * u[None, :] - 1
    r = np.hypot(xs, ys)
    assert np.max(np.abs(r - np.maximum(np.abs(a), np.abs(b)))) < 1e-14
    for rho in (0.2, 0.5, 0.9):
        frac = np.mean(r < rho)
        assert abs(frac - rho * rho) < 3.0 / n, (rho, frac)


def test_disc_sampler_variance():
    """Every point stands for pi fmax^2 / K, and the weighted sum of one set
    of K R2 points reproduces the closed-form variance of the phase PSD
    restricted to the disc (band of the worked example, where the von Karman
    peak near f = 0 spans a few hundred cells)."""
    K, fmax = 8192, 0.25
    fx, fy, area = oracle.sample_disc(1, K, fmax, index=10)
    assert np.all(np.hypot(fx, fy) < fmax)
    assert abs(np.sum(area) / (math.pi * fmax ** 2) - 1) < 1e-14
    w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0)
    exact = A.variance_truncated(0.1, 25.0, 0.0, fmax)
    rel = np.sum(w ** 2) / exact - 1
    print("disc variance rel err", rel)
    assert abs(rel) < 5e-3


def test_stopping_rule_closed_form():
    """Without an aperture the von Karman radial integral has a closed form,
    g(x) = (3/5) c r0^-5/3 (L0^(5/3) - (x^2 + L0^-2)^(-5/6)); N from the
    oracle's quadrature matches the rule applied to the closed form."""
    r0, L0 = 0.1, 22.0
    c = oracle.psd_constant()
    df = 0.25 / L0
    k = 0.6 * c * r0 ** (-5.0 / 3.0)

    def g(x):
        return k * (L0 ** (5.0 / 3.0) - (x * x + L0 ** -2) ** (-5.0 / 6.0))
    for eps in (1e-2, 1e-3, 1e-4):
        n = np.arange(1, 2000 * 4 + 1)  # up to 2000/L0
        inc = g(n * df) - g((n - 1) * df)
        nstar = int(n[np.nonzero(inc >= eps * k * L0 ** (5.0 / 3.0))[0][-1]])
        N, s2 = oracle.choose_cartesian(df, eps, r0=r0, L0=L0)
        print(eps, N, 2 * nstar)
        assert N == 2 * nstar
        assert abs(s2 / (2 * math.pi * k * L0 ** (5.0 / 3.0)) - 1) < 1e-5


def test_stopping_rule_worked_example():
    """The worked example (UT filter, L0 = 22 m, df = 0.25/L0) chooses N = 44
    for a tolerance just under 1e-4 of the variance; N grows as eps falls,
    and Kolmogorov (diverging g) is refused."""
    Ns = [oracle.choose_cartesian(0.25 / 22, e, r0=0.1, L0=22.0, D=8.0, d=1.1)[0]
          for e in (1e-2, 1e-3, 1e-4, 5e-5)]
    print(Ns)
    assert Ns == sorted(Ns) and Ns[2] <= 44 <= Ns[3]
    assert oracle.choose_cartesian(0.01, 1e-3, model=oracle.PSD_KOLMOGOROV)[0] == 0
