"""Pins of the randomised frequency samplers (Sec. 3.1: fully random
frequencies, the jittered grid of Eq. 4), of the point-set measures (clashes,
gaps, L2 star discrepancy) and of the noise-free per-set structure function,
each against closed forms, brute force or an independent library routine."""
import math

import numpy as np
import pytest
from scipy import special, stats
from scipy.spatial.distance import pdist

import oracle
import workloads
from oracle import analytic as A


# ------------------------------------------------ pseudo-random stream ----

def test_pseudo_points_are_uniform():
    ux, uy = oracle.pseudo_points(400000, index=123)
    assert ux.min() >= 0.0 and ux.max() < 1.0 and uy.min() >= 0.0 and uy.max() < 1.0
    for u in (ux, uy):
        assert stats.kstest(u, "uniform").pvalue > 1e-4
        assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    n = ux.size
    for a, b in ((ux, uy), (ux[:-1], ux[1:]), (uy[:-1], uy[1:])):
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(n)


def test_pseudo_points_jump_ahead():
    """Point n depends on n only: a call starting at index m returns the
    tail of a call starting earlier."""
    ux, uy = oracle.pseudo_points(1000, index=5)
    vx, vy = oracle.pseudo_points(10, index=5 + 990)
    assert np.array_equal(ux[990:], vx) and np.array_equal(uy[990:], vy)
    wx, _ = oracle.pseudo_points(10, index=5, seed_y=3)
    assert not np.array_equal(ux[:10], wx)  # the stream id changes the points


# ----------------------------------------------------------- samplers ----

def test_jitter_one_point_per_cell():
    """Eq. 4: point k = iy N + ix of every set lies in cell (ix, iy) of the
    N x N grid of side df centred on the origin; the offsets in their cells
    are uniform."""
    N, df, n_sets = 44, 0.25 / 22, 50
    fx, fy, area = oracle.sample_jitter(n_sets, N, df, index=77)
    assert np.all(area == df * df)
    k = np.arange(fx.size) % (N * N)
    tx, ty = fx / df + N / 2, fy / df + N / 2
    assert np.array_equal(np.floor(tx), k % N) and np.array_equal(np.floor(ty), k // N)
    for t in (tx - np.floor(tx), ty - np.floor(ty)):
        assert stats.kstest(t, "uniform").pvalue > 1e-4


def _gauss_square(s, L):
    """int over [-L/2, L/2]^2 of exp(-|f|^2 / (2 s^2))."""
    return (s * math.sqrt(2 * math.pi) * special.erf(L / (2 * math.sqrt(2) * s))) ** 2


def _gauss_annulus(s, r1, r2):
    return 2 * math.pi * s * s * (math.exp(-r1 * r1 / (2 * s * s)) - math.exp(-r2 * r2 / (2 * s * s)))


@pytest.mark.parametrize("scheme", ["jitter", "random_cartesian", "random_logpolar",
                                    "random_disc"])
def test_weighted_sums_are_unbiased(scheme):
    """Each randomised set gives an unbiased estimate of an integral over its
    domain: the mean over sets of sum_k area_k g(f_k), g a Gaussian,
    against the integral in closed form (a misplaced grid, a wrong cell area
    or a biased map fails it)."""
    n_sets, s = 400, 0.3
    if scheme == "jitter":
        N, df = 20, 0.1
        fx, fy, area = oracle.sample_jitter(n_sets, N, df)
        K, exact = N * N, _gauss_square(s, N * df)
    elif scheme == "random_cartesian":
        K, N, df = 300, 20, 0.1
        fx, fy, area = oracle.sample_pseudo(oracle.MAP_CARTESIAN, n_sets, K, N=N, df=df)
        exact = _gauss_square(s, N * df)
    elif scheme == "random_logpolar":
        K, fmin, fmax = 300, 1e-3, 2.0
        fx, fy, area = oracle.sample_pseudo(oracle.MAP_LOGPOLAR, n_sets, K, fmin=fmin, fmax=fmax)
        exact = _gauss_annulus(s, fmin, fmax)
    else:
        K, fmax = 300, 1.0
        fx, fy, area = oracle.sample_pseudo(oracle.MAP_DISC, n_sets, K, fmax=fmax)
        exact = _gauss_annulus(s, 0.0, fmax)
    g = np.exp(-(fx * fx + fy * fy) / (2 * s * s))
    est = (area * g).reshape(n_sets, K).sum(axis=1)
    z = (est.mean() - exact) / (est.std(ddof=1) / math.sqrt(n_sets))
    print(scheme, est.mean() / exact - 1, "z", z)
    assert abs(z) < 4.5


def test_jitter_beats_random_variance():
    """Stratification: the spread of the set estimates is far smaller for
    the jittered grid than for fully random points at equal K."""
    n_sets, N, df, s = 200, 20, 0.1, 0.3
    fx, fy, area = oracle.sample_jitter(n_sets, N, df)
    gx, gy, garea = oracle.sample_pseudo(oracle.MAP_CARTESIAN, n_sets, N * N, N=N, df=df)
    sd_j = (area * np.exp(-(fx ** 2 + fy ** 2) / (2 * s * s))).reshape(n_sets, -1).sum(1).std()
    sd_r = (garea * np.exp(-(gx ** 2 + gy ** 2) / (2 * s * s))).reshape(n_sets, -1).sum(1).std()
    assert sd_j < 0.2 * sd_r


# ---------------------------------------------------- point-set measures ----

def _l2_star_exact(x, y):
    """Squared L2 star discrepancy by exact integration of the squared local
    discrepancy (A(t)/K - t_x t_y)^2 over the cells cut by the points'
    coordinates, on which the count A is constant."""
    K = x.size
    ex = np.unique(np.concatenate([[0.0, 1.0], x]))
    ey = np.unique(np.concatenate([[0.0, 1.0], y]))
    tot = 0.0
    for x1, x2 in zip(ex[:-1], ex[1:]):
        for y1, y2 in zip(ey[:-1], ey[1:]):
            a = np.count_nonzero((x <= x1) & (y <= y1)) / K  # points strictly below the cell
            Ix1, Iy1 = x2 - x1, y2 - y1
            Ix2, Iy2 = (x2 ** 2 - x1 ** 2) / 2, (y2 ** 2 - y1 ** 2) / 2
            Ix3, Iy3 = (x2 ** 3 - x1 ** 3) / 3, (y2 ** 3 - y1 ** 3) / 3
            tot += a * a * Ix1 * Iy1 - 2 * a * Ix2 * Iy2 + Ix3 * Iy3
    return tot


@pytest.mark.parametrize("K", [1, 2, 5, 9])
def test_l2_star_matches_exact_integral(K):
    rng = np.random.default_rng(K)
    x, y = rng.random(K), rng.random(K)
    _, _, T = oracle.point_set_measures(x, y, 1, K, 0.0, 0.0, 1.0, 1.0, 0.1)
    assert abs(T[0] ** 2 - _l2_star_exact(x, y)) < 1e-13


def test_l2_star_expectation_for_random_points():
    """iid uniform points: E[T^2] = (1/K)(1/4 - 1/9) in two dimensions."""
    n_sets, K = 400, 64
    ux, uy = oracle.pseudo_points(n_sets * K)
    _, _, T = oracle.point_set_measures(ux, uy, n_sets, K, 0.0, 0.0, 1.0, 1.0, 0.0)
    T2 = T ** 2
    exact = (0.25 - 1.0 / 9.0) / K
    z = (T2.mean() - exact) / (T2.std(ddof=1) / math.sqrt(n_sets))
    print("E[T^2]", T2.mean(), exact, "z", z)
    assert abs(z) < 4.5


def test_min_distance_and_clashes_match_pdist():
    rng = np.random.default_rng(0)
    n_sets, K, r = 5, 300, 0.01
    fx, fy = rng.uniform(-3, 5, n_sets * K), rng.uniform(2, 4, n_sets * K)
    md, nc, _ = oracle.point_set_measures(fx, fy, n_sets, K, -3.0, 2.0, 8.0, 2.0, r)
    for s in range(n_sets):
        u = np.stack([(fx[s * K:(s + 1) * K] + 3) / 8, (fy[s * K:(s + 1) * K] - 2) / 2], axis=1)
        d = pdist(u)
        assert abs(md[s] - d.min()) <= 1e-15 * max(1.0, d.min())
        assert nc[s] == np.count_nonzero(d < r)


def test_clash_expectation_for_random_points():
    """iid uniform points in the unit square: a pair is closer than r with
    probability pi r^2 - 8 r^3 / 3 + r^4 / 2 (r <= 1)."""
    n_sets, K, r = 300, 200, 0.02
    ux, uy = oracle.pseudo_points(n_sets * K, index=999)
    _, nc, _ = oracle.point_set_measures(ux, uy, n_sets, K, 0.0, 0.0, 1.0, 1.0, r)
    p = math.pi * r * r - 8 * r ** 3 / 3 + r ** 4 / 2
    exact = K * (K - 1) / 2 * p
    z = (nc.mean() - exact) / (nc.std(ddof=1) / math.sqrt(n_sets))
    print("clashes", nc.mean(), exact, "z", z)
    assert abs(z) < 4.5


def test_r2_sets_have_no_clashes_and_low_discrepancy():
    """Sec. 3.2: the quasi-random sets cover the square evenly, without the
    clusters of the randomised schemes: larger minimum distance, no pairs
    within a tenth of the mean spacing, and a smaller discrepancy than the
    jittered grid (itself far below fully random points) at the worked
    example's K = 44^2."""
    N, df, n_sets = 44, 0.25 / 22, 20
    K, L = N * N, N * df
    r = 0.1 / N
    res = {}
    for name, (fx, fy, _) in {
            "r2": oracle.sample_cartesian(n_sets, K, N, df),
            "jitter": oracle.sample_jitter(n_sets, N, df),
            "random": oracle.sample_pseudo(oracle.MAP_CARTESIAN, n_sets, K, N=N, df=df)}.items():
        res[name] = oracle.point_set_measures(fx, fy, n_sets, K, -L / 2, -L / 2, L, L, r)
    for name, (md, nc, T) in res.items():
        print(name, "min dist x N", np.round(md.mean() * N, 4), "clashes", nc.mean(),
              "T", T.mean())
    assert np.all(res["r2"][1] == 0)
    assert res["jitter"][1].mean() > 1 and res["random"][1].mean() > 1
    assert res["r2"][0].min() > 3 * res["jitter"][0].max()
    assert res["r2"][2].mean() < res["jitter"][2].mean() < 0.2 * res["random"][2].mean()


# ------------------------------------------- noise-free per-set SF ----

def test_set_sf_expectation_is_the_mean_of_the_estimator():
    """One frequency set, many coefficient draws: the oracle's estimator
    (pistons synthesised term by term) averages to S within its noise."""
    cfg = workloads.diffpiston()
    K, R = 96, 20000
    fx, fy, area = oracle.sample_pseudo(oracle.MAP_LOGPOLAR, 1, K, fmin=cfg["fmin"],
                                        fmax=cfg["fmax"])
    w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=25.0, D=cfg["D"])
    bx, by = cfg["bx"][::5], cfg["by"][::5]
    S = oracle.set_sf_expectation(fx, fy, w, 1, K, bx, by)[0]
    sf, _ = oracle.diff_piston_sf(fx, fy, w, bx, by, R, R, seed=3)
    z = (sf - S) / (S * math.sqrt(2.0 / R))
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)


def test_set_sf_expectation_approaches_the_analytic_curve():
    """A large quasi-random set: the per-set value is the band-limited
    analytic differential-piston SF to within 0.2 %."""
    cfg = workloads.diffpiston()
    K = 65536
    fx, fy, area = oracle.sample_logpolar(1, K, cfg["fmin"], cfg["fmax"])
    w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=25.0, D=cfg["D"])
    bx, by = cfg["bx"][::4], cfg["by"][::4]
    S = oracle.set_sf_expectation(fx, fy, w, 1, K, bx, by)[0]
    ref = A.diff_piston_sf(np.hypot(bx, by), cfg["r0"], 25.0, cfg["D"], fmin=cfg["fmin"],
                           fmax=cfg["fmax"])
    e = S / ref - 1
    print("rel err", np.round(e, 5))
    assert np.max(np.abs(e)) < 2e-3


def test_square_expectation_matches_isotropic_curve():
    """The square-domain integral of W F^2 4 sin^2(pi f.B) (2-D tensor
    quadrature) reaches the isotropic differential-piston curve (1-D Bessel
    form) once the square covers the band the UT filter passes."""
    B = np.array([5.0, 56.5, 130.0])
    sq = A.diff_piston_sf_square(B, 0 * B, 0.1, 22.0, 8.0, 1.1, half_width=2.0, n=600)
    full = A.diff_piston_sf(B, 0.1, 22.0, 8.0, 1.1)
    assert np.max(np.abs(sq / full - 1)) < 1e-6
