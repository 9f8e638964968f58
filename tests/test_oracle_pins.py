"""Pins of the FP64 CPU oracle against things other than itself.

Each test ties one oracle function to a value the paper prints, a closed
form, a textbook or library routine for a special case, an independent
high-precision computation, or brute force on tiny inputs.  What pins what:

  plastic number, R2 increments  -- paper's printed psi (Sec. 3.2); Decimal
                                    Newton iteration at 50 digits
  R2 points                      -- Eq. 6 run literally as an FP64 recurrence;
                                    Decimal evaluation of frac(s0 + n/psi^j)
  Cartesian map                  -- worked example of Sec. 4.4 (N = 44)
  log-polar map + weights        -- closed-form band variance int 2 pi f W df
  PSD constant                   -- textbook Kolmogorov law 6.88 (r/r0)^(5/3)
                                    via independent quadrature; Eq. 7's 0.02289
  aperture filter                -- 2-D quadrature of the aperture's Fourier
                                    transform; first zero j_{1,1}
  Philox4x32-10                  -- Random123 known-answer vectors
  Box-Muller coefficients        -- moments / KS test against N(0,1)
  direct sum                     -- brute-force Python loop; inverse FFT on a
                                    DFT grid; K = 1 zeros
  piston                         -- average of the synthesized phase over the
                                    disk by polar Gauss quadrature
  diff-piston SF                 -- conditional expectation sum w^2 2(1-cos);
                                    analytic curve (statistical)
  analytic curves                -- Bessel-K closed form vs quadrature;
                                    Kolmogorov closed form; limits
"""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from oracle import analytic as A
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _psi_decimal():
    getcontext().prec = 60
    x = Decimal("1.3")
    for _ in range(100):
        x = x - (x ** 3 - x - 1) / (3 * x ** 2 - 1)
    return x


# ---------------------------------------------------------------- R2 ----

def test_plastic_number_matches_paper_and_definition():
    psi = oracle.plastic_number()
    assert abs(psi ** 3 - psi - 1.0) < 1e-15
    assert psi == pytest.approx(GOLD["plastic_number"]["value"], abs=1e-15)


def test_r2_increments_decimal():
    psi = _psi_decimal()
    two64 = Decimal(2) ** 64
    ax = int((two64 / psi).to_integral_value())
    ay = int((two64 / (psi * psi)).to_integral_value())
    assert oracle.r2_increments() == (ax, ay)


def test_r2_points_decimal_first_points():
    psi = _psi_decimal()
    ux, uy = oracle.r2_points(50, index=0)
    for i in range(50):
        n = i + 1  # the state is updated before it is used
        ex = (Decimal("0.5") + n / psi) % 1
        ey = (Decimal("0.5") + n / (psi * psi)) % 1
        assert abs(ux[i] - float(ex)) < 2.0 ** -52
        assert abs(uy[i] - float(ey)) < 2.0 ** -52


def test_r2_matches_eq6_fp64_recurrence():
    """Eq. 6 run literally: s <- {s + 1/psi} in FP64, never reinitialised."""
    n = 100000
    psi = oracle.plastic_number()
    ax, ay = 1.0 / psi, 1.0 / (psi * psi)
    sx = sy = 0.5
    rx = np.empty(n)
    ry = np.empty(n)
    for i in range(n):
        sx = (sx + ax) % 1.0
        sy = (sy + ay) % 1.0
        rx[i] = sx
        ry[i] = sy
    ux, uy = oracle.r2_points(n, index=0)
    dx = np.abs(((ux - rx) + 0.5) % 1.0 - 0.5)
    dy = np.abs(((uy - ry) + 0.5) % 1.0 - 0.5)
    bound = np.arange(1, n + 1) * 2.0 ** -52 + 2.0 ** -50
    assert np.all(dx <= bound) and np.all(dy <= bound)


def test_r2_jump_ahead_is_continuation():
    """The sequence is never reinitialised (Sec. 3.2): points from index i on
    equal the tail of a longer run from 0."""
    ux, uy = oracle.r2_points(3000, index=0)
    vx, vy = oracle.r2_points(1000, index=2000)
    assert np.array_equal(ux[2000:], vx) and np.array_equal(uy[2000:], vy)


def test_r2_low_discrepancy_no_clashes():
    """Sec. 3.2: R2 points avoid clashes: the minimum pairwise distance of
    N points is a fixed fraction of 1/sqrt(N), unlike uniform random points."""
    n = 2048
    ux, uy = oracle.r2_points(n)
    P = np.stack([ux, uy], 1)
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)) + np.eye(n) * 9
    assert d.min() * math.sqrt(n) > 0.3
    rng = np.random.default_rng(0)
    Q = rng.random((n, 2))
    dq = np.sqrt(((Q[:, None, :] - Q[None, :, :]) ** 2).sum(-1)) + np.eye(n) * 9
    assert dq.min() * math.sqrt(n) < 0.05


# ------------------------------------------------------------ maps ------

def test_cartesian_worked_example():
    g = GOLD["worked_example"]
    N = int(round(2 * g["fmax"] / g["df"]))
    assert N == g["N"]
    K = N * N
    fx, fy, area = oracle.sample_cartesian(2, K, N, g["df"])
    assert np.all(np.abs(fx) <= g["fmax"]) and np.all(np.abs(fy) <= g["fmax"])
    assert np.max(np.abs(fx)) > 0.99 * g["fmax"]
    assert np.allclose(area, g["df"] ** 2, rtol=1e-15)


def test_logpolar_band_variance_closed_form():
    """sum_k W(f_k) area_k -> int_{fmin}^{fmax} 2 pi f W df (closed form)."""
    cfg = workloads.phase_fp64()
    exact = A.variance_truncated(cfg["r0"], cfg["L0"], cfg["fmin"], cfg["fmax"])
    quad = integrate.quad(lambda f: 2 * np.pi * f * oracle.psd([f])[0], cfg["fmin"], cfg["fmax"],
                          limit=500, points=[0.04, 0.1, 1.0])[0]
    assert exact == pytest.approx(quad, rel=1e-8)
    for K, tol in ((1024, 3e-3), (65536, 3e-4)):
        fx, fy, area = oracle.sample_logpolar(1, K, cfg["fmin"], cfg["fmax"])
        w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=cfg["L0"])
        assert np.sum(w * w) == pytest.approx(exact, rel=tol)
    f = np.hypot(fx, fy)
    assert f.min() >= cfg["fmin"] * (1 - 1e-12) and f.max() <= cfg["fmax"] * (1 + 1e-12)


def test_cartesian_band_variance():
    """Cartesian cells of area delta_f^2 tile the square: sum W df^2 -> the
    integral of W over the square (brute-force fine midpoint grid)."""
    L0, r0 = 22.0, 0.1
    df = 0.25 / L0
    N = 44
    fx, fy, area = oracle.sample_cartesian(64, N * N, N, df)
    w = oracle.weights(fx, fy, area, r0=r0, L0=L0)
    est = np.sum(w * w) / 64
    m = 4000
    g = (np.arange(m) + 0.5) / m * N * df - N * df / 2
    FX, FY = np.meshgrid(g, g)
    c = oracle.psd_constant()
    Wg = c * r0 ** (-5 / 3) * (FX ** 2 + FY ** 2 + L0 ** -2) ** (-11 / 6)
    ref = Wg.sum() * (N * df / m) ** 2
    assert est == pytest.approx(ref, rel=2e-3)


# ------------------------------------------------------------- PSD ------

def test_psd_constant_kolmogorov_law():
    """With c*, 4 pi int f W (1 - J0) df equals the textbook 6.88 (r/r0)^(5/3)."""
    c = oracle.psd_constant()
    assert abs(c - GOLD["psd_constant_eq7"]["value"]) < 1e-5
    r = np.array([0.05, 0.3, 1.0])
    q = A.sf_band(r, 0.1, 1.0, 1e-15, 1e5, model=0)
    assert np.allclose(q, 6.88 * (r / 0.1) ** (5 / 3), rtol=2e-3)
    assert np.allclose(q, A.sf_kolmogorov(r, 0.1), rtol=2e-5)


def test_psd_values_and_kolmogorov_zero():
    c = oracle.psd_constant()
    f = np.array([1e-5, 0.1, 3.0])
    vk = oracle.psd(f, model=1, r0=0.1, L0=25.0)
    kol = oracle.psd(f, model=0, r0=0.1)
    # von Karman -> Kolmogorov for f >> 1/L0; flat below
    assert vk[2] == pytest.approx(kol[2], rel=1e-3)
    assert vk[0] == pytest.approx(c * 0.1 ** (-5 / 3) * 25.0 ** (11 / 3), rel=1e-6)
    fx = np.array([0.0, 1.0])
    w = oracle.weights(fx, np.zeros(2), np.ones(2), model=0, r0=0.1)
    assert w[0] == 0.0 and w[1] > 0


# ---------------------------------------------------------- filter ------

def _aperture_ft(f, D, d):
    """(1/area) int over the annulus of cos(2 pi f x) dA, polar Gauss quadrature."""
    xr, wr = np.polynomial.legendre.leggauss(200)
    xt, wt = np.polynomial.legendre.leggauss(400)
    a, b = d / 2, D / 2
    r = 0.5 * (b - a) * xr + 0.5 * (b + a)
    wr = 0.5 * (b - a) * wr
    th = np.pi * (xt + 1)
    wt = np.pi * wt
    R, T = np.meshgrid(r, th, indexing="ij")
    val = np.cos(2 * np.pi * f * R * np.cos(T)) * R
    I = np.einsum("i,j,ij->", wr, wt, val)
    return I / (np.pi * (b * b - a * a))


@pytest.mark.parametrize("D,d", [(1.8, 0.0), (8.0, 1.1)])
def test_aperture_filter_is_aperture_average(D, d):
    for f in (0.0, 0.05, 0.3, 0.9):
        assert oracle.aperture_filter([f], D, d)[0] == pytest.approx(_aperture_ft(f, D, d),
                                                                       abs=1e-10)


def test_aperture_filter_first_zero():
    j11 = special.jn_zeros(1, 1)[0]
    for D in (1.8, 8.0):
        f0 = j11 / (np.pi * D)
        assert abs(oracle.aperture_filter([f0], D)[0]) < 1e-13
    assert oracle.aperture_filter([0.0], 1.8)[0] == 1.0


# ------------------------------------------------------------- RNG ------

def test_philox_known_answers():
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, out in kat:
        assert list(oracle.philox4x32_10(ctr, key)) == out


def test_gaussian_coefficients_are_standard_normal():
    K = 2000
    c = np.concatenate([oracle.coefficients(0, r, K) for r in range(50)])
    n = c.size
    assert abs(c.mean()) < 5 / math.sqrt(n)
    assert abs(c.var() - 1) < 5 * math.sqrt(2 / n)
    assert stats.kstest(c, "norm").pvalue > 1e-4
    a, b = c[0::2], c[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)
    # independent streams for neighbouring realisations and seeds
    assert not np.array_equal(oracle.coefficients(0, 1, K), oracle.coefficients(0, 2, K))
    assert not np.array_equal(oracle.coefficients(0, 1, K), oracle.coefficients(1, 1, K))


def test_gaussian_coefficients_block_layout():
    """Block t of Philox gives coefficients 4t..4t+3 (Box-Muller of word pairs)."""
    seed, r = 0x1234567890ABCDEF, 77
    c = oracle.coefficients(seed, r, 6)
    x = oracle.philox4x32_10([1, r, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
    u = ((x >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
    rho = math.sqrt(-2 * math.log(u[0]))
    assert c[4] == pytest.approx(rho * math.cos(2 * math.pi * u[1]), rel=1e-14)
    assert c[5] == pytest.approx(rho * math.sin(2 * math.pi * u[1]), rel=1e-14)


def test_eq3_mode_moments():
    """Eq. 3 form: a = sqrt2 Rn cos 2pi Ru, b = -sqrt2 Rn sin 2pi Ru has
    E a^2 = E b^2 = 1 (same second moments as the Gaussian cos/sin form)."""
    K = 2000
    c = np.concatenate([oracle.coefficients(3, r, K, mode=1) for r in range(50)])
    n = c.size // 2
    for v in (c[0::2], c[1::2]):
        assert abs(np.mean(v * v) - 1) < 6 * math.sqrt(2 / n)


# ------------------------------------------------------- synthesis ------

def test_synthesize_brute_force():
    rng = np.random.default_rng(5)
    K, P, R, Rb = 3, 4, 5, 2
    n_sets = 3
    fx, fy = rng.normal(size=n_sets * K), rng.normal(size=n_sets * K)
    w = rng.random(n_sets * K)
    px, py = rng.normal(size=P), rng.normal(size=P)
    out = oracle.synthesize(fx, fy, w, px, py, R, Rb, K=K, seed=9, counter=11)
    for r in range(R):
        c = oracle.coefficients(9, 11 + r, K)
        s = r // Rb
        for p in range(P):
            acc = 0.0
            for k in range(K):
                i = s * K + k
                t = 2 * math.pi * (fx[i] * px[p] + fy[i] * py[p])
                acc += w[i] * (c[2 * k] * math.cos(t) + c[2 * k + 1] * math.sin(t))
            assert out[r, p] == pytest.approx(acc, rel=1e-12, abs=1e-14)
    coef = rng.normal(size=(R, 2 * K))
    out2 = oracle.synthesize(fx, fy, w, px, py, R, Rb, K=K, coef=coef)
    r, p, s = 4, 1, 2
    t = 2 * np.pi * (fx[s * K:(s + 1) * K] * px[p] + fy[s * K:(s + 1) * K] * py[p])
    ref = np.sum(w[s * K:(s + 1) * K] * (coef[r, 0::2] * np.cos(t) + coef[r, 1::2] * np.sin(t)))
    assert out2[r, p] == pytest.approx(ref, rel=1e-12)


def test_synthesize_single_frequency_zeros():
    """K = 1 with coefficients (1, 0): phi = w cos(2 pi f.x): w at 0, zero at f.x = 1/4."""
    f = 0.7
    px = np.array([0.0, 0.25 / f, 0.5 / f])
    out = oracle.synthesize([f], [0.0], [2.0], px, np.zeros(3), 1, 1, coef=np.array([[1.0, 0.0]]))
    assert out[0] == pytest.approx([2.0, 0.0, -2.0], abs=1e-14)
    out = oracle.synthesize([f], [0.0], [2.0], px, np.zeros(3), 1, 1, coef=np.array([[0.0, 1.0]]))
    assert out[0] == pytest.approx([0.0, 2.0, 0.0], abs=1e-14)


def test_synthesize_dft_grid_equals_inverse_fft():
    """Frequencies on a DFT grid and points on the matching spatial grid:
    sum_k w (a cos + b sin)(2 pi f.x) = Re[M^2 ifft2(w (a - i b))]."""
    M, Lbox = 8, 3.0
    rng = np.random.default_rng(1)
    ms, ns = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    fx, fy = (ms.ravel() / Lbox), (ns.ravel() / Lbox)
    w = rng.random(M * M)
    coef = rng.normal(size=(2, 2 * M * M))
    gi, gj = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    px, py = gi.ravel() * Lbox / M, gj.ravel() * Lbox / M
    out = oracle.synthesize(fx, fy, w, px, py, 2, 2, coef=coef)
    for r in range(2):
        spec = (w * (coef[r, 0::2] - 1j * coef[r, 1::2])).reshape(M, M)
        ref = np.real(np.fft.ifft2(spec)) * M * M
        assert np.allclose(out[r].reshape(M, M), ref, atol=1e-12)


def test_eq3_mode_is_eq3():
    """Mode 1 reproduces Eq. 3 term by term: (2/sqrt2) Rn w cos(2 pi (f.x + Ru))."""
    K = 5
    seed, r = 4, 3
    rng = np.random.default_rng(2)
    fx, fy, w = rng.normal(size=K), rng.normal(size=K), rng.random(K)
    px, py = rng.normal(size=3), rng.normal(size=3)
    out = oracle.synthesize(fx, fy, w, px, py, 1, 1, seed=seed, counter=r, mode=1)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for p in range(3):
        acc = 0.0
        for k in range(K):
            x = oracle.philox4x32_10([k, r, 0, 0], key)
            u = ((x >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
            Rn = math.sqrt(-2 * math.log(u[0])) * math.cos(2 * math.pi * u[1])
            Ru = u[2]
            acc += 2 / math.sqrt(2) * Rn * w[k] * math.cos(
                2 * math.pi * (fx[k] * px[p] + fy[k] * py[p] + Ru))
        assert out[0, p] == pytest.approx(acc, rel=1e-11, abs=1e-13)


# ---------------------------------------------------------- piston ------

def test_piston_equals_disk_average_of_phase():
    D, d = 1.8, 0.4
    K = 24
    rng = np.random.default_rng(3)
    f = rng.uniform(0.01, 2.0, K)
    th = rng.uniform(0, 2 * np.pi, K)
    fx, fy = f * np.cos(th), f * np.sin(th)
    w = rng.random(K)
    cx, cy = np.array([0.3, -2.0]), np.array([0.1, 5.0])
    R = 3
    pist = oracle.piston(fx, fy, w, cx, cy, D, d, R, R, seed=2, counter=5)
    xr, wr = np.polynomial.legendre.leggauss(60)
    xt, wt = np.polynomial.legendre.leggauss(120)
    a, b = d / 2, D / 2
    rr = 0.5 * (b - a) * xr + 0.5 * (b + a)
    wr = 0.5 * (b - a) * wr
    tt = np.pi * (xt + 1)
    wt = np.pi * wt
    RR, TT = np.meshgrid(rr, tt, indexing="ij")
    wq = (wr[:, None] * wt[None, :] * RR).ravel() / (np.pi * (b * b - a * a))
    for j in range(2):
        px = cx[j] + (RR * np.cos(TT)).ravel()
        py = cy[j] + (RR * np.sin(TT)).ravel()
        ph = oracle.synthesize(fx, fy, w, px, py, R, R, seed=2, counter=5)
        assert np.allclose(ph @ wq, pist[:, j], rtol=1e-9, atol=1e-11)


# ---------------------------------------------------- diff-piston SF ----

def test_diff_sf_conditional_expectation():
    """Given one frequency set, dp = p(B) - p(0) is N(0, S) with
    S = sum_k w_k^2 2 (1 - cos 2 pi f_k.B): the SF estimate is S chi2_R / R."""
    cfg = workloads.diffpiston()
    K, R = 64, 20000
    fx, fy, area = oracle.sample_logpolar(1, K, cfg["fmin"], cfg["fmax"])
    w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=25.0, D=cfg["D"])
    bx, by = cfg["bx"][::4], cfg["by"][::4]
    sf, se = oracle.diff_piston_sf(fx, fy, w, bx, by, R, R, seed=7)
    S = np.array([np.sum(w * w * 2 * (1 - np.cos(2 * np.pi * (fx * x + fy * y))))
                  for x, y in zip(bx, by)])
    z = (sf - S) / (S * math.sqrt(2.0 / R))
    assert np.all(np.abs(z) < 4.5)
    assert np.allclose(se / S, math.sqrt(2.0 / R), rtol=0.1)


@pytest.mark.slow
def test_diff_sf_matches_analytic_curve():
    """Fresh frequencies per realisation (R_block = 1, the paper's usage):
    the mean over realisations converges to the band-limited analytic SF."""
    cfg = workloads.diffpiston()
    K, R = 512, 3000
    fx, fy, area = oracle.sample_logpolar(R, K, cfg["fmin"], cfg["fmax"])
    w = oracle.weights(fx, fy, area, r0=cfg["r0"], L0=25.0, D=cfg["D"])
    bx, by = cfg["bx"][::3], cfg["by"][::3]
    sf, se = oracle.diff_piston_sf(fx, fy, w, bx, by, R, 1, K=K, seed=0)
    an = A.sf_band(bx, cfg["r0"], 25.0, cfg["fmin"], cfg["fmax"], D=cfg["D"])
    z = (sf - an) / se
    assert np.all(np.abs(z) < 4.5), z


# -------------------------------------------------------- analytic ------

def test_vk_closed_form_vs_quadrature():
    r = np.array([1 / 31, 0.1, 1.0, math.sqrt(2), 20.0])
    q = A.sf_band(r, 0.1, 25.0, 1e-9, 1e4)
    assert np.allclose(q, A.sf_vk(r, 0.1, 25.0), rtol=1e-5)


def test_vk_variance_and_limits():
    s2 = A.variance_vk(0.1, 25.0)
    q = integrate.quad(lambda f: 2 * np.pi * f * oracle.psd([f], r0=0.1, L0=25.0)[0], 0, np.inf,
                       limit=500)[0]
    assert s2 == pytest.approx(q, rel=1e-7)
    assert A.sf_vk([1e4], 0.1, 25.0)[0] == pytest.approx(2 * s2, rel=1e-6)
    # large outer scale: the von Karman SF approaches Kolmogorov's from below
    # (the leading correction is of relative order (r/L0)^(1/3), ~1.5 % here)
    ratio = A.sf_vk([1.0], 0.1, 1e6)[0] / A.sf_kolmogorov([1.0], 0.1)[0]
    assert 0.97 < ratio < 1.0


def test_diff_piston_limits():
    D = 1.8
    C0 = A.piston_cov([0.0], 0.1, 25.0, D)[0]
    # very long baseline: pistons decorrelate
    assert A.diff_piston_sf([600.0], 0.1, 25.0, D)[0] == pytest.approx(2 * C0, rel=1e-4)
    # vanishing aperture: differential piston -> phase structure function
    assert A.diff_piston_sf([3.0], 0.1, 25.0, 1e-4, fmax=1e3)[0] == pytest.approx(
        A.sf_vk([3.0], 0.1, 25.0)[0], rel=1e-4)
    # piston variance = phase variance filtered: below the phase variance
    assert C0 < A.variance_vk(0.1, 25.0)


def test_optical_path_weights_are_achromatic():
    """Optical path = (lambda / 2 pi) phase (Sec. 4.4) and r0 = r0(lambda)
    grows as lambda^(6/5) (Sec. 4.1): the phase variance then falls as
    lambda^-2, so OPD weights do not depend on the wavelength; and their
    squares sum to (lambda / 2 pi)^2 times the closed-form band variance."""
    fx, fy, area = oracle.sample_logpolar(1, 4096, 1e-3, 1e2)
    lam0, r00 = 0.5e-6, 0.1
    ref = None
    for lam in (0.5e-6, 1.65e-6, 2.2e-6, 10e-6):
        r0 = r00 * (lam / lam0) ** 1.2
        w = oracle.weights(fx, fy, area, r0=r0, L0=25.0, D=1.8, wavelength=lam)
        if ref is None:
            ref = w
        assert np.max(np.abs(w - ref)) <= 1e-13 * np.max(np.abs(ref))
        w = oracle.weights(fx, fy, area, r0=r0, L0=25.0, wavelength=lam)
        band = A.variance_truncated(r0, 25.0, 1e-3, 1e2) * (lam / (2 * np.pi)) ** 2
        assert np.sum(w * w) == pytest.approx(band, rel=2e-3)
