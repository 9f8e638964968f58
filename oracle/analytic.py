"""Analytic second-order statistics the estimator of Eq. 3 converges to.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Plain numpy/scipy, FP64.

The paper states the phase PSD (Sec. 4.1, Eq. 7, first factor) and the
circular-aperture filter (Eq. 7, second factor), and says the differential
piston structure function "can be predicted analytically" (Sec. 1) without
printing the prediction.  The forms below follow from the isotropic PSD by
the Wiener-Khinchin theorem (Sec. 2.1):

  covariance      B(r) = 2 pi int_0^inf f W(f) J0(2 pi f r) df
  structure fn    D(r) = 2 (B(0) - B(r)) = 4 pi int f W(f) (1 - J0(2 pi f r)) df

For the piston the PSD is multiplied by F(f)^2 (Eq. 7).  "Truncated" forms
restrict the integral to the sampled band [fmin, fmax]; they are the exact
expectation of the estimator when the frequencies cover that band.
"""
import numpy as np
from scipy import special

from . import psd_constant

_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


def variance_vk(r0, L0, c=None):
    """sigma^2 = int 2 pi f W df over (0, inf) = (6 pi/5) c (L0/r0)^(5/3) (von Karman)."""
    c = psd_constant() if c is None else c
    return 6.0 * np.pi / 5.0 * c * (L0 / r0) ** (5.0 / 3.0)


def variance_truncated(r0, L0, fmin, fmax, c=None, model=1):
    """int_{fmin}^{fmax} 2 pi f W(f) df in closed form."""
    c = psd_constant() if c is None else c
    a2 = 1.0 / L0 ** 2 if model == 1 else 0.0
    return 6.0 * np.pi / 5.0 * c * r0 ** (-5.0 / 3.0) * (
        (fmin ** 2 + a2) ** (-5.0 / 6.0) - (fmax ** 2 + a2) ** (-5.0 / 6.0))


def sf_vk(r, r0, L0, c=None):
    """Von Karman phase structure function, closed form with the modified
    Bessel function: D = 2 sigma^2 [1 - 2^(1/6)/Gamma(5/6) z^(5/6) K_{5/6}(z)],
    z = 2 pi r / L0."""
    r = np.asarray(r, dtype=np.float64)
    s2 = variance_vk(r0, L0, c)
    z = 2.0 * np.pi * r / L0
    with np.errstate(invalid="ignore"):
        cov = 2.0 ** (1.0 / 6.0) / special.gamma(5.0 / 6.0) * z ** (5.0 / 6.0) * special.kv(5.0 / 6.0, z)
    cov = np.where(z == 0, 1.0, cov)
    return 2.0 * s2 * (1.0 - cov)


def sf_kolmogorov(r, r0, c=None):
    """Kolmogorov phase structure function 2 [24/5 Gamma(6/5)]^(5/6) (r/r0)^(5/3),
    scaled by c / c* when the PSD constant differs from the exact one."""
    cstar = psd_constant()
    c = cstar if c is None else c
    k = 2.0 * (24.0 / 5.0 * special.gamma(6.0 / 5.0)) ** (5.0 / 6.0)
    return k * (c / cstar) * (np.asarray(r, dtype=np.float64) / r0) ** (5.0 / 3.0)


def _panel_edges(fmin, fmax, scale):
    """Panel edges: log-spaced (for the power-law part) merged with a uniform
    grid of width 1/(8 scale) (for the J0 oscillation of period ~1/scale)."""
    edges = np.geomspace(fmin, fmax, 2000)
    if scale > 0:
        h = 1.0 / (8.0 * scale)
        lin = np.arange(fmin, fmax, h)
        edges = np.union1d(edges, lin)
    return edges


def _integrate(g, fmin, fmax, scale):
    e = _panel_edges(fmin, fmax, scale)
    a, b = e[:-1], e[1:]
    half = 0.5 * (b - a)
    mid = 0.5 * (b + a)
    x = mid[:, None] + half[:, None] * _GL_X[None, :]
    return float(np.sum(half[:, None] * _GL_W[None, :] * g(x)))


def one_minus_j0(x):
    """1 - J0(x) without cancellation: the power series
    x^2/4 - x^4/64 + x^6/2304 - x^8/147456 for |x| < 0.1, scipy's J0 above."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    series = x2 / 4.0 * (1.0 - x2 / 16.0 * (1.0 - x2 / 36.0 * (1.0 - x2 / 64.0)))
    with np.errstate(invalid="ignore"):
        direct = 1.0 - special.j0(x)
    return np.where(np.abs(x) < 0.1, series, direct)


def _psd(f, r0, L0, c, model):
    a2 = 1.0 / L0 ** 2 if model == 1 else 0.0
    return c * r0 ** (-5.0 / 3.0) * (f * f + a2) ** (-11.0 / 6.0)


def aperture_filter(f, D, d=0.0):
    """Eq. 7's aperture factor F (so that Eq. 7's 4(...)^2 is F^2), via scipy's J1."""
    f = np.asarray(f, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        num = D * special.j1(np.pi * D * f) - (d * special.j1(np.pi * d * f) if d > 0 else 0.0)
        F = 2.0 * num / (np.pi * (D * D - d * d) * f)
    return np.where(f == 0, 1.0, F)


def sf_band(r, r0, L0, fmin, fmax, c=None, model=1, D=None, d=0.0):
    """Structure function of the (optionally aperture-filtered) PSD restricted
    to the band [fmin, fmax]: 4 pi int f W F^2 (1 - J0(2 pi f r)) df."""
    c = psd_constant() if c is None else c
    out = []
    for rr in np.atleast_1d(r):
        def g(f, rr=rr):
            v = f * _psd(f, r0, L0, c, model) * one_minus_j0(2.0 * np.pi * f * rr)
            if D is not None:
                v = v * aperture_filter(f, D, d) ** 2
            return v
        out.append(4.0 * np.pi * _integrate(g, fmin, fmax, rr))
    return np.array(out)


def piston_cov(u, r0, L0, D, d=0.0, c=None, model=1, fmin=1e-7, fmax=None):
    """Piston covariance C(u) = 2 pi int f W F^2 J0(2 pi f u) df."""
    c = psd_constant() if c is None else c
    fmax = fmax if fmax is not None else 40.0 / D
    out = []
    for uu in np.atleast_1d(u):
        def g(f, uu=uu):
            return f * _psd(f, r0, L0, c, model) * aperture_filter(f, D, d) ** 2 * special.j0(
                2.0 * np.pi * f * uu)
        out.append(2.0 * np.pi * _integrate(g, fmin, fmax, uu))
    return np.array(out)


def diff_piston_sf(B, r0, L0, D, d=0.0, c=None, model=1, fmin=1e-7, fmax=None):
    """Differential-piston structure function over a baseline B between two
    equal apertures: 2 (C(0) - C(B)) = 4 pi int f W F^2 (1 - J0(2 pi f B)) df.
    Default band: effectively untruncated."""
    fmax = fmax if fmax is not None else 40.0 / D
    return sf_band(B, r0, L0, fmin, fmax, c=c, model=model, D=D, d=d)


def temporal_sf(tau, B, v, r0, L0, D, d=0.0, c=None, model=1, fmin=1e-7, fmax=None):
    """Frozen-flow structure function of the differential piston between two
    equal apertures separated by the vector B, wind velocity vector v, at
    lags tau (Sec. 4.4): with u = v tau and the piston covariance C,
    D(tau) = 4 C(0) - 4 C(|B|) - 4 C(|u|) + 2 C(|B - u|) + 2 C(|B + u|)
    (the variance of dp(t + tau) - dp(t), dp = p(c1 - v t) - p(c2 - v t))."""
    B = np.asarray(B, dtype=float)
    v = np.asarray(v, dtype=float)
    tau = np.atleast_1d(np.asarray(tau, dtype=float))
    kw = dict(r0=r0, L0=L0, D=D, d=d, c=c, model=model, fmin=fmin, fmax=fmax)
    C0 = piston_cov(0.0, **kw)[0]
    CB = piston_cov(np.hypot(*B), **kw)[0]
    out = []
    for t in tau:
        u = v * t
        Cu = piston_cov(np.hypot(*u), **kw)[0]
        Cm = piston_cov(np.hypot(*(B - u)), **kw)[0]
        Cp = piston_cov(np.hypot(*(B + u)), **kw)[0]
        out.append(4.0 * C0 - 4.0 * CB - 4.0 * Cu + 2.0 * Cm + 2.0 * Cp)
    return np.array(out)


def _square_rule(half_width, n):
    """Nodes and weights of a tensor Gauss-Legendre rule on n x n panels of
    the square [-half_width, half_width)^2 (6 points per panel and axis)."""
    xg, wg = np.polynomial.legendre.leggauss(6)
    edges = np.linspace(-half_width, half_width, n + 1)
    h = np.diff(edges)
    nodes = (edges[:-1, None] + 0.5 * h[:, None] * (xg[None, :] + 1.0)).ravel()
    wts = (0.5 * h[:, None] * wg[None, :]).ravel()
    return nodes, wts


def temporal_sf_square(tau, B, v, r0, L0, D, d=0.0, half_width=0.25, c=None, model=1, n=801):
    """Exact expectation of the temporal estimator when the frequencies fill
    the square [-half_width, half_width)^2 (the Cartesian R2 domain of Eq. 5,
    N df = 2 fmax): the double integral of W F^2 16 sin^2(pi f.B)
    sin^2(pi f.v tau) over the square, by a tensor Gauss-Legendre rule on
    sub-squares (the integrand is smooth; W is finite for von Karman)."""
    c = psd_constant() if c is None else c
    B = np.asarray(B, dtype=float)
    v = np.asarray(v, dtype=float)
    tau = np.atleast_1d(np.asarray(tau, dtype=float))
    nodes, wts = _square_rule(half_width, n)
    out = np.zeros(tau.size)
    step = 256  # one strip of rows at a time
    for i0 in range(0, nodes.size, step):
        FX, FY = np.meshgrid(nodes[i0:i0 + step], nodes, indexing="ij")
        WW = np.outer(wts[i0:i0 + step], wts)
        f = np.maximum(np.hypot(FX, FY), 1e-300)
        base = (WW * _psd(f, r0, L0, c, model) * aperture_filter(f, D, d) ** 2
                * np.sin(np.pi * (FX * B[0] + FY * B[1])) ** 2)
        for j, t in enumerate(tau):
            u = v * t
            out[j] += 16.0 * np.sum(base * np.sin(np.pi * (FX * u[0] + FY * u[1])) ** 2)
    return out


def diff_piston_sf_square(Bx, By, r0, L0, D, d=0.0, half_width=0.25, c=None, model=1, n=401):
    """Expectation of the differential-piston structure function when the
    frequencies fill the square [-half_width, half_width)^2: the double
    integral of W F^2 2 (1 - cos 2 pi f.B) = W F^2 4 sin^2(pi f.B) over the
    square, by the same tensor Gauss-Legendre rule."""
    c = psd_constant() if c is None else c
    Bx = np.atleast_1d(np.asarray(Bx, dtype=float))
    By = np.atleast_1d(np.asarray(By, dtype=float))
    nodes, wts = _square_rule(half_width, n)
    out = np.zeros(Bx.size)
    step = 256
    for i0 in range(0, nodes.size, step):
        FX, FY = np.meshgrid(nodes[i0:i0 + step], nodes, indexing="ij")
        WW = np.outer(wts[i0:i0 + step], wts)
        f = np.maximum(np.hypot(FX, FY), 1e-300)
        base = WW * _psd(f, r0, L0, c, model) * aperture_filter(f, D, d) ** 2
        for j in range(Bx.size):
            out[j] += 4.0 * np.sum(base * np.sin(np.pi * (FX * Bx[j] + FY * By[j])) ** 2)
    return out


def tilt_variance(r0, L0, D, d=0.0, c=None, model=1, fmin=1e-12, fmax=None):
    """One-axis variance of the aperture-averaged phase gradient (G-tilt),
    rad^2/m^2: int d^2f W F^2 (2 pi f_x)^2 = 4 pi^3 int f^3 W F^2 df (for
    Kolmogorov the integrand grows as f^(-2/3) at f -> 0: the band starts at
    1e-12, which leaves out 3 (1e-12 D)^(1/3) of the scaled integral)."""
    c = psd_constant() if c is None else c
    fmax = fmax if fmax is not None else 400.0 / D

    def g(f):
        return f ** 3 * _psd(f, r0, L0, c, model) * aperture_filter(f, D, d) ** 2
    return 4.0 * np.pi ** 3 * _integrate(g, fmin, fmax, D)
