"""FP64 CPU oracle for quasi-random frequency sampling (arXiv 2404.02978).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the HIP path (``paper_2404_02978_amd``) and never imports it.

The arithmetic lives in ``qrfs_oracle.c`` (plain double-precision loops,
compiled with gcc); this module only marshals numpy arrays.  The analytic
structure functions the estimator converges to live in ``oracle.analytic``.

Parity status of each function (what pins it) is listed in the module
docstring of ``tests/test_oracle_pins.py``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "oracle_plastic_number": (None, [_p]),
        "oracle_r2_increments": (None, [_p]),
        "oracle_r2_points": (None, [_u64, _u64, _u64, _i64, _p, _p]),
        "oracle_sample_cartesian": (None, [_u64, _u64, _u64, _i64, _i64, _i32, _d, _p, _p, _p]),
        "oracle_sample_logpolar": (None, [_u64, _u64, _u64, _i64, _i64, _d, _d, _p, _p, _p]),
        "oracle_psd_constant": (_d, []),
        "oracle_psd": (_d, [_i32, _d, _d, _d, _d]),
        "oracle_aperture_filter": (_d, [_d, _d, _d]),
        "oracle_weights": (None, [_i32, _d, _d, _d, _i32, _d, _d, _d, _i64, _p, _p, _p, _p]),
        "oracle_philox4x32_10": (None, [_p, _p, _p]),
        "oracle_coefficients": (None, [_u64, _u64, _i64, _i32, _p]),
        "oracle_synthesize": (None, [_i64, _p, _p, _p, _i64, _p, _p, _i64, _i64, _u64, _u64,
                                     _i32, _p, _p]),
        "oracle_piston": (None, [_i64, _p, _p, _p, _i64, _p, _p, _p, _p, _i64, _i64, _u64,
                                 _u64, _i32, _p, _p]),
        "oracle_diff_piston_sf": (None, [_i64, _p, _p, _p, _i64, _p, _p, _i64, _i64, _u64,
                                         _u64, _i32, _p, _p]),
        "oracle_temporal_sf": (None, [_p, _i64, _i64, _p, _p]),
        "oracle_concentric_map": (None, [_d, _d, _p, _p]),
        "oracle_tilt": (None, [_i64, _p, _p, _p, _i64, _p, _p, _p, _p, _i64, _i64, _u64, _u64,
                               _i32, _p, _i32, _p]),
        "oracle_sample_disc": (None, [_u64, _u64, _u64, _i64, _i64, _d, _p, _p, _p]),
        "oracle_pseudo_points": (None, [_u64, _u64, _u64, _i64, _p, _p]),
        "oracle_sample_pseudo": (None, [_i32, _u64, _u64, _u64, _i64, _i64, _i32, _d, _d, _d,
                                        _p, _p, _p]),
        "oracle_sample_jitter": (None, [_u64, _u64, _u64, _i64, _i32, _d, _p, _p, _p]),
        "oracle_point_set_measures": (None, [_i64, _i64, _p, _p, _d, _d, _d, _d, _d, _p, _p,
                                             _p]),
        "oracle_set_sf_expectation": (None, [_i64, _p, _p, _p, _i64, _i64, _p, _p, _p]),
        "oracle_choose_cartesian": (_i64, [_i32, _d, _d, _d, _i32, _d, _d, _d, _d, _d, _p]),
        "oracle_temporal_experiment": (None, [_i64, _p, _p, _p, _p, _p, _p, _d, _i64, _i64,
                                              _i64, _u64, _u64, _i32, _p, _p]),
    }
    sig.update({
        "oracle_mlp_param_count": (_i64, [ctypes.c_int]),
        "oracle_mlp_forward": (None, [_p, ctypes.c_int, _d, _d, _i64, _p, _p, _p]),
        "oracle_mlp_loss_grad": (_d, [_p, ctypes.c_int, _d, _d, _i64, _i64, _p, _p, _p, _p,
                                      ctypes.c_int, _p]),
        "oracle_proposal_rows": (None, [_u64, _u64, _u64, _i64, _i64, _p, _d, _d, _d, _d, _p, _p,
                                        _p]),
        "oracle_proposal_table": (None, [_p, ctypes.c_int, _d, _d, ctypes.c_int, _d, _d, _i64, _p,
                                         _p, _d, _p, _p, _p, _p]),
        "oracle_sample_learned": (None, [_u64, _u64, _u64, _i64, _i64, _d, _d, ctypes.c_int, _p,
                                         _p, _p, _p, _p, _p, _p]),
    })
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data


PSD_KOLMOGOROV = 0
PSD_VON_KARMAN = 1
COEF_GAUSS_CS = 0
COEF_EQ3 = 1
SEED_HALF = 1 << 63  # s0 = 1/2 in 0.64 fixed point


def plastic_number():
    out = np.zeros(1)
    _load().oracle_plastic_number(_ptr(out))
    return float(out[0])


def r2_increments():
    out = np.zeros(2, dtype=np.uint64)
    _load().oracle_r2_increments(_ptr(out))
    return int(out[0]), int(out[1])


def r2_points(n, index=0, s0x=SEED_HALF, s0y=SEED_HALF):
    ux = np.zeros(n)
    uy = np.zeros(n)
    _load().oracle_r2_points(s0x, s0y, index, n, _ptr(ux), _ptr(uy))
    return ux, uy


def sample_cartesian(n_sets, K, N, df, index=0, s0x=SEED_HALF, s0y=SEED_HALF):
    n = n_sets * K
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_cartesian(s0x, s0y, index, n_sets, K, N, df, _ptr(fx), _ptr(fy),
                                    _ptr(area))
    return fx, fy, area


def sample_logpolar(n_sets, K, fmin, fmax, index=0, s0x=SEED_HALF, s0y=SEED_HALF):
    n = n_sets * K
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_logpolar(s0x, s0y, index, n_sets, K, fmin, fmax, _ptr(fx), _ptr(fy),
                                   _ptr(area))
    return fx, fy, area


def concentric_map(ux, uy):
    """Square-to-disc map of one point (ux, uy) in [0,1)^2 -> (x, y), |(x, y)| < 1."""
    x, y = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _load().oracle_concentric_map(float(ux), float(uy), ctypes.byref(x), ctypes.byref(y))
    return x.value, y.value


def sample_disc(n_sets, K, fmax, index=0, s0x=SEED_HALF, s0y=SEED_HALF):
    """Polar quasi-random frequencies on the disc |f| < fmax (Sec. 3.2)."""
    n = n_sets * K
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_disc(s0x, s0y, index, n_sets, K, fmax, _ptr(fx), _ptr(fy), _ptr(area))
    return fx, fy, area


MAP_CARTESIAN, MAP_LOGPOLAR, MAP_DISC = 0, 1, 3


def pseudo_points(n, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    """Unit-square points index+1 .. index+n of the pseudo-random frequency
    stream (Philox4x32-10 in its own counter domain)."""
    ux, uy = np.zeros(n), np.zeros(n)
    _load().oracle_pseudo_points(seed_x, seed_y, index, n, _ptr(ux), _ptr(uy))
    return ux, uy


def sample_pseudo(map_, n_sets, K, N=0, df=0.0, fmin=0.0, fmax=0.0, index=0, seed_x=SEED_HALF,
                  seed_y=SEED_HALF):
    """Fully random frequencies (Sec. 3.1) through the Cartesian (map 0),
    log-polar (1) or disc (3) map."""
    n = n_sets * K
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_pseudo(map_, seed_x, seed_y, index, n_sets, K, N, df, fmin, fmax,
                                 _ptr(fx), _ptr(fy), _ptr(area))
    return fx, fy, area


def sample_jitter(n_sets, N, df, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    """Randomly jittered grid of Eq. 4: one point per df x df cell of the
    N x N grid centred on the origin (K = N^2)."""
    n = n_sets * N * N
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_jitter(seed_x, seed_y, index, n_sets, N, df, _ptr(fx), _ptr(fy),
                                 _ptr(area))
    return fx, fy, area


def point_set_measures(fx, fy, n_sets, K, x0, y0, Lx, Ly, r_clash):
    """Per set: (minimum pairwise distance, pairs closer than r_clash, L2
    star discrepancy) of the points mapped to the unit square."""
    fx, fy = _f64(fx), _f64(fy)
    md, T = np.zeros(n_sets), np.zeros(n_sets)
    nc = np.zeros(n_sets, dtype=np.int64)
    _load().oracle_point_set_measures(n_sets, K, _ptr(fx), _ptr(fy), x0, y0, Lx, Ly, r_clash,
                                      _ptr(md), nc.ctypes.data_as(ctypes.c_void_p), _ptr(T))
    return md, nc, T


def set_sf_expectation(fx, fy, w, n_sets, K, bx, by):
    """Noise-free differential-piston structure function of each set,
    [n_sets][nB]: sum_k w_k^2 2 (1 - cos 2 pi f_k.B)."""
    fx, fy, w, bx, by = map(_f64, (fx, fy, w, bx, by))
    S = np.zeros((n_sets, bx.size))
    _load().oracle_set_sf_expectation(K, _ptr(fx), _ptr(fy), _ptr(w), n_sets, bx.size, _ptr(bx),
                                      _ptr(by), _ptr(S))
    return S


def choose_cartesian(df, eps, r0=0.1, L0=25.0, D=None, d=0.0, c=None, model=PSD_VON_KARMAN,
                     wavelength=0.0):
    """Stopping rule for N (Sec. 4.3): returns (N, sigma^2) with N df = 2 max f
    (N = -1: not settled within the integration range)."""
    c = psd_constant() if c is None else c
    s2 = ctypes.c_double(0.0)
    N = _load().oracle_choose_cartesian(model, c, r0, L0, 0 if D is None else 1,
                                        0.0 if D is None else D, d, df, eps, wavelength,
                                        ctypes.byref(s2))
    return int(N), s2.value


def psd_constant():
    return _load().oracle_psd_constant()


def psd(f, model=PSD_VON_KARMAN, c=None, r0=0.1, L0=25.0):
    c = psd_constant() if c is None else c
    lib = _load()
    f = np.atleast_1d(np.asarray(f, dtype=np.float64))
    return np.array([lib.oracle_psd(model, c, r0, L0, float(x)) for x in f])


def aperture_filter(f, D, d=0.0):
    lib = _load()
    f = np.atleast_1d(np.asarray(f, dtype=np.float64))
    return np.array([lib.oracle_aperture_filter(D, d, float(x)) for x in f])


def weights(fx, fy, area, model=PSD_VON_KARMAN, c=None, r0=0.1, L0=25.0, D=None, d=0.0,
            wavelength=0.0):
    c = psd_constant() if c is None else c
    fx, fy, area = _f64(fx), _f64(fy), _f64(area)
    w = np.zeros(fx.size)
    has_ap = 0 if D is None else 1
    _load().oracle_weights(model, c, r0, L0, has_ap, D or 0.0, d, wavelength, fx.size, _ptr(fx),
                           _ptr(fy), _ptr(area), _ptr(w))
    return w


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def coefficients(seed, realisation, K, mode=COEF_GAUSS_CS):
    c = np.zeros(2 * K)
    _load().oracle_coefficients(seed, realisation, K, mode, _ptr(c))
    return c


def synthesize(fx, fy, w, px, py, R, R_block, K=None, seed=0, counter=0,
               mode=COEF_GAUSS_CS, coef=None):
    fx, fy, w, px, py = map(_f64, (fx, fy, w, px, py))
    K = fx.size if K is None else K
    coef = None if coef is None else _f64(coef)
    out = np.zeros((R, px.size))
    _load().oracle_synthesize(K, _ptr(fx), _ptr(fy), _ptr(w), px.size, _ptr(px), _ptr(py), R,
                              R_block, seed, counter, mode, _ptr(coef), _ptr(out))
    return out


def piston(fx, fy, w, cx, cy, D, d, R, R_block, K=None, seed=0, counter=0,
           mode=COEF_GAUSS_CS, coef=None):
    fx, fy, w, cx, cy = map(_f64, (fx, fy, w, cx, cy))
    D = _f64(np.broadcast_to(D, cx.shape))
    d = _f64(np.broadcast_to(d, cx.shape))
    K = fx.size if K is None else K
    coef = None if coef is None else _f64(coef)
    out = np.zeros((R, cx.size))
    _load().oracle_piston(K, _ptr(fx), _ptr(fy), _ptr(w), cx.size, _ptr(cx), _ptr(cy), _ptr(D),
                          _ptr(d), R, R_block, seed, counter, mode, _ptr(coef), _ptr(out))
    return out


def tilt(fx, fy, w, cx, cy, D, d, R, R_block, axis=0, K=None, seed=0, counter=0,
         mode=COEF_GAUSS_CS, coef=None):
    """Aperture-averaged phase gradient (G-tilt, rad/m) along axis 0 (x) or
    1 (y) at each aperture, [R][n_ap]; w is the unfiltered phase weight."""
    fx, fy, w, cx, cy, D, d = map(_f64, (fx, fy, w, cx, cy, D, d))
    K = fx.size if K is None else K
    coef = None if coef is None else _f64(coef)
    out = np.zeros((R, cx.size))
    _load().oracle_tilt(K, _ptr(fx), _ptr(fy), _ptr(w), cx.size, _ptr(cx), _ptr(cy), _ptr(D),
                        _ptr(d), R, R_block, seed, counter, mode, _ptr(coef), axis, _ptr(out))
    return out


def diff_piston_sf(fx, fy, w, bx, by, R, R_block, K=None, seed=0, counter=0,
                   mode=COEF_GAUSS_CS):
    fx, fy, w, bx, by = map(_f64, (fx, fy, w, bx, by))
    K = fx.size if K is None else K
    sf = np.zeros(bx.size)
    se = np.zeros(bx.size)
    _load().oracle_diff_piston_sf(K, _ptr(fx), _ptr(fy), _ptr(w), bx.size, _ptr(bx), _ptr(by),
                                  R, R_block, seed, counter, mode, _ptr(sf), _ptr(se))
    return sf, se


def temporal_sf(pist):
    """Time-lag structure function of the differential piston (Sec. 4.4):
    pist [R][2][M] pistons of telescopes 1, 2 at t_m = m dt; returns
    (sf[M], sf_stderr[M]) averaged over pairs and realisations."""
    pist = np.ascontiguousarray(np.asarray(pist, dtype=np.float64))
    R, two, M = pist.shape
    assert two == 2
    sf, se = np.zeros(M), np.zeros(M)
    _load().oracle_temporal_sf(_ptr(pist), R, M, _ptr(sf), _ptr(se))
    return sf, se


def temporal_experiment(fx, fy, w, c1, c2, v, dt, M, R, R_block, K=None, seed=0, counter=0,
                        mode=COEF_GAUSS_CS):
    """Frozen-flow pistons at c1 - v t_m and c2 - v t_m (t_m = m dt) with the
    aperture-filtered weights w, then temporal_sf."""
    fx, fy, w = map(_f64, (fx, fy, w))
    c1, c2, v = (_f64(np.asarray(x, dtype=np.float64)) for x in (c1, c2, v))
    K = fx.size if K is None else K
    sf, se = np.zeros(M), np.zeros(M)
    _load().oracle_temporal_experiment(K, _ptr(fx), _ptr(fy), _ptr(w), _ptr(c1), _ptr(c2),
                                       _ptr(v), float(dt), M, R, R_block, seed, counter, mode,
                                       _ptr(sf), _ptr(se))
    return sf, se


# ------------------------------------------------------ learned proposal
def mlp_param_count(H=128):
    return int(_load().oracle_mlp_param_count(H))


def mlp_forward(prm, ell, ctx, lmin, Lw, H=128):
    prm, ell = _f64(prm), _f64(ell)
    ctx = _f64(np.broadcast_to(np.asarray(ctx, dtype=np.float64), (ell.size, 4)))
    out = np.zeros((ell.size, 2))
    _load().oracle_mlp_forward(_ptr(prm), H, lmin, Lw, ell.size, _ptr(ell), _ptr(ctx), _ptr(out))
    return out


def mlp_loss_grad(prm, ctx, ell, theta, h, lmin, Lw, G=64, H=128):
    prm, ctx, ell, theta, h = map(_f64, (prm, ctx, ell, theta, h))
    n_ctx = ctx.size // 4
    m = ell.size // n_ctx
    grad = np.zeros(prm.size)
    loss = _load().oracle_mlp_loss_grad(_ptr(prm), H, lmin, Lw, n_ctx, m, _ptr(ctx), _ptr(ell),
                                        _ptr(theta), _ptr(h), G, _ptr(grad))
    return loss, grad


def proposal_rows(ctx, m, r0, fmin, fmax, index=0, c=None, s0x=SEED_HALF, s0y=SEED_HALF):
    ctx = _f64(ctx)
    n = ctx.size // 4 * m
    ell, theta, h = np.zeros(n), np.zeros(n), np.zeros(n)
    c = psd_constant() if c is None else c
    _load().oracle_proposal_rows(s0x, s0y, index, ctx.size // 4, m, _ptr(ctx), r0, c, fmin, fmax,
                                 _ptr(ell), _ptr(theta), _ptr(h))
    return ell, theta, h


def proposal_table(prm, D, L0, bl, bth, fmin, fmax, n_cells=256, beta=0.1, H=128):
    prm, bl, bth = _f64(prm), _f64(bl), _f64(bth)
    p, al, ph, cdf = (np.zeros(n_cells) for _ in range(4))
    _load().oracle_proposal_table(_ptr(prm), H, np.log(fmin), np.log(fmax / fmin), n_cells, D, L0,
                                  bl.size, _ptr(bl), _ptr(bth), beta, _ptr(p), _ptr(al), _ptr(ph),
                                  _ptr(cdf))
    return p, al, ph, cdf


def sample_learned(table, n_sets, K, fmin, fmax, index=0, s0x=SEED_HALF, s0y=SEED_HALF):
    p, al, ph, cdf = map(_f64, table)
    n = n_sets * K
    fx, fy, area = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().oracle_sample_learned(s0x, s0y, index, n_sets, K, np.log(fmin), np.log(fmax / fmin),
                                  p.size, _ptr(p), _ptr(al), _ptr(ph), _ptr(cdf), _ptr(fx),
                                  _ptr(fy), _ptr(area))
    return fx, fy, area
