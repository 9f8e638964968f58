"""Python binding of libqrfs: quasi-random frequency sampling for optical
turbulence (arXiv 2404.02978) on AMD Instinct MI355X (gfx950).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libqrfs.so``; torch provides device memory and the current stream.
The functions mirror the C ABI in ``include/qrfs.h`` (same names without the
``qrfs_`` prefix).  If the library is missing or no GPU is present, calls
raise immediately; there is no CPU fallback.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqrfs.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_OUT_OF_MEMORY = -2
ERR_DEVICE = -3
ERR_UNSUPPORTED = -4
ERR_NOT_CONVERGED = -5

PSD_KOLMOGOROV = 0
PSD_VON_KARMAN = 1
SAMPLER_R2_CARTESIAN = 0
SAMPLER_R2_LOGPOLAR = 1
SAMPLER_LEARNED = 2
SAMPLER_R2_DISC = 3
SAMPLER_JITTER = 4
SAMPLER_RANDOM_CARTESIAN = 5
SAMPLER_RANDOM_LOGPOLAR = 6
SAMPLER_RANDOM_DISC = 7
COEF_GAUSS_CS = 0
COEF_EQ3 = 1
PREC_FP64 = 0
PREC_FP32 = 1
PREC_SPLIT_BF16 = 2
PREC_BF16X6 = 3
PREC_FP16X3 = 4
SEED_HALF = 1 << 63


class QrfsError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"qrfs status {status}: {detail}")
        self.status = status
        self.detail = detail


class Psd(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("c", ctypes.c_double), ("r0", ctypes.c_double),
                ("L0", ctypes.c_double), ("wavelength", ctypes.c_double)]


class Aperture(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("d", ctypes.c_double)]


class Sampler(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("N", ctypes.c_int32), ("df", ctypes.c_double),
                ("fmin", ctypes.c_double), ("fmax", ctypes.c_double),
                ("seed_x", ctypes.c_uint64), ("seed_y", ctypes.c_uint64),
                ("index", ctypes.c_uint64), ("proposal", ctypes.c_void_p)]


class Rng(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("counter", ctypes.c_uint64), ("mode", ctypes.c_int32)]


class BatchInstance(ctypes.Structure):
    _fields_ = [("psd", Psd), ("sampler", Sampler), ("K", ctypes.c_int64), ("P", ctypes.c_int64),
                ("px", ctypes.c_void_p), ("py", ctypes.c_void_p), ("R", ctypes.c_int64),
                ("R_block", ctypes.c_int64), ("rng", Rng), ("phase", ctypes.c_void_p),
                ("apD", ctypes.c_void_p), ("apd", ctypes.c_void_p), ("ux", ctypes.c_double),
                ("uy", ctypes.c_double)]


def psd(r0, L0=None, model=None, c=0.0, wavelength=0.0):
    """Phase PSD; r0 at `wavelength`.  wavelength > 0 (m) makes every
    PSD-weighted output optical path (m, m^2) instead of phase (rad, rad^2)."""
    if model is None:
        model = PSD_KOLMOGOROV if L0 is None else PSD_VON_KARMAN
    return Psd(model, c, r0, 0.0 if L0 is None else L0, wavelength)


def logpolar_sampler(fmin, fmax, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    return Sampler(SAMPLER_R2_LOGPOLAR, 0, 0.0, fmin, fmax, seed_x, seed_y, index, None)


def disc_sampler(fmax, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    """Polar quasi-random frequencies on the disc |f| < fmax (Sec. 3.2)."""
    return Sampler(SAMPLER_R2_DISC, 0, 0.0, 0.0, fmax, seed_x, seed_y, index, None)


def choose_cartesian(psd_, aperture=None, df=0.0, eps=1e-4):
    """Cartesian hyper-parameters by the stopping rule of Sec. 4.3 (host
    only): returns (N, df, sigma2)."""
    N = _I32(0)
    dfo = ctypes.c_double(0.0)
    s2 = ctypes.c_double(0.0)
    _check(load_library().qrfs_choose_cartesian(
        ctypes.byref(psd_), None if aperture is None else ctypes.byref(aperture), float(df),
        float(eps), ctypes.byref(N), ctypes.byref(dfo), ctypes.byref(s2)))
    return N.value, dfo.value, s2.value


def cartesian_sampler(N, df, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    return Sampler(SAMPLER_R2_CARTESIAN, N, df, 0.0, 0.0, seed_x, seed_y, index, None)


def jitter_sampler(N, df, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    """Randomly jittered grid of Eq. 4 (K must be N^2); seed_x is the
    Philox key, the low word of seed_y the stream id."""
    return Sampler(SAMPLER_JITTER, N, df, 0.0, 0.0, seed_x, seed_y, index, None)


def random_sampler(scheme, N=0, df=0.0, fmin=0.0, fmax=0.0, index=0, seed_x=SEED_HALF,
                   seed_y=SEED_HALF):
    """Fully random frequencies (Sec. 3.1) through the Cartesian, log-polar
    or disc map: scheme SAMPLER_RANDOM_CARTESIAN / _LOGPOLAR / _DISC."""
    return Sampler(scheme, N, df, fmin, fmax, seed_x, seed_y, index, None)


def learned_sampler(proposal, index=0, seed_x=SEED_HALF, seed_y=SEED_HALF):
    """R2 points warped through the sampling table of `proposal`."""
    return Sampler(SAMPLER_LEARNED, 0, 0.0, proposal.fmin, proposal.fmax, seed_x, seed_y, index,
                   proposal.handle.value)


PROPOSAL_NPARAM = 17538


BATCH_SHAPES = 5
BATCH_SHAPE_TWO_PHASE = 4

TUNE_WIDE_PATH = 1
TUNE_RANGE_FREQS = 2
TUNE_TILE_BYTES = 3

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def load_library():
    """Loads libqrfs.so (built by ``paper_2404_02978_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2404_02978_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_int32
    sig = {
        "qrfs_error_string": (ctypes.c_char_p, [S]),
        "qrfs_last_error_detail": (ctypes.c_char_p, []),
        "qrfs_abi_version": (ctypes.c_int32, []),
        "qrfs_context_create": (S, [ctypes.POINTER(_P), _I32, ctypes.c_size_t]),
        "qrfs_context_destroy": (S, [_P]),
        "qrfs_context_set_tuning": (S, [_P, _I32, _I64]),
        "qrfs_choose_cartesian": (S, [ctypes.POINTER(Psd), ctypes.POINTER(Aperture), ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(_I32),
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
        "qrfs_sample_frequencies": (S, [_P, ctypes.POINTER(Sampler), _I64, _I64, _P, _P, _P, _P]),
        "qrfs_weights": (S, [_P, ctypes.POINTER(Psd), ctypes.POINTER(Aperture), _I64, _P, _P, _P,
                             _I32, _P, _P]),
        "qrfs_sample_weights": (S, [_P, ctypes.POINTER(Sampler), _I64, _I64, ctypes.POINTER(Psd),
                                    ctypes.POINTER(Aperture), _I32, _P, _P, _P, _P]),
        "qrfs_synthesize_phase": (S, [_P, _I64, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                      ctypes.POINTER(Rng), _P, _I32, _P, _P]),
        "qrfs_piston": (S, [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _I64, _I64,
                            ctypes.POINTER(Rng), _P, _I32, _P, _P]),
        "qrfs_tilt": (S, [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, ctypes.c_double,
                          ctypes.c_double, _I64, _I64, ctypes.POINTER(Rng), _P, _I32, _P, _P]),
        "qrfs_diff_piston": (S, [_P, _I64, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                 ctypes.POINTER(Rng), _P, _I32, _P, _P]),
        "qrfs_diff_piston_structure_sets": (S, [_P, _I64, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                                ctypes.POINTER(Rng), _I32, _P, _P, _P]),
        "qrfs_diff_piston_structure": (S, [_P, ctypes.POINTER(Psd), ctypes.POINTER(Aperture), _I64,
                                           _P, _P, ctypes.POINTER(Sampler), _I64, _I64, _I64,
                                           ctypes.POINTER(Rng), _I32, _P, _P, _P]),
        "qrfs_temporal_sf": (S, [_P, _I64, _I64, _I32, _P, _P, _P, _P]),
        "qrfs_point_set_measures": (S, [_P, _I64, _I64, _P, _P, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _P, _P, _P, _P]),
        "qrfs_set_sf_expectation": (S, [_P, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P, _P]),
        "qrfs_temporal_piston_structure": (
            S, [_P, ctypes.POINTER(Psd), ctypes.POINTER(Aperture), ctypes.POINTER(ctypes.c_double),
                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                _I64, ctypes.POINTER(Sampler), _I64, _I64, _I64, ctypes.POINTER(Rng), _I32, _P, _P,
                _P]),
    }
    _D = ctypes.c_double
    sig.update({
        "qrfs_proposal_create": (S, [_P, _D, _D, _P, ctypes.POINTER(_P)]),
        "qrfs_proposal_destroy": (S, [_P]),
        "qrfs_proposal_get_params": (S, [_P, _P, _P]),
        "qrfs_proposal_set_params": (S, [_P, _P, _P]),
        "qrfs_proposal_forward": (S, [_P, _I64, _P, _P, _P, _P]),
        "qrfs_proposal_rows": (S, [_P, ctypes.POINTER(Sampler), _I64, _I64, _P, _D, _D, _P, _P, _P,
                                   _P]),
        "qrfs_proposal_loss_grad": (S, [_P, _I64, _I64, _P, _P, _P, _P, _I32, _P, _P, _P]),
        "qrfs_proposal_train": (S, [_P, _I64, _I64, _P, _P, _P, _P, _I64, _I64, _I32, _D,
                                    ctypes.c_uint64, _P, _P]),
        "qrfs_proposal_tabulate": (S, [_P, _D, _D, _I64, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                       _I32, _D, _P]),
        "qrfs_proposal_get_table": (S, [_P, ctypes.POINTER(_I32), _P, _P, _P, _P, _P]),
        "qrfs_proposal_set_table": (S, [_P, _I32, _P, _P, _P, _P, _P]),
        "qrfs_proposal_save": (S, [_P, ctypes.c_char_p]),
        "qrfs_proposal_load": (S, [_P, ctypes.c_char_p]),
    })
    sig.update({
        "qrfs_batch_create": (S, [_P, _I64, ctypes.POINTER(BatchInstance), _I32,
                                  ctypes.POINTER(_P)]),
        "qrfs_batch_autotune": (S, [_P, _P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]),
        "qrfs_batch_execute": (S, [_P, _I32, _P]),
        "qrfs_batch_set_shape": (S, [_P, _I32]),
        "qrfs_batch_info": (S, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                ctypes.POINTER(ctypes.c_double)]),
        "qrfs_batch_destroy": (S, [_P]),
    })
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != OK:
        lib = load_library()
        raise QrfsError(status, lib.qrfs_last_error_detail().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, name, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns a libqrfs context (device workspace) on one HIP device."""

    def __init__(self, device=0, workspace_cap=0):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libqrfs needs an MI355X")
        self.device = torch.device("cuda", device)
        h = _P()
        _check(lib.qrfs_context_create(ctypes.byref(h), device, int(workspace_cap)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().qrfs_context_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_tuning(self, key, value):
        """Launch policy: TUNE_WIDE_PATH (0 auto, 1 fused kernel, 2 two-phase
        kernel), TUNE_RANGE_FREQS, TUNE_TILE_BYTES (see include/qrfs.h)."""
        _check(load_library().qrfs_context_set_tuning(self._h, int(key), int(value)))

    # ---------------------------------------------------------------- API
    def sample_frequencies(self, sampler, n_sets, K):
        """R2 sampling (Sec. 3.2); returns (fx, fy, area) float64 [n_sets*K];
        advances sampler.index."""
        n = n_sets * K
        fx = torch.empty(n, dtype=torch.float64, device=self.device)
        fy = torch.empty_like(fx)
        area = torch.empty_like(fx)
        _check(load_library().qrfs_sample_frequencies(self._h, ctypes.byref(sampler), n_sets, K,
                                                      _ptr(fx), _ptr(fy), _ptr(area), _stream()))
        return fx, fy, area

    def sample_weights(self, sampler, n_sets, K, psd_, aperture=None, precision=PREC_FP64):
        """Sampling and weights in one pass (no cell areas); returns
        (fx, fy, w) float64 [n_sets*K]; advances sampler.index.  precision:
        that of the sums the weights feed (FP64: binary64 weights)."""
        n = n_sets * K
        fx = torch.empty(n, dtype=torch.float64, device=self.device)
        fy = torch.empty_like(fx)
        w = torch.empty_like(fx)
        ap = ctypes.byref(aperture) if aperture is not None else None
        _check(load_library().qrfs_sample_weights(self._h, ctypes.byref(sampler), n_sets, K,
                                                  ctypes.byref(psd_), ap, precision, _ptr(fx),
                                                  _ptr(fy), _ptr(w), _stream()))
        return fx, fy, w

    def weights(self, psd_, fx, fy, area, aperture=None, precision=PREC_FP64):
        n = fx.numel()
        w = torch.empty(n, dtype=torch.float64, device=self.device)
        ap = ctypes.byref(aperture) if aperture is not None else None
        _check(load_library().qrfs_weights(self._h, ctypes.byref(psd_), ap, n,
                                           _dev_f64(fx, "fx"), _dev_f64(fy, "fy", n),
                                           _dev_f64(area, "area", n), precision, _ptr(w),
                                           _stream()))
        return w

    def _out(self, R, P, precision):
        dt = torch.float64 if precision == PREC_FP64 else torch.float32
        return torch.empty((R, P), dtype=dt, device=self.device)

    @staticmethod
    def _rng(rng, coef):
        if coef is not None:
            return None
        return ctypes.byref(rng if rng is not None else Rng(0, 0, COEF_GAUSS_CS))

    def synthesize_phase(self, K, fx, fy, w, px, py, R, R_block, rng=None, coef=None,
                         precision=PREC_FP32, out=None):
        n_sets = math.ceil(R / R_block)
        P = px.numel()
        out = self._out(R, P, precision) if out is None else out
        _check(load_library().qrfs_synthesize_phase(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), P, _dev_f64(px, "px"), _dev_f64(py, "py", P), R, R_block,
            self._rng(rng, coef), None if coef is None else _dev_f64(coef, "coef", R * 2 * K),
            precision, _ptr(out), _stream()))
        return out

    def piston(self, K, fx, fy, w, cx, cy, apD, apd, R, R_block, rng=None, coef=None,
               precision=PREC_FP32, out=None):
        n_sets = math.ceil(R / R_block)
        n_ap = cx.numel()
        out = self._out(R, n_ap, precision) if out is None else out
        _check(load_library().qrfs_piston(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), n_ap, _dev_f64(cx, "cx"), _dev_f64(cy, "cy", n_ap),
            _dev_f64(apD, "apD", n_ap), _dev_f64(apd, "apd", n_ap), R, R_block,
            self._rng(rng, coef), None if coef is None else _dev_f64(coef, "coef", R * 2 * K),
            precision, _ptr(out), _stream()))
        return out

    def tilt(self, K, fx, fy, w, cx, cy, apD, apd, u, R, R_block, rng=None, coef=None,
             precision=PREC_FP32, out=None):
        """Aperture-averaged phase gradient along u = (ux, uy), rad/m
        (G-tilt; w is the unfiltered phase weight).  [R][n_ap]."""
        n_sets = math.ceil(R / R_block)
        n_ap = cx.numel()
        out = self._out(R, n_ap, precision) if out is None else out
        _check(load_library().qrfs_tilt(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), n_ap, _dev_f64(cx, "cx"), _dev_f64(cy, "cy", n_ap),
            _dev_f64(apD, "apD", n_ap), _dev_f64(apd, "apd", n_ap), float(u[0]), float(u[1]),
            R, R_block, self._rng(rng, coef),
            None if coef is None else _dev_f64(coef, "coef", R * 2 * K), precision, _ptr(out),
            _stream()))
        return out

    def diff_piston(self, K, fx, fy, w, bx, by, R, R_block, rng=None, coef=None,
                    precision=PREC_FP32, out=None):
        n_sets = math.ceil(R / R_block)
        nB = bx.numel()
        out = self._out(R, nB, precision) if out is None else out
        _check(load_library().qrfs_diff_piston(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), nB, _dev_f64(bx, "bx"), _dev_f64(by, "by", nB), R,
            R_block, self._rng(rng, coef),
            None if coef is None else _dev_f64(coef, "coef", R * 2 * K), precision, _ptr(out),
            _stream()))
        return out

    def diff_piston_structure(self, psd_, aperture, bx, by, sampler, K, R, R_block, rng=None,
                              precision=PREC_FP32, with_stderr=True):
        """End-to-end differential-piston structure function (Sec. 4.4).
        Returns (sf, stderr) float64 [nB] on the device; advances sampler.index."""
        nB = bx.numel()
        sf = torch.empty(nB, dtype=torch.float64, device=self.device)
        se = torch.empty_like(sf) if with_stderr else None
        rng = rng if rng is not None else Rng(0, 0, COEF_GAUSS_CS)
        _check(load_library().qrfs_diff_piston_structure(
            self._h, ctypes.byref(psd_), ctypes.byref(aperture), nB, _dev_f64(bx, "bx"),
            _dev_f64(by, "by", nB), ctypes.byref(sampler), K, R, R_block, ctypes.byref(rng),
            precision, _ptr(sf), _ptr(se), _stream()))
        return sf, se

    def point_set_measures(self, fx, fy, n_sets, K, x0, y0, Lx, Ly, r_clash):
        """Per set: minimum pairwise distance, clash count and L2 star
        discrepancy of the points mapped to the unit square (device
        tensors: float64, int64, float64 [n_sets])."""
        md = torch.empty(n_sets, dtype=torch.float64, device=self.device)
        nc = torch.empty(n_sets, dtype=torch.int64, device=self.device)
        T = torch.empty_like(md)
        _check(load_library().qrfs_point_set_measures(
            self._h, n_sets, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            float(x0), float(y0), float(Lx), float(Ly), float(r_clash), _ptr(md), _ptr(nc),
            _ptr(T), _stream()))
        return md, nc, T

    def set_sf_expectation(self, K, fx, fy, w, n_sets, bx, by):
        """Noise-free differential-piston structure function of each set,
        float64 [n_sets][nB] on the device."""
        nB = bx.numel()
        S = torch.empty((n_sets, nB), dtype=torch.float64, device=self.device)
        _check(load_library().qrfs_set_sf_expectation(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), n_sets, nB, _dev_f64(bx, "bx"), _dev_f64(by, "by", nB),
            _ptr(S), _stream()))
        return S

    def temporal_sf(self, pistons, with_stderr=True):
        """Time-lag structure function of the differential piston (Sec. 4.4)
        from pistons [R][2][M] (float64 -> FP64 path, float32 otherwise).
        Returns (sf, stderr) float64 [M] on the device."""
        if not isinstance(pistons, torch.Tensor) or not pistons.is_cuda or pistons.dim() != 3 \
                or pistons.shape[1] != 2 or not pistons.is_contiguous():
            raise TypeError("pistons must be a contiguous CUDA tensor [R][2][M]")
        if pistons.dtype not in (torch.float64, torch.float32):
            raise TypeError("pistons must be float64 or float32")
        R, _, M = pistons.shape
        prec = PREC_FP64 if pistons.dtype == torch.float64 else PREC_FP32
        sf = torch.empty(M, dtype=torch.float64, device=self.device)
        se = torch.empty_like(sf) if with_stderr else None
        _check(load_library().qrfs_temporal_sf(self._h, R, M, prec, _ptr(pistons), _ptr(sf),
                                               _ptr(se), _stream()))
        return sf, se

    def temporal_piston_structure(self, psd_, aperture, c1, c2, v, dt, M, sampler, K, R,
                                  R_block, rng=None, precision=PREC_FP32, with_stderr=True):
        """The frozen-flow experiment of Sec. 4.4 end to end: telescopes at
        c1, c2 (m), wind v (m/s), M samples dt apart.  Returns (sf, stderr)
        float64 [M] (rad^2) on the device; advances sampler.index."""
        D2 = ctypes.c_double * 2
        sf = torch.empty(M, dtype=torch.float64, device=self.device)
        se = torch.empty_like(sf) if with_stderr else None
        rng = rng if rng is not None else Rng(0, 0, COEF_GAUSS_CS)
        _check(load_library().qrfs_temporal_piston_structure(
            self._h, ctypes.byref(psd_), ctypes.byref(aperture), D2(*c1), D2(*c2), D2(*v),
            float(dt), M, ctypes.byref(sampler), K, R, R_block, ctypes.byref(rng), precision,
            _ptr(sf), _ptr(se), _stream()))
        return sf, se

    def diff_piston_structure_sets(self, K, fx, fy, w, bx, by, R, R_block, rng=None,
                                   precision=PREC_FP32, with_stderr=True, sf=None, se=None):
        """Structure function from caller-supplied frequency sets (w carries
        the aperture filter).  Returns (sf, stderr) float64 [nB] on the device."""
        n_sets = math.ceil(R / R_block)
        nB = bx.numel()
        sf = torch.empty(nB, dtype=torch.float64, device=self.device) if sf is None else sf
        if with_stderr and se is None:
            se = torch.empty_like(sf)
        rng = rng if rng is not None else Rng(0, 0, COEF_GAUSS_CS)
        _check(load_library().qrfs_diff_piston_structure_sets(
            self._h, K, _dev_f64(fx, "fx", n_sets * K), _dev_f64(fy, "fy", n_sets * K),
            _dev_f64(w, "w", n_sets * K), nB, _dev_f64(bx, "bx"), _dev_f64(by, "by", nB), R,
            R_block, ctypes.byref(rng), precision, _ptr(sf), _ptr(se if with_stderr else None),
            _stream()))
        return sf, se


class Batch:
    """Many uneven instances in one persistent launch.

    instances: list of dicts with keys psd, sampler, K, px, py (float64 CUDA
    tensors), R, R_block, rng; optional apD, apd (float64 CUDA tensors [P]:
    pistons of apertures centred at the points instead of the phase) and u
    (with apertures: G-tilts along u instead of pistons).  Outputs are
    allocated here (float32 [R][P]).
    """

    def __init__(self, ctx, instances, precision=PREC_BF16X6):
        lib = load_library()
        self.ctx = ctx
        self.outputs = []
        self._keep = []
        arr = (BatchInstance * len(instances))()
        for i, d in enumerate(instances):
            px, py = d["px"], d["py"]
            P = px.numel()
            out = torch.empty((d["R"], P), dtype=torch.float32, device=ctx.device)
            self.outputs.append(out)
            self._keep += [px, py]
            apD, apd = d.get("apD"), d.get("apd")
            if apD is not None:
                self._keep += [apD, apd]
            ux, uy = d.get("u", (0.0, 0.0))
            arr[i] = BatchInstance(d["psd"], d["sampler"], d["K"], P, _dev_f64(px, "px"),
                                   _dev_f64(py, "py", P), d["R"], d.get("R_block", d["R"]),
                                   d.get("rng", Rng(0, 0, COEF_GAUSS_CS)), _ptr(out),
                                   None if apD is None else _dev_f64(apD, "apD", P),
                                   None if apd is None else _dev_f64(apd, "apd", P),
                                   float(ux), float(uy))
        h = _P()
        _check(lib.qrfs_batch_create(ctx.handle, len(instances), arr, precision, ctypes.byref(h)))
        self._h = h

    def autotune(self, cache_path=None):
        """Times the launch shapes and keeps the fastest; with cache_path, a
        batch of the same sizes tuned before reuses the stored choice."""
        ms = ctypes.c_double(0.0)
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load_library().qrfs_batch_autotune(self._h, _stream(), path, ctypes.byref(ms)))
        return ms.value

    def execute(self, use_graph=False):
        _check(load_library().qrfs_batch_execute(self._h, 1 if use_graph else 0, _stream()))
        return self.outputs

    def set_shape(self, shape):
        """Launch shape 0..BATCH_SHAPES-1 (4 = two-phase)."""
        _check(load_library().qrfs_batch_set_shape(self._h, int(shape)))

    def info(self):
        n = _I64(0)
        shape = _I32(0)
        terms = ctypes.c_double(0.0)
        _check(load_library().qrfs_batch_info(self._h, ctypes.byref(n), ctypes.byref(shape),
                                              ctypes.byref(terms)))
        return {"n_items": n.value, "shape": shape.value, "terms": terms.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().qrfs_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Proposal:
    """Learned proposal density of the frequency sampler (see qrfs.h)."""

    def __init__(self, ctx, fmin, fmax, init_params):
        lib = load_library()
        self.ctx = ctx
        self.fmin, self.fmax = float(fmin), float(fmax)
        init = torch.as_tensor(init_params, dtype=torch.float32).to(ctx.device).contiguous()
        if init.numel() != PROPOSAL_NPARAM:
            raise ValueError(f"need {PROPOSAL_NPARAM} parameters")
        h = _P()
        _check(lib.qrfs_proposal_create(ctx.handle, self.fmin, self.fmax, _ptr(init),
                                        ctypes.byref(h)))
        torch.cuda.synchronize()
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self):
        out = torch.empty(PROPOSAL_NPARAM, dtype=torch.float32, device=self.ctx.device)
        _check(load_library().qrfs_proposal_get_params(self._h, _ptr(out), _stream()))
        return out

    def set_params(self, prm):
        prm = torch.as_tensor(prm, dtype=torch.float32).to(self.ctx.device).contiguous()
        _check(load_library().qrfs_proposal_set_params(self._h, _ptr(prm), _stream()))
        torch.cuda.synchronize()

    def forward(self, ell, ctx4):
        n = ell.numel()
        out = torch.empty((n, 2), dtype=torch.float32, device=self.ctx.device)
        _check(load_library().qrfs_proposal_forward(self._h, n, _dev_f64(ell, "ell"),
                                                    _dev_f64(ctx4, "ctx4", 4 * n), _ptr(out),
                                                    _stream()))
        return out

    def rows(self, plain_sampler, ctx4, m, r0, c_psd=0.0):
        n_ctx = ctx4.numel() // 4
        n = n_ctx * m
        ell = torch.empty(n, dtype=torch.float64, device=self.ctx.device)
        theta, h = torch.empty_like(ell), torch.empty_like(ell)
        _check(load_library().qrfs_proposal_rows(self._h, ctypes.byref(plain_sampler), n_ctx, m,
                                                 _dev_f64(ctx4, "ctx4"), r0, c_psd, _ptr(ell),
                                                 _ptr(theta), _ptr(h), _stream()))
        return ell, theta, h

    def loss_grad(self, ctx4, ell, theta, h, G=64):
        n_ctx = ctx4.numel() // 4
        m = ell.numel() // n_ctx
        grad = torch.empty(PROPOSAL_NPARAM, dtype=torch.float32, device=self.ctx.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.ctx.device)
        _check(load_library().qrfs_proposal_loss_grad(
            self._h, n_ctx, m, _dev_f64(ctx4, "ctx4"), _dev_f64(ell, "ell"),
            _dev_f64(theta, "theta"), _dev_f64(h, "h"), G, _ptr(grad), _ptr(loss), _stream()))
        return float(loss.item()), grad

    def train(self, ctx4, ell, theta, h, steps, ctx_per_step=16, G=64, lr=1e-3, seed=0):
        n_ctx = ctx4.numel() // 4
        m = ell.numel() // n_ctx
        log = torch.empty(steps, dtype=torch.float64, device=self.ctx.device)
        _check(load_library().qrfs_proposal_train(
            self._h, n_ctx, m, _dev_f64(ctx4, "ctx4"), _dev_f64(ell, "ell"),
            _dev_f64(theta, "theta"), _dev_f64(h, "h"), ctx_per_step, steps, G, lr, seed,
            _ptr(log), _stream()))
        return log

    def tabulate(self, D, L0, blen, bth, n_cells=256, beta=0.1):
        import numpy as np
        bl = np.ascontiguousarray(blen, dtype=np.float64)
        bt = np.ascontiguousarray(bth, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load_library().qrfs_proposal_tabulate(
            self._h, D, L0, bl.size, bl.ctypes.data_as(dp), bt.ctypes.data_as(dp), n_cells, beta,
            _stream()))

    def get_table(self):
        n = _I32(0)
        lib = load_library()
        _check(lib.qrfs_proposal_get_table(self._h, ctypes.byref(n), None, None, None, None,
                                           _stream()))
        t = [torch.empty(n.value, dtype=torch.float64, device=self.ctx.device) for _ in range(4)]
        _check(lib.qrfs_proposal_get_table(self._h, ctypes.byref(n), *[_ptr(x) for x in t],
                                           _stream()))
        return t

    def set_table(self, p, alpha, phi, cdf):
        n = p.numel()
        _check(load_library().qrfs_proposal_set_table(
            self._h, n, _dev_f64(p, "p"), _dev_f64(alpha, "alpha", n), _dev_f64(phi, "phi", n),
            _dev_f64(cdf, "cdf", n), _stream()))

    def save(self, path):
        _check(load_library().qrfs_proposal_save(self._h, str(path).encode()))

    def load(self, path):
        _check(load_library().qrfs_proposal_load(self._h, str(path).encode()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().qrfs_proposal_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
