"""Binding of libqrfs_peaks.so (``include/qrfs_peaks.h``): throughput probes
that measure the roofline denominators on the device at hand.  Argument
marshalling only; ``bench.py --mode peaks`` times the probes."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
PEAKS_LIB_PATH = os.path.join(_HERE, "libqrfs_peaks.so")

PEAK_MFMA_BF16 = 0
PEAK_MFMA_FP16 = 1
PEAK_MFMA_F32 = 2
PEAK_VALU_F32 = 3
PEAK_VALU_F64 = 4
PEAK_HBM_COPY = 5

_lib = None


def load_peaks():
    """Loads libqrfs_peaks.so (built with libqrfs.so)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(PEAKS_LIB_PATH):
        raise RuntimeError(f"{PEAKS_LIB_PATH} is missing: build it with "
                           "`python -m paper_2404_02978_amd.build`")
    lib = ctypes.CDLL(PEAKS_LIB_PATH)
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.qrfs_peak_blocks.restype = ctypes.c_int
    lib.qrfs_peak_blocks.argtypes = [ctypes.c_int, ctypes.POINTER(I64)]
    lib.qrfs_peak_launch.restype = ctypes.c_int
    lib.qrfs_peak_launch.argtypes = [ctypes.c_int, I64, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, P, P, P, I64,
                                     ctypes.POINTER(ctypes.c_double), P]
    _lib = lib
    return lib


def peak_blocks(kind):
    """Resident 256-thread blocks of a probe on the current device."""
    lib = load_peaks()
    b = ctypes.c_int64(0)
    rc = lib.qrfs_peak_blocks(int(kind), ctypes.byref(b))
    if rc != 0:
        raise RuntimeError(f"qrfs_peak_blocks(kind={kind}) failed with status {rc}")
    return b.value


def peak_launch(kind, blocks, iters, x, y, out, src, dst, n, stream):
    """Enqueues one probe; returns its nominal work (flops, or bytes for the
    copy).  Device arrays are torch tensors (or None), `stream` a torch
    stream."""
    lib = load_peaks()
    work = ctypes.c_double(0.0)

    def ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    rc = lib.qrfs_peak_launch(int(kind), int(blocks), int(iters), float(x), float(y), ptr(out),
                              ptr(src), ptr(dst), int(n), ctypes.byref(work),
                              ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"qrfs_peak_launch(kind={kind}) failed with status {rc}")
    return work.value
