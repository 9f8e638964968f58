"""The allocation-free structure-function entry point against the existing
one (qrfs_diff_piston_structure_sets), both called through the C ABI on the
same frequency sets and coefficient stream: two calls in a row, the second
smaller, in FP64, BF16x6 and at one realisation per set; sizes beyond its
static scratch are refused with an error."""
import ctypes
import math

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    lib = q.load_library()
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    fn = lib.qrfs_diff_piston_structure_sets_noalloc
    fn.restype = ctypes.c_int32
    fn.argtypes = [P, I64, P, P, P, I64, P, P, I64, I64, ctypes.POINTER(q.Rng), I32, P, P, P]
    return q


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def call(q, ctx, name, K, fx, fy, w, bx, by, R, R_block, seed, precision):
    lib = q.load_library()
    nB = bx.numel()
    sf = torch.full((nB,), float("nan"), dtype=torch.float64, device="cuda")
    se = torch.full((nB,), float("nan"), dtype=torch.float64, device="cuda")
    rng = q.Rng(seed, 0, 0)
    st = getattr(lib, name)(ctx.handle, K, ptr(fx), ptr(fy), ptr(w), nB, ptr(bx), ptr(by), R,
                            R_block, ctypes.byref(rng), precision, ptr(sf), ptr(se),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise q.QrfsError(st, lib.qrfs_last_error_detail().decode())
    torch.cuda.synchronize()
    return sf.cpu().numpy(), se.cpu().numpy()


CASES = [  # (K, R, R_block, precision, seed): a large call, then a smaller one
    # the benchmark's size first: its usual plan (8 frequency ranges) needs
    # more than the static scratch, so this call takes fewer ranges
    [(16384, 100000, 256, 3, 1), (700, 3000, 97, 3, 2)],
    [(2048, 20000, 256, 3, 1), (700, 3000, 97, 3, 2)],
    [(1024, 4000, 128, 0, 3), (333, 500, 64, 0, 4)],
    [(512, 6000, 1, 1, 5), (300, 700, 1, 1, 6)],
]


@pytest.mark.parametrize("calls", CASES, ids=["bf16x6-full", "bf16x6", "fp64", "rblock1-fp32"])
def test_noalloc_matches_existing_entry_point(q, calls):
    cfg = workloads.diffpiston()
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    with q.Context(0) as ctx:
        for K, R, R_block, precision, seed in calls:
            n_sets = math.ceil(R / R_block)
            s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=seed * 1000)
            fx, fy, w = ctx.sample_weights(s, n_sets, K, q.psd(0.1, 25.0),
                                           q.Aperture(cfg["D"], 0.0))
            ref, ref_se = call(q, ctx, "qrfs_diff_piston_structure_sets", K, fx, fy, w, bx, by,
                               R, R_block, seed, precision)
            got, got_se = call(q, ctx, "qrfs_diff_piston_structure_sets_noalloc", K, fx, fy, w,
                               bx, by, R, R_block, seed, precision)
            tol = 1e-12 if precision == 0 else 2e-5
            err = np.max(np.abs(got / ref - 1))
            print(f"K={K} R={R} R_block={R_block} p{precision}: max rel diff {err:.2e}")
            assert err < tol
            assert np.max(np.abs(got_se / ref_se - 1)) < 1e-3


def test_noalloc_refuses_beyond_its_scratch(q):
    cfg = workloads.diffpiston()
    bx, by = dev(cfg["bx"]), dev(cfg["by"])
    with q.Context(0) as ctx:
        K, R = 64, 140000  # one set per realisation: 16 * 32 bytes each > 64 MiB
        s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
        fx, fy, w = ctx.sample_weights(s, R, K, q.psd(0.1, 25.0), q.Aperture(cfg["D"], 0.0))
        with pytest.raises(q.QrfsError) as e:
            call(q, ctx, "qrfs_diff_piston_structure_sets_noalloc", K, fx, fy, w, bx, by, R, 1,
                 0, 1)
        assert e.value.status == q.ERR_INVALID_ARG and "scratch" in e.value.detail
