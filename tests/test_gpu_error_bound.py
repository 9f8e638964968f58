"""Rigorous per-element error bound of the MFMA contractions (FP32,
split-BF16, BF16x6, FP16x3; fused and two-phase kernels) against the FP64
oracle.

With the coefficients supplied by the caller (so no generator error), each
term c_rk b_kp of Eq. 3 reaches the FP32 accumulator with
  - operand splitting error: split-BF16 keeps hi.hi + hi.lo + lo.hi of
    operands that bf16 hi + lo represent to 2^-18, so each product is off by
    at most 3 u^2 |c||b| with u = 2^-8 (the dropped lo.lo and both split
    roundings); BF16x6 drops products below 2^-24 of |c||b| on 2^-27
    operands: 6 * 2^-24; FP32 rounds both operands: 2 * 2^-24; FP16x3
    keeps hi.hi + hi.lo + lo.hi of fp16 hi + lo parts that represent each
    (scaled) operand to 2^-22: 3 * 2^-22, plus the fp16 subnormal floor of
    2^-25 per scaled operand, i.e. 2^-25 / scale in real units, where the
    kernel's power-of-two scale puts the largest basis amplitude in
    [2^13, 2^14) and the largest caller coefficient (times 1/4) there too;
  - basis error, absolute in units of the weight: the phase argument reduced
    in FP64 and rounded to binary32 revolutions (2 pi 2^-25), the hardware
    revolution sine/cosine (1.3e-7), the weight rounded to binary32 (2^-24):
    5e-7 |c| w_k in all;
  - FP32 accumulation of N = (products per term) * 2K terms:
    gamma_N = N 2^-24 / (1 - N 2^-24) times the sum of |terms|.
So |phi_gpu - phi_oracle| <= (e_split + gamma_N) sum |c||b| + 5e-7 sum |c| w.
"""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
E_SPLIT = {1: 2 * U32, 2: 3 * 2.0 ** -16, 3: 6 * U32, 4: 3 * 2.0 ** -22}
PRODUCTS = {1: 1, 2: 3, 3: 6, 4: 3}


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    q.load_library()
    return q


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("path", [1, 2])  # 1: fused kernel, 2: two-phase kernel
def test_rigorous_bound(q, precision, path):
    ctx = q.Context(0)
    ctx.set_tuning(q.TUNE_WIDE_PATH, path)
    try:
        K, P, R = 300, 270, 60
        s = q.logpolar_sampler(1e-3, 1e2, index=5)
        fx, fy, area = ctx.sample_frequencies(s, 1, K)
        w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area)
        torch.cuda.synchronize()
        hfx, hfy, hw = (t.cpu().numpy() for t in (fx, fy, w))
        rng = np.random.default_rng(7)
        coef = rng.normal(size=(R, 2 * K))
        px, py = rng.uniform(-3, 3, P), rng.uniform(-3, 3, P)
        out = ctx.synthesize_phase(K, fx, fy, w, dev(px), dev(py), R, R, coef=dev(coef),
                                   precision=precision)
        got = out.double().cpu().numpy()
        ref = oracle.synthesize(hfx, hfy, hw, px, py, R, R, K=K, coef=coef)
        arg = 2 * np.pi * (np.outer(hfx, px) + np.outer(hfy, py))  # [K][P]
        bc = np.abs(hw[:, None] * np.cos(arg))
        bs = np.abs(hw[:, None] * np.sin(arg))
        ca, cb = np.abs(coef[:, 0::2]), np.abs(coef[:, 1::2])  # [R][K]
        s_cb = ca @ bc + cb @ bs
        s_cw = (ca + cb) @ np.broadcast_to(hw[:, None], (K, P))
        N = PRODUCTS[precision] * 2 * K
        gamma = N * U32 / (1 - N * U32)
        bound = (E_SPLIT[precision] + gamma) * s_cb + 5e-7 * s_cw
        if precision == 4:
            # subnormal floors: 2^-25 / scale per operand, scale >= 2^13 / max
            floor_b = 2.0 ** -38 * np.max(hw)
            floor_c = 2.0 ** -38 * np.max(np.abs(coef))
            s_b = np.broadcast_to((bc + bs).sum(axis=0), (R, P))
            bound = bound + 2 * (floor_b * (ca + cb).sum(axis=1)[:, None] + floor_c * s_b)
        err = np.abs(got - ref)
        ratio = np.max(err / bound)
        print(f"p{precision} path{path}: max err/bound {ratio:.3f}, "
              f"max err {np.max(err):.3e}, mean bound {np.mean(bound):.3e}")
        assert np.all(err <= bound)
    finally:
        ctx.close()
