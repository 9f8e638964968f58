"""Statistical agreement of the synthesized phase with the closed forms, at
a stated confidence (the plain FP64 phase workload: von Karman r0 = 0.1 m,
L0 = 25 m, log-polar R2 K = 1024 over [1e-3, 1e2] cycles/m, 32 x 32 points
over a 1 m square, R = 128, seed 0).

Point pairs within one realisation are correlated, so each realisation's
mean of (phi(x + d) - phi(x))^2 over all pairs at separation d (one bin per
separation of 1..31 pitches along x and along y) is one sample, and the R
samples of a bin are tested with Student's t against:
  * R_block = 1 (fresh frequencies per realisation, as the paper draws
    them): the band-limited von Karman structure function
    4 pi int_fmin^fmax f W(f) (1 - J0(2 pi f r)) df, the exact expectation
    of the estimator (sampling error averages out over the sets);
  * R_block = R (one static set): the set's conditional expectation
    sum_k w_k^2 2 (1 - cos 2 pi f_k.d) (coefficient noise only), and the
    band-limited curve (noise plus the one set's sampling error).
Two-sided 99.9 % over all bins together (Bonferroni over 62 bins)."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import analytic as A
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    q.load_library()
    return q


def bin_means(ph, n=32):
    """Per-realisation mean squared differences: [R][2 axes][n-1 separations]."""
    g = ph.reshape(ph.shape[0], n, n)  # [r][iy][ix]
    out = np.empty((ph.shape[0], 2, n - 1))
    for s in range(1, n):
        out[:, 0, s - 1] = np.mean((g[:, :, s:] - g[:, :, :-s]) ** 2, axis=(1, 2))
        out[:, 1, s - 1] = np.mean((g[:, s:, :] - g[:, :-s, :]) ** 2, axis=(1, 2))
    return out


def t_stats(samples, expected):
    R = samples.shape[0]
    m = samples.mean(axis=0)
    se = samples.std(axis=0, ddof=1) / math.sqrt(R)
    return (m - expected) / se


@pytest.mark.parametrize("R_block", [1, 128])
def test_phase_structure_function_t_test(q, R_block):
    cfg = workloads.phase_fp64()
    K, R = cfg["K"], cfg["R"]
    n_sets = math.ceil(R / R_block)
    with q.Context(0) as ctx:
        s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
        fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
        w = ctx.weights(q.psd(cfg["r0"], cfg["L0"]), fx, fy, area)
        ph = ctx.synthesize_phase(K, fx, fy, w, torch.as_tensor(cfg["px"]).cuda(),
                                  torch.as_tensor(cfg["py"]).cuda(), R, R_block,
                                  rng=q.Rng(cfg["seed"], 0, 0), precision=q.PREC_FP64)
        torch.cuda.synchronize()
        ph = ph.cpu().numpy()
        hfx, hfy, hw = (t.cpu().numpy() for t in (fx, fy, w))
    samples = bin_means(ph)
    pitch = 1.0 / 31.0
    seps = np.arange(1, 32) * pitch
    band = A.sf_band(seps, cfg["r0"], cfg["L0"], cfg["fmin"], cfg["fmax"])
    n_bins = 2 * seps.size
    crit = stats.t.ppf(1.0 - 0.001 / (2 * n_bins), R - 1)
    targets = {"band-limited curve": np.stack([band, band])}
    if R_block == R:
        cond = np.empty((2, seps.size))
        for ax, (ux, uy) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            arg = 2 * np.pi * np.outer(seps, ux * hfx + uy * hfy)
            cond[ax] = (2.0 * (1.0 - np.cos(arg))) @ (hw * hw)
        targets["set's conditional expectation"] = cond
    for name, exp in targets.items():
        t = t_stats(samples, exp)
        rel = samples.mean(axis=0) / exp - 1
        print(f"R_block {R_block} vs {name}: max |t| {np.max(np.abs(t)):.2f} (critical "
              f"{crit:.2f}), relative deviation rms {np.sqrt(np.mean(rel ** 2)):.2%}")
        assert np.all(np.abs(t) < crit), (name, t)
    # the band-limited curve itself against the closed forms it must approach
    assert np.allclose(A.sf_band([0.1], 0.1, 25.0, 1e-3, 1e2)[0], 5.2579, rtol=2e-4)
