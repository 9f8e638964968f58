"""Frozen-flow temporal structure function of the differential piston (the
statistical test of Sec. 4.4) through the C ABI, against the FP64 oracle and
the exact expectation of the estimator.

Tolerances: the structure function at short lags is the mean square of
small differences of pistons, so errors are stated relative to the largest
value of the curve: 1e-9 (FP64), 1e-4 (FP32, BF16x6), 5e-3 (split-BF16).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A

pytestmark = pytest.mark.gpu

TOL = {0: 1e-9, 1: 1e-4, 2: 5e-3, 3: 1e-4, 4: 1e-4}
# the worked example: UTs (D = 8 m, d = 1.1 m) 56.5 m apart, L0 = 22 m,
# Cartesian R2 with df = 0.25/22 and fmax = 0.25 (N = 44)
D, d, L0, R0 = 8.0, 1.1, 22.0, 0.1


@pytest.fixture(scope="module")
def q():
    import paper_2404_02978_amd as q
    q.load_library()
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_temporal_sf_parity(q, ctx, dtype):
    rng = np.random.default_rng(1)
    R, M = 37, 300  # ragged against the 8-realisation blocks
    p = torch.as_tensor(rng.normal(size=(R, 2, M)), dtype=dtype).cuda()
    sf, se = ctx.temporal_sf(p)
    rsf, rse = oracle.temporal_sf(host(p).reshape(R, 2, M))
    assert host(sf)[0] == 0.0
    assert np.max(np.abs(host(sf) - rsf)) <= 1e-12 * np.max(rsf)
    assert np.max(np.abs(host(se)[1:] / rse[1:] - 1)) < 1e-9


@pytest.mark.parametrize("precision", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("R_block", [1, 7])
def test_temporal_experiment_parity(q, ctx, precision, R_block):
    N, df = 12, 0.5 / 12
    K, R, M, dt = N * N, 45, 200, 0.01
    c1, c2, v = (0.0, 0.0), (56.5, 0.0), (10.2, 2.0)
    n_sets = math.ceil(R / R_block)
    s = q.cartesian_sampler(N, df, index=300)
    print(f"temporal p{precision} Rb{R_block}", flush=True)
    sf, se = ctx.temporal_piston_structure(q.psd(R0, L0), q.Aperture(D, d), c1, c2, v, dt, M, s,
                                           K, R, R_block, rng=q.Rng(3, 11, 0),
                                           precision=precision)
    assert s.index == 300 + n_sets * K
    fx, fy, area = oracle.sample_cartesian(n_sets, K, N, df, index=300)
    w = oracle.weights(fx, fy, area, r0=R0, L0=L0, D=D, d=d)
    rsf, rse = oracle.temporal_experiment(fx, fy, w, c1, c2, v, dt, M, R, R_block, K=K, seed=3,
                                          counter=11)
    e = np.max(np.abs(host(sf) - rsf)) / np.max(rsf)
    print(f"  max err / max sf {e:.3e}")
    assert e <= TOL[precision]


def test_temporal_equals_composed_calls(q, ctx):
    """End to end equals qrfs_synthesize_phase (filtered weights, Taylor
    points) followed by qrfs_temporal_sf on a problem large enough to be cut
    into several pieces of sets (the device forms c - v t with a fused
    multiply-add, so the points may differ from numpy's in the last bit)."""
    N, df = 44, 0.25 / 22
    K, R, M, dt = N * N, 20000, 1024, 0.001
    c1, c2, v = (0.0, 0.0), (56.5, 0.0), (10.2, 0.0)
    s = q.cartesian_sampler(N, df, index=0)
    sf, se = ctx.temporal_piston_structure(q.psd(R0, L0), q.Aperture(D, d), c1, c2, v, dt, M, s,
                                           K, R, 1, rng=q.Rng(0, 0, 0), precision=1)
    s2 = q.cartesian_sampler(N, df, index=0)
    fx, fy, area = ctx.sample_frequencies(s2, R, K)
    w = ctx.weights(q.psd(R0, L0), fx, fy, area, q.Aperture(D, d))
    t = np.arange(M) * dt
    px = np.concatenate([c1[0] - v[0] * t, c2[0] - v[0] * t])
    py = np.concatenate([c1[1] - v[1] * t, c2[1] - v[1] * t])
    ph = ctx.synthesize_phase(K, fx, fy, w, torch.as_tensor(px).cuda(),
                              torch.as_tensor(py).cuda(), R, 1, rng=q.Rng(0, 0, 0), precision=1)
    sf2, se2 = ctx.temporal_sf(ph.view(R, 2, M))
    a, b = host(sf), host(sf2)
    print("max rel diff", np.max(np.abs(a[1:] / b[1:] - 1)))
    assert a[0] == 0.0 and np.allclose(a, b, rtol=1e-9, atol=0)
    assert np.allclose(host(se), host(se2), rtol=1e-7, atol=0)


def test_paper_configuration_statistics(q, ctx):
    """The worked example's configuration (fresh frequencies for every
    realisation, 2000 realisations, 1 ms sampling, wind along the baseline):
    the estimate agrees with the exact expectation of the estimator over the
    Cartesian sampling square at every lag within its standard error."""
    N, df = 44, 0.25 / 22
    K, R, M, dt = N * N, 2000, 512, 0.001
    B, v = np.array([56.5, 0.0]), np.array([10.2, 0.0])
    s = q.cartesian_sampler(N, df)
    sf, se = ctx.temporal_piston_structure(q.psd(R0, L0), q.Aperture(D, d), (0.0, 0.0),
                                           tuple(-B), tuple(v), dt, M, s, K, R, 1,
                                           rng=q.Rng(0, 0, 0), precision=0)
    lags = np.array([1, 2, 5, 10, 20, 50, 100, 200, 300, 400, 511])
    ex = A.temporal_sf_square(lags * dt, B, v, R0, L0, D, d, half_width=0.25, n=200)
    g, gs = host(sf)[lags], host(se)[lags]
    z = (g - ex) / gs
    print("lag ms", lags, "\nz", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)
    iso = A.temporal_sf(lags * dt, B, v, R0, L0, D, d)
    print("square / isotropic", np.round(ex / iso, 4))
