"""Randomised samplers (Sec. 3.1: fully random frequencies, the jittered
grid of Eq. 4), point-set measures and the noise-free per-set structure
function through the C ABI, against the FP64 oracle.

Bars: jittered and random Cartesian points bit for bit; random log-polar
and disc points to 1e-14 of the band edge (exp and sincos differ in the
last bits); clash counts exactly; minimum distances to 1 ulp; squared L2
star discrepancy to 8 K eps (its closed form cancels terms of order one,
summed in another order); per-set
structure function to 1e-10 relative (the oracle's 2(1 - cos) loses up to
~1e-16 / (1 - cos) per term at short baselines, the kernel's 4 sin^2 form
does not).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------ samplers ----

@pytest.mark.parametrize("index", [0, 4321, (1 << 40) + 3])
def test_jitter_bit_exact(q, ctx, index):
    N, df, n_sets = 44, 0.25 / 22, 3
    s = q.jitter_sampler(N, df, index=index, seed_y=17)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, N * N)
    assert s.index == index + n_sets * N * N
    rx, ry, ra = oracle.sample_jitter(n_sets, N, df, index=index, seed_y=17)
    assert np.array_equal(host(fx), rx) and np.array_equal(host(fy), ry)
    assert np.array_equal(host(area), ra)


def test_jitter_needs_square_K(q, ctx):
    s = q.jitter_sampler(44, 0.01)
    with pytest.raises(q.QrfsError) as e:
        ctx.sample_frequencies(s, 1, 44 * 44 - 1)
    assert "N^2" in e.value.detail


def test_random_cartesian_bit_exact(q, ctx):
    n_sets, K, N, df = 4, 777, 44, 0.25 / 22
    s = q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df, index=99, seed_x=12345)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    rx, ry, ra = oracle.sample_pseudo(oracle.MAP_CARTESIAN, n_sets, K, N=N, df=df, index=99,
                                      seed_x=12345)
    assert np.array_equal(host(fx), rx) and np.array_equal(host(fy), ry)
    assert np.array_equal(host(area), ra)


@pytest.mark.parametrize("scheme", ["logpolar", "disc"])
def test_random_polar_maps(q, ctx, scheme):
    n_sets, K = 3, 1000
    if scheme == "logpolar":
        s = q.random_sampler(q.SAMPLER_RANDOM_LOGPOLAR, fmin=1e-3, fmax=1e2, index=7)
        ref = oracle.sample_pseudo(oracle.MAP_LOGPOLAR, n_sets, K, fmin=1e-3, fmax=1e2, index=7)
        edge = 1e2
    else:
        s = q.random_sampler(q.SAMPLER_RANDOM_DISC, fmax=0.25, index=7)
        ref = oracle.sample_pseudo(oracle.MAP_DISC, n_sets, K, fmax=0.25, index=7)
        edge = 0.25
    got = ctx.sample_frequencies(s, n_sets, K)
    for g, r in zip(got[:2], ref[:2]):
        assert np.max(np.abs(host(g) - r)) <= 1e-14 * edge
    assert np.allclose(host(got[2]), ref[2], rtol=1e-13, atol=0)


# --------------------------------------------------------------- measures ----

def _square(N, df):
    L = N * df
    return -L / 2, -L / 2, L, L


@pytest.mark.parametrize("scheme,K,n_sets", [("r2", 1936, 12), ("jitter", 1936, 12),
                                             ("random", 300, 40), ("random", 1, 5),
                                             ("r2", 257, 9)])
def test_point_set_measures_parity(q, ctx, scheme, K, n_sets):
    N = int(round(math.sqrt(K))) if scheme == "jitter" else 44
    df = 0.25 / 22
    if scheme == "r2":
        s = q.cartesian_sampler(N, df, index=5)
        rx, ry, _ = oracle.sample_cartesian(n_sets, K, N, df, index=5)
    elif scheme == "jitter":
        s = q.jitter_sampler(N, df, index=5)
        rx, ry, _ = oracle.sample_jitter(n_sets, N, df, index=5)
    else:
        s = q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df, index=5)
        rx, ry, _ = oracle.sample_pseudo(oracle.MAP_CARTESIAN, n_sets, K, N=N, df=df, index=5)
    fx, fy, _ = ctx.sample_frequencies(s, n_sets, K)
    x0, y0, Lx, Ly = _square(N, df)
    r = 0.3 / math.sqrt(K)
    print(f"measures {scheme} K{K} sets{n_sets}", flush=True)
    md, nc, T = ctx.point_set_measures(fx, fy, n_sets, K, x0, y0, Lx, Ly, r)
    rmd, rnc, rT = oracle.point_set_measures(rx, ry, n_sets, K, x0, y0, Lx, Ly, r)
    assert np.array_equal(host(nc), rnc)
    gmd = host(md)
    if K == 1:
        assert np.all(np.isinf(gmd)) and np.all(np.isinf(rmd))
    else:
        assert np.all(np.abs(gmd - rmd) <= np.spacing(rmd))
    # T^2 = 1/9 - s1/(2K) + s2/K^2 cancels: terms of order 1 leave ~1e-6.
    # Sums of K^2 terms in [0, 1] in two orders differ by ~K eps times the
    # terms' size (at most 1/9 + 1/2 + 1), allowed eight times over.
    gT2, rT2 = host(T) ** 2, rT ** 2
    bound = 8 * np.finfo(float).eps * (K + 1) * 1.61
    print("max |dT^2|", np.max(np.abs(gT2 - rT2)), "bound", bound, "T^2", rT2.min())
    assert np.all(np.abs(gT2 - rT2) <= bound)


def test_set_sf_expectation_parity(q, ctx):
    cfg = workloads.diffpiston()
    n_sets, K = 7, 1000
    s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"], index=3)
    fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
    w = ctx.weights(q.psd(cfg["r0"], 25.0), fx, fy, area, q.Aperture(cfg["D"], 0.0))
    bx, by = cfg["bx"], cfg["by"] + 0.3  # 32 baselines, ragged against 8 per pass
    bx = np.concatenate([bx, [0.0]])
    by = np.concatenate([by, [1e-3]])
    S = host(ctx.set_sf_expectation(K, fx, fy, w, n_sets, dev(bx), dev(by)))
    ref = oracle.set_sf_expectation(host(fx), host(fy), host(w), n_sets, K, bx, by)
    e = np.max(np.abs(S / ref - 1))
    print("set sf max rel", e)
    assert e <= 1e-10


# ------------------------------------------------------ sampler ablation ----

def test_sampling_error_ordering(q, ctx):
    """The worked example's Cartesian geometry (UT filter, L0 = 22 m,
    df = 0.25/22, N = 44): across 200 sets the per-set noise-free structure
    function scatters least for R2, more for the jittered grid and most for
    fully random frequencies (the sampling error alone, at equal K)."""
    N, df, n_sets, D, d = 44, 0.25 / 22, 200, 8.0, 1.1
    K = N * N
    B = np.array([5.0, 20.0, 56.5, 100.0])
    bx, by = dev(B), dev(np.zeros_like(B))
    spread = {}
    for name, s in {"r2": q.cartesian_sampler(N, df),
                    "jitter": q.jitter_sampler(N, df),
                    "random": q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df)}.items():
        fx, fy, area = ctx.sample_frequencies(s, n_sets, K)
        w = ctx.weights(q.psd(0.1, 22.0), fx, fy, area, q.Aperture(D, d))
        S = host(ctx.set_sf_expectation(K, fx, fy, w, n_sets, bx, by))
        spread[name] = S.std(axis=0) / S.mean(axis=0)
        print(name, "relative spread of S per baseline", np.round(spread[name], 5))
    assert np.all(spread["r2"] < spread["jitter"]) and np.all(spread["jitter"] < spread["random"])


# ------------------------------------------------- sampling + weights ----

@pytest.mark.parametrize("scheme", ["cartesian", "logpolar", "disc", "jitter", "random_logpolar",
                                    "random_cartesian", "random_disc"])
@pytest.mark.parametrize("ap", [None, (8.0, 1.1)])
@pytest.mark.parametrize("precision", [0, 4])
def test_sample_weights_equal_two_calls(q, ctx, scheme, ap, precision):
    """qrfs_sample_weights (one fused kernel) gives exactly the frequencies
    and weights of qrfs_sample_frequencies followed by qrfs_weights (binary64
    weights, and those for FP32-class sums), and advances the sampler the
    same way."""
    N, df, n_sets = 44, 0.25 / 22, 3
    K = N * N
    make = {
        "cartesian": lambda: q.cartesian_sampler(N, df, index=9),
        "logpolar": lambda: q.logpolar_sampler(1e-3, 1e2, index=9),
        "disc": lambda: q.disc_sampler(0.25, index=9),
        "jitter": lambda: q.jitter_sampler(N, df, index=9),
        "random_logpolar": lambda: q.random_sampler(q.SAMPLER_RANDOM_LOGPOLAR, fmin=1e-3,
                                                    fmax=1e2, index=9),
        "random_cartesian": lambda: q.random_sampler(q.SAMPLER_RANDOM_CARTESIAN, N=N, df=df,
                                                     index=9),
        "random_disc": lambda: q.random_sampler(q.SAMPLER_RANDOM_DISC, fmax=0.25, index=9),
    }[scheme]
    p = q.psd(0.1, 22.0)
    aperture = None if ap is None else q.Aperture(*ap)
    s1, s2 = make(), make()
    fx, fy, w = ctx.sample_weights(s1, n_sets, K, p, aperture, precision=precision)
    fx2, fy2, area = ctx.sample_frequencies(s2, n_sets, K)
    w2 = ctx.weights(p, fx2, fy2, area, aperture, precision=precision)
    torch.cuda.synchronize()
    assert s1.index == s2.index == 9 + n_sets * K
    assert torch.equal(fx, fx2) and torch.equal(fy, fy2) and torch.equal(w, w2)


@pytest.mark.parametrize("ap,precision", [((1.8, 0.0), 0), ((8.0, 1.1), 0), ((1.8, 0.0), 4)])
def test_sample_weights_lane_order_equal_two_calls(q, ctx, ap, precision):
    """Large log-polar requests with binary64 weights and a filter run in
    lane order (lanes of a wave 12096 indices apart, from 32 tiles of 774144
    indices on): every frequency and weight equals the two-call result, over
    33.9 tiles (the last one partly filled); the FP32-class weights of the
    same request (plain order) too."""
    n_sets, K = 1601, 16384
    p = q.psd(0.1, 25.0)
    aperture = q.Aperture(*ap)
    s1 = q.logpolar_sampler(1e-3, 1e2, index=12345)
    s2 = q.logpolar_sampler(1e-3, 1e2, index=12345)
    fx, fy, w = ctx.sample_weights(s1, n_sets, K, p, aperture, precision=precision)
    fx2, fy2, area = ctx.sample_frequencies(s2, n_sets, K)
    w2 = ctx.weights(p, fx2, fy2, area, aperture, precision=precision)
    torch.cuda.synchronize()
    assert s1.index == s2.index == 12345 + n_sets * K
    assert torch.equal(fx, fx2) and torch.equal(fy, fy2) and torch.equal(w, w2)


def test_sample_weights_rejects_bad_arguments(q, ctx):
    with pytest.raises(q.QrfsError) as e:
        ctx.sample_weights(q.logpolar_sampler(2.0, 1.0), 1, 8, q.psd(0.1, 25.0))
    assert e.value.status == q.ERR_INVALID_ARG
    with pytest.raises(q.QrfsError) as e:
        ctx.sample_weights(q.logpolar_sampler(1e-3, 1e2), 1, 8, q.psd(-0.1, 25.0))
    assert e.value.status == q.ERR_INVALID_ARG
