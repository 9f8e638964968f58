"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds NO arithmetic of the method: only point sets, baselines,
parameter records and seeded draws of instance parameters.  Both the oracle
and the HIP path consume what it returns; neither is imported here.

Workloads (all synthetic: the paper's data are not public, Sec. 6):
  phase_fp64    -- von Karman r0 = 0.10 m, L0 = 25 m; log-polar K = 1024 over
                   [1e-3, 1e2] cycles/m; 32 x 32 points over a 1 m square
                   (endpoints included, pitch 1/31 m); R = 128, seed 0.
  diffpiston    -- two D = 1.8 m apertures (the VLTI auxiliary telescopes,
                   Sec. 4.3), 32 baselines log-spaced over 1-130 m along x,
                   K = 16384, L0 in {10, 25, 100} m, r0 = 0.1 m, R = 100000.
  large_screen  -- K = 65536, 256 x 256 points over an 8 m square, R = 4096.
  batched       -- 64 uneven instances (D, grid, K, L0 drawn from seed 0).
  learned       -- c2 geometry, L0 = 25 m, learned K = 4096 vs plain 65536.
"""
import numpy as np

SEED_HALF = 1 << 63  # R2 seed (1/2, 1/2) in 0.64 fixed point

FMIN = 1e-3
FMAX = 1e2


def grid_points(n, lo, hi):
    """n x n grid over [lo, hi]^2, endpoints included; row-major (y slow)."""
    g = np.linspace(lo, hi, n)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    return xx.ravel().copy(), yy.ravel().copy()


def disk_mask_points(n, D):
    """n x n grid over [-D/2, D/2]^2 masked to |x| <= D/2."""
    px, py = grid_points(n, -D / 2.0, D / 2.0)
    keep = px * px + py * py <= (D / 2.0) ** 2 * (1.0 + 1e-12)
    return px[keep].copy(), py[keep].copy()


def baselines(n=32, bmin=1.0, bmax=130.0):
    """Baseline vectors along x, log-spaced lengths."""
    bx = np.logspace(np.log10(bmin), np.log10(bmax), n)
    return bx, np.zeros_like(bx)


def phase_fp64():
    px, py = grid_points(32, 0.0, 1.0)
    return dict(name="phase_fp64", model=1, r0=0.10, L0=25.0, fmin=FMIN, fmax=FMAX, K=1024,
                px=px, py=py, R=128, seed=0)


def diffpiston(L0=25.0, R=100000, K=16384):
    bx, by = baselines()
    return dict(name="diffpiston", model=1, r0=0.10, L0=L0, L0_list=(10.0, 25.0, 100.0),
                fmin=FMIN, fmax=FMAX, K=K, D=1.8, d=0.0, bx=bx, by=by, R=R, seed=0)


def large_screen(r0=0.1):
    px, py = grid_points(256, -4.0, 4.0)
    return dict(name="large_screen", model=1, r0=r0, r0_list=(0.05, 0.1, 0.2), L0=25.0,
                fmin=FMIN, fmax=FMAX, K=65536, px=px, py=py, R=4096, seed=0)


def batched(n_inst=64, seed=0, R=256):
    """Uneven instances: D ~ U[0.5, 39] m, grid side 2^U{5..9} masked to the
    disk, K = 2^U{11..16}, L0 ~ U[10, 100] m, r0 = 0.1 m, R realisations each."""
    rng = np.random.default_rng(seed)
    inst = []
    for i in range(n_inst):
        D = float(rng.uniform(0.5, 39.0))
        n = int(2 ** rng.integers(5, 10))
        K = int(2 ** rng.integers(11, 17))
        L0 = float(rng.uniform(10.0, 100.0))
        px, py = disk_mask_points(n, D)
        inst.append(dict(D=D, n=n, K=K, L0=L0, r0=0.1, px=px, py=py, R=R, seed=seed,
                         counter=i * R))
    return inst


def small_batched(n_inst=6, seed=1, R=40):
    """A few small uneven instances that the oracle finishes in seconds."""
    rng = np.random.default_rng(seed)
    inst = []
    for i in range(n_inst):
        D = float(rng.uniform(0.5, 8.0))
        n = int(rng.integers(5, 13))
        K = int(rng.integers(20, 200))
        L0 = float(rng.uniform(10.0, 100.0))
        px, py = disk_mask_points(n, D)
        inst.append(dict(D=D, n=n, K=K, L0=L0, r0=0.1, px=px, py=py, R=R - 7 * (i % 3),
                         seed=seed, counter=1000 * i))
    return inst


def mlp_init(seed=0, H=128, scale=1.0):
    """Seeded initial parameters of the 5 -> H -> H -> 2 proposal network
    (flat layout W1[H][5], b1[H], W2[H][H], b2[H], W3[2][H], b3[2]):
    uniform(-s, s) with s = scale / sqrt(fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((5, H), (H, H), (H, 2)):
        s = scale / np.sqrt(fan_in)
        parts.append(rng.uniform(-s, s, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def proposal_contexts(n_ctx=512, seed=0):
    """Training contexts (D, L0, |B|, theta_B): half the apertures at
    D = 1.8 m, the rest log-uniform in [0.5, 10] m; L0 log-uniform in
    [10, 100] m; |B| log-uniform in [1, 130] m; theta_B uniform in [0, pi)."""
    rng = np.random.default_rng(seed)
    D = np.where(np.arange(n_ctx) % 2 == 0, 1.8, np.exp(rng.uniform(np.log(0.5), np.log(10.0), n_ctx)))
    L0 = np.exp(rng.uniform(np.log(10.0), np.log(100.0), n_ctx))
    B = np.exp(rng.uniform(0.0, np.log(130.0), n_ctx))
    th = rng.uniform(0.0, np.pi, n_ctx)
    return np.stack([D, L0, B, th], axis=1)


def learned(L0=25.0, R=100000):
    """Differential piston with the learned proposal: D = 1.8 m, 32 x-baselines
    1-130 m; learned K = 4096 vs plain K = 65536."""
    bx, by = baselines()
    return dict(name="learned", model=1, r0=0.10, L0=L0, fmin=FMIN, fmax=FMAX, K_learned=4096,
                K_plain=65536, D=1.8, d=0.0, bx=bx, by=by, R=R, seed=0)
