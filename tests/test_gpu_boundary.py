"""The boundary's arguments beyond the sums themselves, through the C ABI:
the wavelength of the PSD (optical path outputs, Sec. 4.4), the context's
workspace cap, and the autotuner's cache file."""
import math
import os

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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("ap", [None, (8.0, 1.1)])
def test_weights_in_optical_path(q, ap):
    lam = 1.65e-6
    with q.Context(0) as ctx:
        s = q.logpolar_sampler(1e-3, 1e2, index=3)
        fx, fy, area = ctx.sample_frequencies(s, 2, 777)
        aperture = None if ap is None else q.Aperture(*ap)
        w = ctx.weights(q.psd(0.12, 30.0, wavelength=lam), fx, fy, area, aperture)
        ref = oracle.weights(host(fx), host(fy), host(area), r0=0.12, L0=30.0,
                             D=None if ap is None else ap[0], d=0.0 if ap is None else ap[1],
                             wavelength=lam)
        g = host(w)
        assert np.max(np.abs(g - ref)) / np.max(np.abs(ref)) < 1e-13
        # the fused sampler + weights gives the same values
        s = q.logpolar_sampler(1e-3, 1e2, index=3)
        _, _, w2 = ctx.sample_weights(s, 2, 777, q.psd(0.12, 30.0, wavelength=lam), aperture)
        assert np.max(np.abs(host(w2) - ref)) / np.max(np.abs(ref)) < 1e-13


def test_structure_function_in_optical_path(q):
    """qrfs_diff_piston_structure with a wavelength: (lambda / 2 pi)^2 times
    the phase result of the same draws."""
    cfg = workloads.diffpiston()
    lam = 2.2e-6
    out = {}
    with q.Context(0) as ctx:
        for wl in (0.0, lam):
            s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
            sf, _ = ctx.diff_piston_structure(q.psd(0.1, 25.0, wavelength=wl),
                                              q.Aperture(cfg["D"], 0.0), dev(cfg["bx"]),
                                              dev(cfg["by"]), s, 512, 400, 100,
                                              rng=q.Rng(3, 0, 0), precision=q.PREC_FP64)
            out[wl] = host(sf)
    assert np.max(np.abs(out[lam] / (out[0.0] * (lam / (2 * math.pi)) ** 2) - 1)) < 1e-12


def test_workspace_cap(q):
    """A call whose workspace exceeds the context's cap fails with
    QRFS_ERR_OUT_OF_MEMORY before enqueueing; calls that fit still run, and
    the two-phase kernel cuts its tiles to fit a cap that allows it."""
    cfg = workloads.diffpiston()
    with q.Context(0, workspace_cap=1 << 16) as ctx:
        s = q.logpolar_sampler(cfg["fmin"], cfg["fmax"])
        with pytest.raises(q.QrfsError) as e:
            ctx.diff_piston_structure(q.psd(0.1, 25.0), q.Aperture(cfg["D"], 0.0),
                                      dev(cfg["bx"]), dev(cfg["by"]), s, 1024, 20000, 256,
                                      rng=q.Rng(0, 0, 0), precision=q.PREC_FP32)
        assert e.value.status == q.ERR_OUT_OF_MEMORY and "cap" in e.value.detail
        assert s.index == 0
    # two-phase phase field under a cap smaller than the whole coefficient
    # staging: pieces of 256 rows, same result as without the cap
    K, P, R = 1500, 1500, 512
    rng = np.random.default_rng(1)
    px, py = dev(rng.uniform(-2, 2, P)), dev(rng.uniform(-2, 2, P))
    res = []
    for cap in (0, 6 << 20):
        with q.Context(0, workspace_cap=cap) as ctx:
            ctx.set_tuning(q.TUNE_WIDE_PATH, 2)
            s = q.logpolar_sampler(1e-3, 1e2)
            fx, fy, area = ctx.sample_frequencies(s, 1, K)
            w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area)
            res.append(host(ctx.synthesize_phase(K, fx, fy, w, px, py, R, R,
                                                 rng=q.Rng(2, 0, 0), precision=q.PREC_BF16X6)))
    assert np.array_equal(res[0], res[1])


def test_workspace_cap_fp16x3_many_sets(q):
    """FP16x3 in the two-phase kernel keeps one tile scale per set behind the
    coefficient tiles: under a cap that splits 64 sets into pieces the
    result equals the uncapped one bit for bit."""
    K, P, R, R_block = 1500, 1500, 64 * 128, 128
    rng = np.random.default_rng(4)
    px, py = dev(rng.uniform(-2, 2, P)), dev(rng.uniform(-2, 2, P))
    res = []
    for cap in (0, 8 << 20):
        with q.Context(0, workspace_cap=cap) as ctx:
            ctx.set_tuning(q.TUNE_WIDE_PATH, 2)
            s = q.logpolar_sampler(1e-3, 1e2)
            fx, fy, area = ctx.sample_frequencies(s, R // R_block, K)
            w = ctx.weights(q.psd(0.1, 25.0), fx, fy, area)
            res.append(host(ctx.synthesize_phase(K, fx, fy, w, px, py, R, R_block,
                                                 rng=q.Rng(5, 0, 0), precision=q.PREC_FP16X3)))
    assert np.all(np.isfinite(res[0]))
    assert np.array_equal(res[0], res[1])


def test_autotune_cache(q, tmp_path):
    """The first autotune of a batch times it and appends its choice to the
    cache; a batch of the same sizes then takes the stored choice."""
    path = tmp_path / "tune.txt"
    inst = []
    for i, d in enumerate(workloads.small_batched()):
        inst.append(dict(psd=q.psd(d["r0"], d["L0"]),
                         sampler=q.logpolar_sampler(workloads.FMIN, workloads.FMAX, index=i),
                         K=d["K"], px=dev(d["px"]), py=dev(d["py"]), R=d["R"], R_block=d["R"],
                         rng=q.Rng(d["seed"], d["counter"], 0)))
    with q.Context(0) as ctx:
        b = q.Batch(ctx, inst, precision=3)
        ms = b.autotune(cache_path=str(path))
        shape = b.info()["shape"]
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("qrfs-autotune-1 ")
        assert int(lines[0].split()[2]) == shape
        b.close()
        # tamper with the stored choice: the cached shape is what a new
        # batch of the same sizes takes, without timing
        other = (shape + 1) % q.BATCH_SHAPES
        path.write_text(f"{lines[0].split()[0]} {lines[0].split()[1]} {other} 1.5\n")
        b = q.Batch(ctx, inst, precision=3)
        assert b.autotune(cache_path=str(path)) == 1.5
        assert b.info()["shape"] == other
        b.close()
        # another precision is another key: timed and appended
        b = q.Batch(ctx, inst, precision=2)
        b.autotune(cache_path=str(path))
        assert len(path.read_text().splitlines()) == 2
        b.close()
        with pytest.raises(q.QrfsError):
            b = q.Batch(ctx, inst, precision=3)
            try:
                b.autotune(cache_path=str(tmp_path / "no_such_dir" / "t.txt"))
            finally:
                b.close()
    assert ms > 0
