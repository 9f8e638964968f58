"""Batched persistent launches of uneven phase-field instances against the
FP64 oracle: eager execution, graph replays (eager work between replays,
every replay checked), and after the autotuner picked a shape."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {1: 1e-5, 2: 1e-3, 3: 1e-5, 4: 1e-5}


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


def instances(q, R_block_div=1):
    out, refs = [], []
    for i, d in enumerate(workloads.small_batched()):
        R = d["R"]
        R_block = max(1, R // R_block_div)
        index = 1000 * i
        s = q.logpolar_sampler(workloads.FMIN, workloads.FMAX, index=index)
        out.append(dict(psd=q.psd(d["r0"], d["L0"]), sampler=s, K=d["K"], px=dev(d["px"]),
                        py=dev(d["py"]), R=R, R_block=R_block,
                        rng=q.Rng(d["seed"], d["counter"], q.COEF_GAUSS_CS)))
        n_sets = math.ceil(R / R_block)
        fx, fy, area = oracle.sample_logpolar(n_sets, d["K"], workloads.FMIN, workloads.FMAX,
                                              index=index)
        w = oracle.weights(fx, fy, area, r0=d["r0"], L0=d["L0"])
        refs.append(oracle.synthesize(fx, fy, w, d["px"], d["py"], R, R_block, K=d["K"],
                                      seed=d["seed"], counter=d["counter"]))
    return out, refs


def check(outs, refs, tol, tag):
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        g = o.double().cpu().numpy()
        e = np.max(np.abs(g - r)) / math.sqrt(np.mean(r * r))
        print(f"{tag} instance {i}: eps_max {e:.3e}")
        assert e <= tol, (tag, i, e)


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("R_block_div", [1, 3])
def test_batch_matches_oracle(q, ctx, precision, R_block_div):
    inst, refs = instances(q, R_block_div)
    b = q.Batch(ctx, inst, precision=precision)
    info = b.info()
    assert info["n_items"] > 0
    check(b.execute(), refs, TOL[precision], f"eager p{precision}")
    b.close()


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_batch_every_shape(q, ctx, precision, shape):
    """Each launch shape (fused 0-3, two-phase 4) against the oracle, with
    several sets per instance."""
    inst, refs = instances(q, 3)
    b = q.Batch(ctx, inst, precision=precision)
    b.set_shape(shape)
    assert b.info()["shape"] == shape
    check(b.execute(), refs, TOL[precision], f"shape {shape} p{precision}")
    b.close()


def test_batch_two_phase_is_default(q, ctx):
    inst, _ = instances(q, 1)
    b = q.Batch(ctx, inst, precision=2)
    assert b.info()["shape"] == q.BATCH_SHAPE_TWO_PHASE
    with pytest.raises(q.QrfsError):
        b.set_shape(q.BATCH_SHAPES)
    b.close()


@pytest.mark.parametrize("shape", [0, 4])
def test_batch_graph_replays(q, ctx, shape):
    inst, refs = instances(q, 2)
    b = q.Batch(ctx, inst, precision=3)
    b.set_shape(shape)
    eager = [o.clone() for o in b.execute()]
    torch.cuda.synchronize()
    for rep in range(3):
        for o in b.outputs:
            o.fill_(float("nan"))
        x = torch.randn(1 << 20, device="cuda")  # unrelated eager work between replays
        y = (x * 2.0).sum()
        b.execute(use_graph=True)
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for o, e in zip(b.outputs, eager):
            assert torch.equal(o, e), rep
    check(b.outputs, refs, TOL[3], "graph")
    b.close()


@pytest.mark.parametrize("shape", [4, 0])
def test_batch_graph_after_rebuilt_work_list(q, ctx, shape):
    """A graph captured before the work list is rebuilt (set_shape to the same
    shape, then the autotuner) is not replayed with the freed list: the next
    graph execution captures the current one and matches the oracle."""
    inst, refs = instances(q, 2)
    b = q.Batch(ctx, inst, precision=3)
    b.set_shape(shape)
    check(b.execute(use_graph=True), refs, TOL[3], "first graph")
    b.set_shape(shape)
    check(b.execute(use_graph=True), refs, TOL[3], "graph after set_shape")
    b.autotune()
    for o in b.outputs:
        o.fill_(float("nan"))
    check(b.execute(use_graph=True), refs, TOL[3], "graph after autotune")
    b.close()


def test_batch_autotune(q, ctx):
    inst, refs = instances(q, 1)
    b = q.Batch(ctx, inst, precision=3)
    ms = b.autotune()
    assert ms > 0
    shape = b.info()["shape"]
    print("autotuned shape", shape, "ms", ms)
    check(b.execute(use_graph=True), refs, TOL[3], "autotuned graph")
    check(b.execute(), refs, TOL[3], "autotuned eager")
    b.close()


@pytest.mark.parametrize("precision", [4, 3, 2])
def test_batch_full_size_graph(q, ctx, precision):
    """The 64 uneven instances of the benchmark (R = 256 each, K up to 65536,
    grids up to 512^2 masked to the disk) in its timed configuration:
    autotuned, then replayed from a HIP graph.  Two replays equal the eager
    result bit for bit; the first and last eight rows of three instances
    (largest K, most points, fewest points) agree with the oracle at 256
    sampled points."""
    specs = workloads.batched()
    inst = []
    for i, d in enumerate(specs):
        inst.append(dict(psd=q.psd(d["r0"], d["L0"]),
                         sampler=q.logpolar_sampler(workloads.FMIN, workloads.FMAX,
                                                    index=i * (1 << 20)),
                         K=d["K"], px=dev(d["px"]), py=dev(d["py"]), R=d["R"], R_block=d["R"],
                         rng=q.Rng(d["seed"], d["counter"], q.COEF_GAUSS_CS)))
    b = q.Batch(ctx, inst, precision=precision)
    try:
        b.autotune()
        eager = [o.clone() for o in b.execute()]
        torch.cuda.synchronize()
        for rep in range(2):
            for o in b.outputs:
                o.fill_(float("nan"))
            b.execute(use_graph=True)
            torch.cuda.synchronize()
            for o, e in zip(b.outputs, eager):
                assert torch.equal(o, e), rep
        sizes = [d["px"].size for d in specs]
        picks = {int(np.argmax([d["K"] for d in specs])), int(np.argmax(sizes)),
                 int(np.argmin(sizes))}
        for j in sorted(picks):
            d = specs[j]
            fx, fy, area = oracle.sample_logpolar(1, d["K"], workloads.FMIN, workloads.FMAX,
                                                  index=j * (1 << 20))
            w = oracle.weights(fx, fy, area, r0=d["r0"], L0=d["L0"])
            cols = np.random.default_rng(j).choice(d["px"].size, min(256, d["px"].size),
                                                   replace=False)
            ci = torch.as_tensor(cols, device="cuda")
            for r0 in (0, d["R"] - 8):
                ref = oracle.synthesize(fx, fy, w, d["px"][cols], d["py"][cols], 8, 8, K=d["K"],
                                        seed=d["seed"], counter=d["counter"] + r0)
                got = b.outputs[j][r0:r0 + 8][:, ci].double().cpu().numpy()
                e = np.max(np.abs(got - ref)) / math.sqrt(np.mean(ref * ref))
                print(f"p{precision} instance {j} (K {d['K']}, P {d['px'].size}) rows {r0}+: "
                      f"eps_max {e:.3e}", flush=True)
                assert e <= TOL[precision], (j, r0, e)
    finally:
        b.close()


def test_batch_rejects_bad_instances(q, ctx):
    inst, _ = instances(q, 1)
    bad = dict(inst[0])
    bad["R_block"] = bad["R"] + 1
    with pytest.raises(q.QrfsError) as e:
        q.Batch(ctx, [inst[1], bad], precision=1)
    assert e.value.status == q.ERR_INVALID_ARG
    with pytest.raises(q.QrfsError) as e:
        q.Batch(ctx, inst[:2], precision=0)
    assert e.value.status == q.ERR_UNSUPPORTED


# ------------------------------------------- apertures in the batch ----

def aperture_instances(q):
    """Phase instances mixed with pistons of annular and filled apertures
    (ragged against every column tile: 300 = 256 + 44) and G-tilts along x
    and along an oblique direction."""
    inst, refs = instances(q, 3)
    rng = np.random.default_rng(21)
    for j, u in enumerate([None, (1.0, 0.0), (0.6, -0.8)]):
        P, K, R, R_block = 300 - 37 * j, 203 - 40 * j, 90, 45
        cx, cy = rng.uniform(-60, 60, P), rng.uniform(-60, 60, P)
        D = rng.choice([8.0, 1.8, 4.0], P)
        d = np.where(D > 3.0, 1.1, 0.0)
        index, seed, counter = 50000 + 7000 * j, 4 + j, 300 * j
        s = q.logpolar_sampler(1e-3, 1e2, index=index)
        d_in = dict(psd=q.psd(0.1, 25.0), sampler=s, K=K, px=dev(cx), py=dev(cy), R=R,
                    R_block=R_block, rng=q.Rng(seed, counter, q.COEF_GAUSS_CS), apD=dev(D),
                    apd=dev(d))
        if u is not None:
            d_in["u"] = u
        inst.append(d_in)
        n_sets = math.ceil(R / R_block)
        fx, fy, area = oracle.sample_logpolar(n_sets, K, 1e-3, 1e2, index=index)
        w = oracle.weights(fx, fy, area, r0=0.1, L0=25.0)
        if u is None:
            refs.append(oracle.piston(fx, fy, w, cx, cy, D, d, R, R_block, K=K, seed=seed,
                                      counter=counter))
        else:
            refs.append(sum(u[a] * oracle.tilt(fx, fy, w, cx, cy, D, d, R, R_block, axis=a, K=K,
                                               seed=seed, counter=counter)
                            for a in (0, 1) if u[a] != 0.0))
    return inst, refs


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_batch_apertures_every_shape(q, ctx, precision, shape):
    inst, refs = aperture_instances(q)
    b = q.Batch(ctx, inst, precision=precision)
    b.set_shape(shape)
    print(f"apertures shape {shape} p{precision}", flush=True)
    check(b.execute(), refs, TOL[precision], f"apertures shape {shape} p{precision}")
    b.close()


def test_batch_apertures_graph(q, ctx):
    inst, refs = aperture_instances(q)
    b = q.Batch(ctx, inst, precision=3)
    eager = [o.clone() for o in b.execute()]
    for rep in range(2):
        for o in b.outputs:
            o.fill_(float("nan"))
        b.execute(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(b.outputs, eager):
            assert torch.equal(o, e), rep
    check(b.outputs, refs, TOL[3], "apertures graph")
    b.close()


def test_batch_rejects_bad_apertures(q, ctx):
    inst, _ = aperture_instances(q)
    bad = dict(inst[-1])
    del bad["apd"]
    with pytest.raises(q.QrfsError):
        q.Batch(ctx, [bad], precision=1)
    bad = dict(inst[0])
    bad["u"] = (1.0, 0.0)  # a direction without apertures
    with pytest.raises(q.QrfsError) as e:
        q.Batch(ctx, [bad], precision=1)
    assert "apertures" in e.value.detail
