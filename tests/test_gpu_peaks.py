"""The roofline probes of libqrfs_peaks compute what they claim: after a
short run every lane holds the closed-form sum of its MFMA or FMA chains,
and the copy probe moves the data unchanged (the work they report is then
the work done)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02978_amd import peaks
    peaks.load_peaks()
    return peaks


@pytest.mark.parametrize("kind,kd", [(0, 16), (1, 16), (2, 2)])
def test_mfma_probe_closed_form(pk, kind, kd):
    import torch
    st = torch.cuda.current_stream()
    blocks = pk.peak_blocks(kind)
    assert blocks >= 256
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    x, iters = 2.0 ** -6, 24
    work = pk.peak_launch(kind, blocks, iters, x, 0.0, out, None, None, 0, st)
    torch.cuda.synchronize()
    # four 32x32 accumulators per wave, 16 values per lane, Kd products of x^2 each
    assert torch.all(out == 64 * iters * kd * x * x)
    assert work == blocks * 4 * iters * 4 * 2 * 32 * 32 * kd


@pytest.mark.parametrize("kind", [3, 4])
def test_fma_probe_closed_form(pk, kind):
    import torch
    st = torch.cuda.current_stream()
    blocks = pk.peak_blocks(kind)
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    y, iters = 2.0 ** -10, 40
    work = pk.peak_launch(kind, blocks, iters, 1.0, y, out, None, None, 0, st)
    torch.cuda.synchronize()
    assert torch.all(out == 8 * iters * y)
    assert work == blocks * 256 * iters * 8 * 2


def test_copy_probe(pk):
    import torch
    st = torch.cuda.current_stream()
    n = (1 << 20) + 12
    src = torch.randn(n, device="cuda")
    dst = torch.zeros_like(src)
    work = pk.peak_launch(pk.PEAK_HBM_COPY, 64, 0, 0.0, 0.0, None, src, dst, n, st)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert work == 8 * n


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_mfma_probe_varied_operands_linear(pk, kind):
    """x = 0: each chain multiplies its own varied operands (exact in
    binary32), so the sums after n rounds are n times those after one."""
    import torch
    st = torch.cuda.current_stream()
    blocks = pk.peak_blocks(kind)
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    pk.peak_launch(kind, blocks, 1, 0.0, 0.0, out, None, None, 0, st)
    one = out.clone()
    pk.peak_launch(kind, blocks, 20, 0.0, 0.0, out, None, None, 0, st)
    torch.cuda.synchronize()
    assert bool((one != 0).any())
    assert torch.equal(out, 20 * one)
    # lanes differ: the operands are not all equal
    assert int(torch.unique(one[:64]).numel()) > 4
