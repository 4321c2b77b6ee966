"""Measurement kernels (FMA loop, MFMA loop per operand format, HBM copy):
each computes a closed-form result, checked exactly on small launches."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2604_26477_amd as q
    return q


def test_fma_chains_closed_form(q):
    blocks, iters = 6, 1000
    out = q.qaia_peak_fma(blocks, iters, 1.0, 1.0)
    t = torch.arange(blocks * 256, dtype=torch.int64)
    # chain c of lane t starts at (t + c) mod 8 and adds 1 per iteration
    x0 = sum(((t + c) % 8) for c in range(8)).to(torch.float32)
    assert torch.equal(out.cpu(), x0 + 8 * iters)
    # a = 0.5, b = 0: every chain decays to exactly 0 after enough halvings
    out = q.qaia_peak_fma(2, 200, 0.5, 0.0)
    assert torch.count_nonzero(out).item() == 0


@pytest.mark.parametrize("prec,K", [("fp32", 2), ("bf16", 16), ("fp8", 64)])
def test_mfma_all_ones_closed_form(q, prec, K):
    blocks, iters = 5, 777
    out = q.qaia_peak_mfma(prec, blocks, iters)
    assert torch.all(out == 4.0 * K * iters).item()


def test_valu_mix_closed_form(q):
    """k = 0: the sparse-SB instruction mix leaves every spin at its start value."""
    blocks, iters = 6, 700
    out = q.qaia_peak_valu(blocks, iters, 0.0)
    t = torch.arange(blocks * 256, dtype=torch.int64)
    x0 = sum(((t + i) % 8).to(torch.float64) / 8 - 0.5 for i in range(14))
    y0 = sum(((t + 3 * i) % 4).to(torch.float64) / 4 for i in range(14))
    assert torch.equal(out.cpu().to(torch.float64), x0 + y0)
    # a non-zero coefficient changes the state (the FMAs are really executed)
    moved = q.qaia_peak_valu(blocks, 3, 1e-3)
    assert not torch.equal(moved.cpu(), out.cpu())


def test_copy_is_exact(q):
    g = torch.Generator(device="cuda").manual_seed(11)
    src = torch.randint(-2**31, 2**31 - 1, (1 << 20,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    q.qaia_peak_copy(src, dst)
    assert torch.equal(src, dst)
    # ragged tail of a short copy (fewer 16-byte items than one block's lanes)
    s2 = src[:44].clone()
    d2 = torch.zeros_like(s2)
    q.qaia_peak_copy(s2, d2)
    assert torch.equal(s2, d2)
