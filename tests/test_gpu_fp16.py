"""GPU tests of the half-precision form (QAIA_FP16: the generated sparse
kernel in IEEE binary16, two replicas per lane): trajectories against the
float64 oracle within the first-order binary16 bound, agreement with a CPU
binary16 emulation of the update order, exact cut values, ragged pairings of
replicas and invalid weight rows."""
import numpy as np
import pytest

import fp32_bounds as fb
import oracle
import workloads as wl
from gpu_helpers import unpack_spins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_26477_amd as q
    return q


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case():
    inst = wl.random_instance(12, 3, "deg3", seed=41, num_edges=16)
    c = wl.dirichlet_weights(6, 3, 42)
    return inst, c


@pytest.mark.parametrize("variant,alpha", [("bsb", 0.0), ("bsb", 0.15), ("dsb", 0.0)])
def test_fp16_trace_within_binary16_bound(q, variant, alpha):
    """x after each of the first 30 steps of every replica stays within the
    first-order binary16 bound around the float64 oracle wherever the bound
    is defined (seeds 43..47)."""
    inst, c = _case()
    prob = q.problem_from_instance(inst)
    worst, checked = 0.0, []
    for seed in range(43, 48):
        s = q.make_schedule(variant, "fp16", steps=1000, dt=0.5, seed=seed, noise_alpha=alpha)
        _, _, _, tr = q.qaia_sample_trace(prob, _dev(c), 8, s, 30)
        _, ref = oracle.sb_sample(inst, c, 8, 1000, variant, dt=0.5, seed=seed, alpha=alpha, trace_steps=30)
        b = fb.Bound(inst, c, 8, 1000, variant, alpha=alpha, seed=seed, steps=30, u=fb.U16, rounded_start=True)
        ok, ratio, frac = b.check(tr.cpu().numpy(), ref)
        assert ok, (seed, ratio)
        worst, checked = max(worst, ratio), checked + [frac]
    print(f"{variant} alpha {alpha}: worst ratio {worst:.3f}, checked {np.mean(checked):.2f}")
    assert np.mean(checked) > 0.1


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_fp16_trace_matches_binary16_emulation(q, variant):
    """The device's binary16 trajectory equals a CPU emulation of the same
    update order (binary16 fused multiply-adds) on at least 99 % of the
    replica-steps of 40 steps (the float32 coefficients are formed in a
    different float64 order, which can move one in its last float32 bit)."""
    inst, c = _case()
    prob = q.problem_from_instance(inst)
    s = q.make_schedule(variant, "fp16", steps=1000, dt=0.5, seed=44)
    _, _, _, tr = q.qaia_sample_trace(prob, _dev(c), 8, s, 40)
    emu = fb.emulate_fp16(inst, c, 8, 1000, variant, seed=44, steps=40).astype(np.float32)
    same = (tr.cpu().numpy() == emu).all(axis=2)
    print(f"{variant}: {same.mean():.4f} of replica-steps identical")
    assert same.mean() >= 0.99


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
@pytest.mark.parametrize("W,R", [(7, 5), (1, 1), (3, 2), (20, 33)])
def test_fp16_cuts_exact_and_pairs_ragged(q, variant, W, R):
    """Odd replica counts pair replicas of different weight vectors in one
    lane and leave the last lane half empty; every sample's cut vector is
    exact for its spins; an invalid weight row zeroes exactly its own rows."""
    import torch
    inst = wl.instance_42_node(4, seed=61)
    c = wl.dirichlet_weights(W, 4, 62)
    bad = W // 2
    c[bad, 1] = -1.0
    prob = q.problem_from_instance(inst)
    s = q.make_schedule(variant, "fp16", steps=300, dt=0.5, seed=63)
    spins, obj, ws = q.qaia_sample(prob, _dev(c), R, s)
    torch.cuda.synchronize()
    assert q.qaia_workspace_status(ws) == bad
    sp, ob = spins.cpu().numpy(), obj.cpu().numpy()
    rows = np.arange(W * R)
    inval = rows // R == bad
    assert not sp[inval].any() and not ob[inval].any()
    assert np.array_equal(ob[~inval], oracle.cut_values(inst, unpack_spins(sp[~inval], inst.n)))


def test_fp16_full_workload_sampled_rows(q):
    """The 42-node 4-objective workload at full size in binary16 (20 000 x 256
    replicas x 2000 steps, discrete SB): cut values of 4096 sampled rows are
    exact, and the samples are not all alike."""
    import torch
    inst = wl.workload_instance("c2_n42_m4")
    c = _dev(wl.workload_weights("c2_n42_m4"))
    prob = q.problem_from_instance(inst)
    s = q.make_schedule("dsb", "fp16", steps=2000, dt=0.5, seed=2005)
    spins, obj, _ = q.qaia_sample(prob, c, 256, s)
    torch.cuda.synchronize()
    pick = np.random.default_rng(64).choice(spins.shape[0], 4096, replace=False)
    sp, ob = spins[pick].cpu().numpy(), obj[pick].cpu().numpy()
    assert np.array_equal(ob, oracle.cut_values(inst, unpack_spins(sp, inst.n)))
    assert len({tuple(r) for r in ob}) > 100


def test_fp16_rejected_off_the_generated_kernel(q):
    inst, c = _case()
    prob = q.problem_from_instance(inst)
    for path in ("sparse_lds", "dense", "dense_staged"):
        with pytest.raises(q.QaiaError) as e:
            q.qaia_sample(prob, _dev(c), 2, q.make_schedule("bsb", "fp16", steps=10, path=path))
        assert e.value.status == q.QAIA_UNSUPPORTED
