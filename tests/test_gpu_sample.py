"""GPU parity of the sampler (qaia_sample / qaia_sample_trace / qaia_evaluate)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import fp32_bounds as fb
import noise_model as nm
import oracle
import workloads as wl
from gpu_helpers import pack_spins, rel_inf_error, unpack_spins

pytestmark = pytest.mark.gpu

SPARSE_PATHS = ["sparse_reg", "sparse_lds"]


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


def _sample(q, prob, c, R, **kw):
    s = q.make_schedule(**kw)
    spins, obj, ws = q.qaia_sample(prob, _dev(c), R, s)
    import torch
    torch.cuda.synchronize()
    return spins.cpu().numpy(), obj.cpu().numpy(), ws


# ---------------------------------------------------------------- trajectories

@pytest.mark.parametrize("path", SPARSE_PATHS)
def test_trace_parity_bsb_first_100_steps(q, path):
    """FP32 x stays within 1e-5 (relative infinity norm) of the FP64 oracle for 100 steps."""
    inst = wl.random_instance(12, 3, "deg3", seed=41, num_edges=16)
    c = wl.dirichlet_weights(6, 3, 42)
    R, T, steps = 8, 1000, 100
    prob = q.problem_from_instance(inst)
    s = q.make_schedule("bsb", steps=T, dt=0.5, seed=43, path=path)
    spins, obj, ws, tr = q.qaia_sample_trace(prob, _dev(c), R, s, steps)
    tr = tr.cpu().numpy()
    _, ref = oracle.sb_sample(inst, c, R, T, "bsb", dt=0.5, seed=43, trace_steps=steps)
    err = rel_inf_error(tr, ref)
    print(f"{path}: max rel err over {steps} steps = {err.max():.3e}")
    assert err.max() <= 1e-5


def _dsb_safe_seed(inst, c, R, T, steps):
    """A seed whose oracle trajectories keep |x| >= 1e-4 over the traced steps, so
    the sgn discontinuity of discrete SB is far from FP32 rounding."""
    for seed in range(100, 160):
        _, ref = oracle.sb_sample(inst, c, R, T, "dsb", dt=0.5, seed=seed, trace_steps=steps)
        if np.abs(ref).min() >= 1e-4:
            return seed, ref
    pytest.skip("no seed without near-zero crossings")


@pytest.mark.parametrize("path", SPARSE_PATHS)
def test_trace_parity_dsb_first_100_steps(q, path):
    inst = wl.random_instance(10, 2, "deg3", seed=51, num_edges=12)
    c = wl.dirichlet_weights(2, 2, 52)
    R, T, steps = 2, 1000, 100
    seed, ref = _dsb_safe_seed(inst, c, R, T, steps)
    prob = q.problem_from_instance(inst)
    s = q.make_schedule("dsb", steps=T, dt=0.5, seed=seed, path=path)
    _, _, _, tr = q.qaia_sample_trace(prob, _dev(c), R, s, steps)
    err = rel_inf_error(tr.cpu().numpy(), ref)
    print(f"{path}: dsb max rel err = {err.max():.3e}")
    assert err.max() <= 1e-5


# ---------------------------------------------------------------- exact cuts

@pytest.mark.parametrize("path", SPARSE_PATHS)
@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_c1_cut_values_bit_exact(q, path, variant):
    """42-node, 48-edge, 3-objective workload at full size (200 x 16 x 1000):
    every sampled cut vector equals the oracle's evaluation of the same spins."""
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3")
    prob = q.problem_from_instance(inst)
    spins, obj, _ = _sample(q, prob, c, 16, variant=variant, steps=1000, dt=0.5, seed=1003, path=path)
    s = unpack_spins(spins, inst.n)
    assert np.array_equal(obj, oracle.cut_values(inst, s))
    # the sampler found cuts well above random (mean cut of a random spin vector is T_k / 2)
    scal = (obj.astype(np.float64) * np.repeat(c, 16, axis=0)).sum(axis=1)
    rand = (inst.weights.sum(axis=1) / 2.0 * np.repeat(c, 16, axis=0)).sum(axis=1)
    assert np.mean(scal > rand) > 0.95


def test_evaluate_matches_oracle_sparse_and_dense(q):
    import torch
    rng = np.random.default_rng(3)
    for inst in (wl.random_instance(42, 4, "deg3", seed=61, num_edges=48),
                 wl.random_instance(100, 3, "p0.9", seed=62),          # > 4096 edges: block kernel
                 wl.random_instance(130, 2, "p0.05", seed=63)):        # 3 words per row
        prob = q.problem_from_instance(inst)
        s = (1 - 2 * rng.integers(0, 2, size=(777, inst.n))).astype(np.int8)
        got = q.qaia_evaluate(prob, _dev(pack_spins(s)))
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), oracle.cut_values(inst, s))
        flipped = q.qaia_evaluate(prob, _dev(pack_spins(-s)))
        assert np.array_equal(flipped.cpu().numpy(), got.cpu().numpy())


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("path", SPARSE_PATHS)
def test_scale_invariance_bitwise(q, path):
    """c0 normalises J(c): c -> 4c or every weight -> 8W leaves the spins bit-identical."""
    inst = wl.random_instance(20, 3, "deg3", seed=71, num_edges=26)
    c = wl.dirichlet_weights(16, 3, 72)
    prob = q.problem_from_instance(inst)
    base, _, _ = _sample(q, prob, c, 8, steps=300, seed=73, path=path)
    c4, _, _ = _sample(q, prob, (c * 4).astype(np.float32), 8, steps=300, seed=73, path=path)
    inst8 = wl.Instance(inst.n, inst.m, inst.edge_u, inst.edge_v, inst.weights * 8)
    w8, _, _ = _sample(q, q.problem_from_instance(inst8), c, 8, steps=300, seed=73, path=path)
    assert np.array_equal(base, c4) and np.array_equal(base, w8)


@pytest.mark.parametrize("path", SPARSE_PATHS)
def test_determinism_and_replica_offset(q, path):
    inst = wl.random_instance(30, 4, "deg3", seed=81, num_edges=40)
    c = wl.dirichlet_weights(12, 4, 82)
    prob = q.problem_from_instance(inst)
    a, oa, _ = _sample(q, prob, c, 4, steps=200, seed=83, path=path)
    b, ob, _ = _sample(q, prob, c, 4, steps=200, seed=83, path=path)
    assert np.array_equal(a, b) and np.array_equal(oa, ob)
    tail, otail, _ = _sample(q, prob, c[5:], 4, steps=200, seed=83, replica_offset=20, path=path)
    assert np.array_equal(a[20:], tail) and np.array_equal(oa[20:], otail)


def test_paths_agree_with_each_other_bitwise_on_cuts(q):
    """The two sparse kernels produce cut vectors consistent with their own spins."""
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3", count=20)
    prob = q.problem_from_instance(inst)
    for path in SPARSE_PATHS:
        spins, obj, _ = _sample(q, prob, c, 16, steps=500, seed=5, path=path)
        assert np.array_equal(obj, oracle.cut_values(inst, unpack_spins(spins, inst.n)))


@pytest.mark.parametrize("path", SPARSE_PATHS)
def test_invalid_weight_rows_are_reported(q, path):
    inst = wl.random_instance(12, 3, "deg3", seed=91, num_edges=16)
    c = wl.dirichlet_weights(5, 3, 92)
    c[1] = [0.5, -0.1, 0.6]
    c[3] = [0.0, 0.0, 0.0]
    prob = q.problem_from_instance(inst)
    spins, obj, ws = _sample(q, prob, c, 4, steps=100, seed=1, path=path)
    assert q.qaia_workspace_status(ws) == 1
    assert not spins[4:8].any() and not obj[4:8].any()
    assert not spins[12:16].any() and not obj[12:16].any()
    ok, _, ws2 = _sample(q, prob, wl.dirichlet_weights(5, 3, 92), 4, steps=100, seed=1, path=path)
    assert q.qaia_workspace_status(ws2) is None


def test_argument_errors(q):
    import torch
    inst = wl.random_instance(12, 3, "deg3", seed=91, num_edges=16)
    prob = q.problem_from_instance(inst)
    c = _dev(wl.dirichlet_weights(4, 3, 1))
    for kw, status in ((dict(steps=0), q.QAIA_INVALID_ARGUMENT), (dict(dt=-1.0), q.QAIA_INVALID_ARGUMENT),
                       (dict(variant="bsb", precision="bf16"), q.QAIA_UNSUPPORTED)):
        with pytest.raises(q.QaiaError) as ei:
            q.qaia_sample(prob, c, 4, q.make_schedule(**kw))
        assert ei.value.status == status
    s = q.make_schedule(steps=10)
    need = q.qaia_sample_workspace_bytes(prob, 4, 4, s)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_sample(prob, c, 4, s, workspace=small)
    assert ei.value.status == q.QAIA_WORKSPACE_TOO_SMALL


def test_edge_cases_tiny_graphs(q):
    # one spin, no edges: c0 = 0, cut values are 0
    inst = wl.Instance(1, 2, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((2, 0), np.int32))
    prob = q.problem_from_instance(inst)
    c = wl.dirichlet_weights(3, 2, 1)
    for path in SPARSE_PATHS:
        spins, obj, _ = _sample(q, prob, c, 2, steps=50, seed=1, path=path)
        assert not obj.any() and spins.shape == (6, 1)
    # W = 0 is a no-op
    import torch
    _, obj0, _ = q.qaia_sample(prob, torch.zeros((0, 2), dtype=torch.float32, device="cuda"), 2,
                               q.make_schedule(steps=10))
    assert obj0.numel() == 0


def _traj_rel_error(x_gpu, x_ref):
    """Per row: max over steps and spins of |x_gpu - x_ref|, over max |x_ref| of the
    row's whole traced trajectory.  One- and two-spin trajectories pass close to
    zero every few steps, where a per-step relative norm is undefined."""
    num = np.abs(x_gpu.astype(np.float64) - x_ref).max(axis=(1, 2))
    return num / np.maximum(np.abs(x_ref).max(axis=(1, 2)), 1e-30)


@pytest.mark.parametrize("path", SPARSE_PATHS + ["dense", "dense_staged"])
def test_degenerate_graphs_every_path(q, path):
    """One spin with no edges and two spins with one positive edge, on every path
    and, for discrete SB on the dense paths, every field precision.

    * One spin: c0 = 0 (the c0 fallback of Eq. 9 with no couplings), so the spin
      is a free oscillator with stiffness a0 - a(t); its ballistic trace follows
      the FP64 oracle within 1e-5 of the trajectory's scale (FP32 rounding alone,
      emulated on the CPU with fused multiply-adds, reaches 1.1e-6 over 100
      steps); every cut is 0.
    * Two spins, one edge of positive weight: the antisymmetric normal mode has
      stiffness a0 - a(t) - c0 J = -a(t) and grows, so ballistic SB ends with the
      edge cut in every row (the sign of the coupling term in Eq. 9); the
      oracle ends the same way on these seeds.  Discrete SB can end with both
      spins aligned, so its rows are checked by exact evaluation only.
      This mode starts at zero stiffness, so a last-place rounding of the
      per-step coefficient -dt (a0 - a(t)) is a large relative error in its
      early growth; the trace is held to the first-order FP32 error bound
      carried along the oracle's trajectory (tests/fp32_bounds.py), which
      follows that amplification.
    """
    import torch
    c = wl.dirichlet_weights(5, 2, 81)
    precs = ["fp32"] if path in SPARSE_PATHS else ["fp32", "bf16", "fp8"]

    lone = wl.Instance(1, 2, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((2, 0), np.int32))
    prob = q.problem_from_instance(lone)
    s = q.make_schedule("bsb", steps=1000, dt=0.5, seed=82, path=path)
    _, obj, _, tr = q.qaia_sample_trace(prob, _dev(c), 4, s, 100)
    torch.cuda.synchronize()
    _, ref = oracle.sb_sample(lone, c, 4, 1000, "bsb", dt=0.5, seed=82, trace_steps=100)
    err = _traj_rel_error(tr.cpu().numpy(), ref)
    print(f"{path} one spin: max trajectory-relative error {err.max():.3e}")
    assert err.max() <= 1e-5
    assert not obj.cpu().numpy().any()
    for prec in precs:
        sp, ob, ws = _sample(q, prob, c, 4, variant="dsb", precision=prec, steps=200, seed=83, path=path)
        assert q.qaia_workspace_status(ws) is None
        assert sp.shape == (20, 1) and not ob.any(), prec
    _, obj0, _ = q.qaia_sample(prob, torch.zeros((0, 2), dtype=torch.float32, device="cuda"), 2,
                               q.make_schedule(steps=10, path=path))
    assert obj0.numel() == 0

    # integer weights (5 and 3) x 2^16: exact in bf16 and e4m3 after power-of-two scaling
    w = (np.array([[5], [3]], np.int64) << 16).astype(np.int32)
    pair = wl.Instance(2, 2, np.array([0], np.int32), np.array([1], np.int32), w)
    both_cut = np.array([5 << 16, 3 << 16], np.int64)
    prob = q.problem_from_instance(pair)
    s = q.make_schedule("bsb", steps=1000, dt=0.5, seed=84, path=path)
    spins, obj, _, tr = q.qaia_sample_trace(prob, _dev(c), 32, s, 100)
    torch.cuda.synchronize()
    sp_ref, ref = oracle.sb_sample(pair, c, 32, 1000, "bsb", dt=0.5, seed=84, trace_steps=100)
    assert (oracle.cut_values(pair, sp_ref) == both_cut).all()
    bound = fb.Bound(pair, c, 32, 1000, "bsb", seed=84, steps=100)
    ok, ratio, frac = bound.check(tr.cpu().numpy(), ref)
    print(f"{path} two spins: worst error / FP32 bound {ratio:.3f} over {frac:.0%} of the steps")
    assert ok and frac >= 0.9
    assert (obj.cpu().numpy() == both_cut).all()
    for prec in precs:
        sp, ob, ws = _sample(q, prob, c, 32, variant="dsb", precision=prec, steps=1000, seed=85, path=path)
        assert q.qaia_workspace_status(ws) is None
        assert np.array_equal(ob, oracle.cut_values(pair, unpack_spins(sp, 2))), prec


# ---------------------------------------------------------------- noise injection (Eq. 10)

ALL_PATHS = ["sparse_reg", "sparse_lds", "dense", "dense_staged"]


@pytest.mark.parametrize("path", ALL_PATHS)
def test_noise_draws_elementwise(q, path):
    """The device's Gaussian draws, one by one, against the oracle's float64
    Box-Muller.  Four spins without couplings (c0 = 0) start at x = y = 0
    (init_amp = 0); with dt = 0.5 and alpha = 0.25 the first step makes
    y = fl(dt alpha) eta = eta / 8 and x = dt a0 y = eta / 16 exactly, so the
    first traced x times 16 is the float32 draw itself.  16 384 replicas x 4
    spins = 65 536 draws, each within eta_error_bound(r, theta) of the exact
    value (the logf, sqrtf, cosf and argument roundings, at most
    2^-24 r (6 + 2 theta))."""
    import torch
    n, W, R, T, seed = 4, 64, 256, 1000, 91
    inst = wl.Instance(n, 1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((1, 0), np.int32))
    prob = q.problem_from_instance(inst)
    c = np.ones((W, 1), np.float32)
    s = q.make_schedule("bsb", steps=T, dt=0.5, init_amp=0.0, noise_alpha=0.25, seed=seed, path=path)
    _, _, ws, tr = q.qaia_sample_trace(prob, _dev(c), R, s, 1)
    torch.cuda.synchronize()
    assert q.qaia_workspace_status(ws) is None
    eta_dev = tr.cpu().numpy()[:, 0, :].astype(np.float64) * 16.0
    rows = W * R
    idx = [(g * T) * n + i for g in range(rows) for i in range(n)]
    eta_ref = np.array([oracle.noise_value(seed, k) for k in idx]).reshape(rows, n)
    model = np.array([nm.noise(seed, k) for k in idx]).reshape(rows, n, 3)
    assert (np.abs(model[..., 0] - eta_ref) <= 1e-12 * np.maximum(model[..., 1], 1)).all()
    bound = fb.eta_error_bound(model[..., 1], model[..., 2])
    err = np.abs(eta_dev - eta_ref)
    worst = float((err / np.where(bound > 0, bound, 1)).max())
    print(f"{path}: max |eta_f32 - eta| = {err.max():.3e}, worst fraction of the bound {worst:.3f}")
    assert (err <= bound).all()
    assert not (eta_dev == eta_dev[:, :1]).all()  # spins draw different values


def _noise_trace_case():
    inst = wl.random_instance(12, 3, "deg3", seed=41, num_edges=16)
    c = wl.dirichlet_weights(6, 3, 42)
    return inst, c, 8, 1000, 50, 0.15


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_noise_injected_trace_parity_every_seed(q, variant):
    """NI-SB (Eq. 10) against the FP64 oracle on every kernel family and every
    SB seed 43..59, 50 steps.  The tolerance is the first-order FP32 error
    bound carried along the oracle's trajectory (tests/fp32_bounds.py: local
    roundings, the device draw's error bound, propagation through the
    update's Jacobians, comparisons stopped where a wall or sign decision is
    within the bound of its threshold).  alpha = 0 must differ (the noise
    acts)."""
    import torch
    inst, c, R, T, steps, alpha = _noise_trace_case()
    prob = q.problem_from_instance(inst)
    worst, checked = 0.0, []
    for seed in range(43, 60):
        _, ref = oracle.sb_sample(inst, c, R, T, variant, dt=0.5, seed=seed, alpha=alpha, trace_steps=steps)
        bound = fb.Bound(inst, c, R, T, variant, alpha=alpha, seed=seed, steps=steps)
        for path in ALL_PATHS:
            s = q.make_schedule(variant, steps=T, dt=0.5, seed=seed, noise_alpha=alpha, path=path)
            _, _, _, tr = q.qaia_sample_trace(prob, _dev(c), R, s, steps)
            torch.cuda.synchronize()
            ok, ratio, frac = bound.check(tr.cpu().numpy(), ref)
            assert ok, (seed, path, ratio)
            worst = max(worst, ratio)
            checked.append(frac)
        if seed == 43:
            plain = q.make_schedule(variant, steps=T, dt=0.5, seed=seed, path="sparse_lds")
            _, _, _, tr0 = q.qaia_sample_trace(prob, _dev(c), R, plain, steps)
            assert not np.array_equal(tr0.cpu().numpy(), tr.cpu().numpy())
    print(f"noise-injected {variant}: worst error / bound {worst:.3f}, steps checked {np.mean(checked):.1%}")
    assert np.mean(checked) >= 0.95


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_noise_generated_kernel_matches_generic_kernel(q, variant):
    """Both sparse kernels evaluate the same float operations in the same order,
    noise included, so their spins, cuts and trajectories agree bit for bit."""
    import torch
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3", count=12)
    prob = q.problem_from_instance(inst)
    outs = []
    for path in ("sparse_reg", "sparse_lds"):
        s = q.make_schedule(variant, steps=600, dt=0.5, seed=77, noise_alpha=0.3, path=path,
                            replica_offset=1000)
        sp, ob, _, tr = q.qaia_sample_trace(prob, _dev(c), 16, s, 30)
        torch.cuda.synchronize()
        outs.append((sp.cpu().numpy(), ob.cpu().numpy(), tr.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
@pytest.mark.parametrize("steps", [1, 2, 3, 7, 301])
def test_generated_kernel_matches_generic_kernel_any_step_count(q, variant, steps):
    """The generated kernel's plain loop holds two SB steps (an odd count ends
    with one more), and its wall test is written as "clamping changed x"; the
    generic kernel runs one step per iteration with the |x| > 1 test.  Spins,
    cuts and the traced trajectories agree bit for bit at odd and even counts."""
    import torch
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3", count=10)
    prob = q.problem_from_instance(inst)
    outs = []
    for path in ("sparse_reg", "sparse_lds"):
        s = q.make_schedule(variant, steps=steps, dt=0.5, seed=90 + steps, path=path)
        sp, ob, _ = q.qaia_sample(prob, _dev(c), 8, s)
        _, _, _, tr = q.qaia_sample_trace(prob, _dev(c[:2]), 8, s, min(steps, 20))
        torch.cuda.synchronize()
        outs.append((sp.cpu().numpy(), ob.cpu().numpy(), tr.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
@pytest.mark.parametrize("n,edges", [(50, 75), (60, 90), (77, 78)])
def test_generated_kernel_register_budget_fallbacks(q, variant, n, edges):
    """Larger degree-3 graphs (2n + |E| = 175, 210, 232, the last the largest
    the register path admits) leave three waves per SIMD and, for some, the
    paired wall test behind: the build takes the first of its candidate forms
    whose step loop does not spill.  Whichever it takes, spins and cuts equal
    the generic kernel's bit for bit (odd step count)."""
    inst = wl.random_instance(n, 3, "deg3", seed=n, num_edges=edges)
    assert 2 * inst.n + inst.num_edges == 2 * n + edges
    c = wl.dirichlet_weights(6, 3, n + 1)
    prob = q.problem_from_instance(inst)
    outs = []
    for path in ("sparse_reg", "sparse_lds"):
        outs.append(_sample(q, prob, c, 64, variant=variant, steps=151, dt=0.5, seed=n + 2, path=path)[:2])
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("path", ["sparse_reg", "sparse_lds", "dense_staged"])
def test_noise_injected_sampling_exact_cuts(q, path):
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3", count=40)
    prob = q.problem_from_instance(inst)
    spins, obj, _ = _sample(q, prob, c, 16, steps=1000, seed=9, noise_alpha=0.15, path=path)
    assert np.array_equal(obj, oracle.cut_values(inst, unpack_spins(spins, inst.n)))
