"""qaia_sample_noalloc (the allocation-free sampling entry point, whose
workspace is the library's static device scratch) against qaia_sample through
the C ABI: identical spins and cuts on two calls in a row, the second with a
smaller input, on every kernel family; cut values checked against the oracle;
the invalid-row report; the size limit and the first-use refusal."""
import numpy as np
import pytest

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


def _pair(q, prob, c, R, s):
    """(spins, obj, bad) from qaia_sample and from qaia_sample_noalloc on the same inputs."""
    import torch
    cd = _dev(c)
    spins_a, obj_a, ws = q.qaia_sample(prob, cd, R, s)
    torch.cuda.synchronize()
    bad_a = q.qaia_workspace_status(ws)
    rows = c.shape[0] * R
    spins_b = torch.full((rows, prob.words), -7, dtype=torch.int64, device="cuda")
    obj_b = torch.full((rows, prob.m), -7, dtype=torch.int64, device="cuda")
    bad_b = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    q.qaia_sample_noalloc(prob, cd, R, s, spins_b, obj_b, bad_b)
    torch.cuda.synchronize()
    bad_b = int(bad_b.cpu()[0])
    return (spins_a.cpu().numpy(), obj_a.cpu().numpy(), -1 if bad_a is None else bad_a,
            spins_b.cpu().numpy(), obj_b.cpu().numpy(), bad_b)


CASES = [
    # (label, graph kind, n, m, variant, precision, path)
    ("register bSB", "deg3", 42, 3, "bsb", "fp32", "auto"),
    ("register dSB", "deg3", 42, 4, "dsb", "fp32", "sparse_reg"),
    ("LDS dSB", "deg3", 42, 3, "dsb", "fp32", "sparse_lds"),
    ("dense FP32 bSB", "complete", 40, 3, "bsb", "fp32", "dense_staged"),
    ("dense BF16 dSB", "complete", 40, 3, "dsb", "bf16", "dense_staged"),
]


@pytest.mark.parametrize("label,kind,n,m,variant,prec,path", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_sample_two_calls(q, label, kind, n, m, variant, prec, path):
    inst = (wl.instance_42_node(m, seed=901) if kind == "deg3"
            else wl.random_instance(n, m, "complete", seed=902))
    prob = q.problem_from_instance(inst)
    # first call: 48 weight vectors x 8 replicas, row 5 invalid (negative weight)
    c1 = wl.dirichlet_weights(48, m, 903)
    c1[5, 0] = -0.25
    # second call: smaller, every row valid (the stale invalid-row flag and
    # the larger first call's scratch contents must not leak into it)
    c2 = wl.dirichlet_weights(13, m, 904)
    for call, (c, R, seed) in enumerate([(c1, 8, 905), (c2, 3, 906)]):
        s = q.make_schedule(variant, prec, steps=300, dt=0.5, seed=seed, path=path)
        sa, oa, ba, sb, ob, bb = _pair(q, prob, c, R, s)
        print(f"{label} call {call}: rows {c.shape[0] * R}, bad row {ba} / {bb}", flush=True)
        assert np.array_equal(sa, sb), f"{label} call {call}: spins differ from qaia_sample"
        assert np.array_equal(oa, ob), f"{label} call {call}: cuts differ from qaia_sample"
        assert ba == bb == (5 if call == 0 else -1)
        # the invalid row's samples are zero; every other row's cuts are exact
        ok = np.ones(len(ob), bool)
        if call == 0:
            ok[5 * R:6 * R] = False
            assert not sb[~ok].any() and not ob[~ok].any()
        assert np.array_equal(ob[ok], oracle.cut_values(inst, unpack_spins(sb[ok], inst.n)))


def test_noalloc_size_limit_and_first_use(q):
    import torch
    inst = wl.instance_42_node(4, seed=907)
    prob = q.problem_from_instance(inst)
    s = q.make_schedule("bsb", steps=100, seed=908)
    # W * |E| * 4 bytes of folded coefficients past the 16 MiB scratch
    W = (q.NOALLOC_SCRATCH_BYTES // (4 * inst.num_edges)) + 1
    assert q.qaia_sample_workspace_bytes(prob, W, 1, s) > q.NOALLOC_SCRATCH_BYTES
    c = torch.full((W, inst.m), 0.25, dtype=torch.float32, device="cuda")
    spins = torch.empty((W, prob.words), dtype=torch.int64, device="cuda")
    obj = torch.empty((W, inst.m), dtype=torch.int64, device="cuda")
    with pytest.raises(q.QaiaError) as e:
        q.qaia_sample_noalloc(prob, c, 1, s, spins, obj)
    assert e.value.status == q.QAIA_WORKSPACE_TOO_SMALL
    # the noise-injected generated kernel does not exist before a qaia_sample call builds it
    sn = q.make_schedule("bsb", steps=100, seed=909, noise_alpha=0.15, path="sparse_reg")
    cs = _dev(wl.dirichlet_weights(8, inst.m, 910))
    with pytest.raises(q.QaiaError) as e:
        q.qaia_sample_noalloc(prob, cs, 4, sn, spins[:32], obj[:32])
    assert e.value.status == q.QAIA_UNSUPPORTED
    sa, oa, ba, sb, ob, bb = _pair(q, prob, wl.dirichlet_weights(8, inst.m, 910), 4, sn)
    assert np.array_equal(sa, sb) and np.array_equal(oa, ob) and ba == bb == -1
