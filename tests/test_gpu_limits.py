"""Size limits of each sampling path, exercised at the limit and just past it,
through the C ABI.

* Generated kernel: state and edge coefficients in registers, for graphs with
  2n + |E| <= 232 and m <= 8.  At the limit it runs and agrees bit for bit
  with the generic kernel (both evaluate the same float operations in the same
  order); one edge more and an explicit request is UNSUPPORTED while the
  automatic choice falls to the generic kernel.
* Generic (LDS) kernel: n <= 4096 and degree <= 32.  A 4096-node circulant
  graph of degree exactly 32 (65 536 edges) follows the FP64 oracle; one node
  or one degree more is UNSUPPORTED, and the automatic choice moves to the
  dense path.
* Dense path: m <= 4 and images of at most 4 GiB; past either, an explicit
  request is UNSUPPORTED (the problem itself is still created).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import rel_inf_error, unpack_spins

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


def _run(q, prob, c, R, T, trace_steps, **kw):
    import torch
    s = q.make_schedule(steps=T, dt=0.5, **kw)
    sp, ob, ws, tr = q.qaia_sample_trace(prob, _dev(c), R, s, trace_steps)
    torch.cuda.synchronize()
    assert q.qaia_workspace_status(ws) is None
    return sp.cpu().numpy(), ob.cpu().numpy(), tr.cpu().numpy()


def _circulant(n, half, m, seed):
    """Node i joined to i + 1 .. i + half (mod n): every degree is 2 * half."""
    i = np.repeat(np.arange(n), half)
    j = (i + np.tile(np.arange(1, half + 1), n)) % n
    u, v = np.minimum(i, j), np.maximum(i, j)
    order = np.lexsort((v, u))
    u, v = u[order].astype(np.int32), v[order].astype(np.int32)
    return wl.Instance(n, m, u, v, wl.gaussian_weights(m, u.shape[0], seed, wl.FRAC_BITS))


def _unsupported(q, prob, c, R, path, **kw):
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_sample(prob, _dev(c), R, q.make_schedule(steps=10, path=path, **kw))
    assert ei.value.status == q.QAIA_UNSUPPORTED, ei.value


def test_register_kernel_limit(q):
    m = 8
    inst = wl.random_instance(80, m, "deg3", seed=95, num_edges=72)   # 2n + |E| = 232
    c = wl.dirichlet_weights(6, m, 96)
    prob = q.problem_from_instance(inst)
    outs = {path: _run(q, prob, c, 8, 400, 20, variant="bsb", seed=97, path=path)
            for path in ("sparse_reg", "sparse_lds", "auto")}
    for path in ("sparse_lds", "auto"):
        for a, b in zip(outs["sparse_reg"], outs[path]):
            assert np.array_equal(a, b), path
    sp, ob, tr = outs["sparse_reg"]
    assert np.array_equal(ob, oracle.cut_values(inst, unpack_spins(sp, inst.n)))
    _, ref = oracle.sb_sample(inst, c, 8, 400, "bsb", dt=0.5, seed=97, trace_steps=20)
    err = rel_inf_error(tr, ref)
    print(f"n=80 |E|=72 m=8: max rel err over 20 steps {err.max():.3e}")
    assert err.max() <= 1e-5

    over = wl.random_instance(80, m, "deg3", seed=95, num_edges=73)   # 2n + |E| = 233
    prob = q.problem_from_instance(over)
    _unsupported(q, prob, c, 8, "sparse_reg")
    lds = _run(q, prob, c, 8, 400, 20, variant="dsb", seed=98, path="sparse_lds")
    auto = _run(q, prob, c, 8, 400, 20, variant="dsb", seed=98, path="auto")
    for a, b in zip(lds, auto):
        assert np.array_equal(a, b)
    assert np.array_equal(lds[1], oracle.cut_values(over, unpack_spins(lds[0], over.n)))


def test_lds_kernel_limits(q):
    inst = _circulant(4096, 16, 2, seed=101)   # degree 32 everywhere, 65 536 edges
    assert inst.num_edges == 65536
    c = wl.dirichlet_weights(2, 2, 102)
    prob = q.problem_from_instance(inst)
    sp, ob, tr = _run(q, prob, c, 2, 50, 10, variant="bsb", seed=103, path="sparse_lds")
    assert np.array_equal(ob, oracle.cut_values(inst, unpack_spins(sp, inst.n)))
    _, ref = oracle.sb_sample(inst, c, 2, 50, "bsb", dt=0.5, seed=103, trace_steps=10)
    err = rel_inf_error(tr, ref)
    print(f"n=4096 degree 32: max rel err over 10 steps {err.max():.3e}")
    assert err.max() <= 1e-5
    # the automatic choice at this size is the generic kernel
    auto = _run(q, prob, c, 2, 50, 10, variant="bsb", seed=103, path="auto")
    assert np.array_equal(auto[0], sp) and np.array_equal(auto[2], tr)

    wide = _circulant(4097, 1, 2, seed=104)   # one node more than the LDS kernel holds
    prob = q.problem_from_instance(wide)
    _unsupported(q, prob, c, 2, "sparse_lds")
    staged = _run(q, prob, c, 2, 50, 10, variant="bsb", seed=105, path="dense_staged")
    auto = _run(q, prob, c, 2, 50, 10, variant="bsb", seed=105, path="auto")
    for a, b in zip(staged, auto):
        assert np.array_equal(a, b)
    assert np.array_equal(staged[1], oracle.cut_values(wide, unpack_spins(staged[0], wide.n)))

    hub = wl.Instance(40, 2, np.zeros(33, np.int32), np.arange(1, 34, dtype=np.int32),
                      wl.gaussian_weights(2, 33, 106, wl.FRAC_BITS))   # node 0 has degree 33
    prob = q.problem_from_instance(hub)
    _unsupported(q, prob, c, 2, "sparse_lds")


def test_dense_path_limits(q):
    five = wl.random_instance(60, 5, "p0.3", seed=107)   # maximum degree 24: the LDS kernel takes it
    prob = q.problem_from_instance(five)
    c5 = wl.dirichlet_weights(2, 5, 108)
    for path in ("dense", "dense_staged"):
        _unsupported(q, prob, c5, 2, path)
    sp, ob, _ = _run(q, prob, c5, 2, 50, 1, variant="bsb", seed=109, path="auto")
    assert np.array_equal(ob, oracle.cut_values(five, unpack_spins(sp, five.n)))

    # 4 objectives x 12 416^2 padded entries x 7 bytes (FP32 + BF16 + FP8 images) > 4 GiB
    big = _circulant(12400, 1, 4, seed=110)   # a ring
    prob = q.problem_from_instance(big)
    c4 = wl.dirichlet_weights(2, 4, 111)
    for path in ("dense", "dense_staged"):
        _unsupported(q, prob, c4, 2, path)
    _unsupported(q, prob, c4, 2, "auto", variant="dsb", precision="bf16")
