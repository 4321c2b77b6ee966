"""Full-size parity: the headline workload (42-node, 4-objective graph, 20 000
weight vectors x 256 replicas x 2 000 steps, bSB and dSB) and the precision
workload (complete 2048-node, 3-objective graph, 512 x 8 columns x 1 000 dSB
steps) in the launch configuration the benchmark times.  The oracle cannot
run 10^10 replica-steps, so the checks are on sampled outputs:

* the cut vectors of sampled rows equal the oracle's evaluation of the
  returned spins (bit-exact);
* a replica's arithmetic does not depend on the other replicas of a launch,
  so sampled (weight vector, replica) pairs relaunched alone (one weight
  vector, one replica, replica_offset = its row) reproduce their row of the
  full launch bit for bit;
* for ballistic SB, those single-replica launches follow the FP64 oracle's
  trajectory within 1e-5 over the first 100 steps (the trajectory tolerance).
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


def _rows(rng, W, R, count):
    flat = rng.choice(W * R, size=count, replace=False)
    return [(int(r) // R, int(r) % R) for r in flat]


@pytest.mark.parametrize("variant,seed", [("bsb", 2003), ("dsb", 2004)])
def test_headline_workload_full_launch(q, variant, seed):
    import torch
    cfg = wl.WORKLOADS["c2_n42_m4"]
    W, R, T = cfg["W"], cfg["R"], cfg["T"]
    inst = wl.workload_instance("c2_n42_m4")
    c = wl.workload_weights("c2_n42_m4")
    prob = q.problem_from_instance(inst)
    s = q.make_schedule(variant, steps=T, dt=0.5, seed=seed)
    spins, obj, ws = q.qaia_sample(prob, _dev(c), R, s)
    torch.cuda.synchronize()
    assert q.qaia_workspace_status(ws) is None  # every weight row valid
    spins, obj = spins.cpu().numpy(), obj.cpu().numpy()
    rng = np.random.default_rng(11 if variant == "bsb" else 12)
    sample = _rows(rng, W, R, 64)
    idx = np.array([w * R + r for w, r in sample])
    assert np.array_equal(obj[idx], oracle.cut_values(inst, unpack_spins(spins[idx], inst.n)))
    for w, r in sample[:6]:
        one = q.make_schedule(variant, steps=T, dt=0.5, seed=seed, replica_offset=w * R + r)
        sp1, ob1, _ = q.qaia_sample(prob, _dev(c[w:w + 1]), 1, one)
        torch.cuda.synchronize()
        assert np.array_equal(sp1.cpu().numpy()[0], spins[w * R + r]), (w, r)
        assert np.array_equal(ob1.cpu().numpy()[0], obj[w * R + r]), (w, r)
        if variant == "bsb":
            sp2, _, _, tr = q.qaia_sample_trace(prob, _dev(c[w:w + 1]), 1, one, 100)
            torch.cuda.synchronize()
            assert np.array_equal(sp2.cpu().numpy()[0], spins[w * R + r]), (w, r)
            _, ref = oracle.sb_sample(inst, c[w:w + 1], 1, T, variant, dt=0.5, seed=seed,
                                      replica_offset=w * R + r, trace_steps=100)
            err = rel_inf_error(tr.cpu().numpy(), ref)
            assert err.max() <= 1e-5, (w, r, err.max())


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_precision_workload_full_launch(q, prec):
    import torch
    W, R, T = 512, 8, 1000
    inst = wl.random_instance(2048, 3, "complete", seed=3000)
    c = wl.dirichlet_weights(W, 3, 3002)
    prob = q.problem_from_instance(inst)
    s = q.make_schedule("dsb", precision=prec, steps=T, dt=0.5, seed=3003, path="dense_staged")
    spins, obj, ws = q.qaia_sample(prob, _dev(c), R, s)
    torch.cuda.synchronize()
    assert q.qaia_workspace_status(ws) is None  # every weight row valid
    spins, obj = spins.cpu().numpy(), obj.cpu().numpy()
    rng = np.random.default_rng({"fp32": 21, "bf16": 22, "fp8": 23}[prec])
    sample = _rows(rng, W, R, 16)
    idx = np.array([w * R + r for w, r in sample])
    assert np.array_equal(obj[idx], oracle.cut_values(inst, unpack_spins(spins[idx], inst.n)))
    # good partitions: each sampled row's scalarised cut is positive (a random
    # partition's expectation is half the total weight, near zero here)
    scal = np.array([obj[w * R + r].astype(np.float64) @ c[w] for w, r in sample])
    assert np.all(scal > 0)
    for w, r in sample[:3]:
        one = q.make_schedule("dsb", precision=prec, steps=T, dt=0.5, seed=3003, path="dense_staged",
                              replica_offset=w * R + r)
        sp1, ob1, _ = q.qaia_sample(prob, _dev(c[w:w + 1]), 1, one)
        torch.cuda.synchronize()
        assert np.array_equal(sp1.cpu().numpy()[0], spins[w * R + r]), (w, r)
        assert np.array_equal(ob1.cpu().numpy()[0], obj[w * R + r]), (w, r)


def test_headline_filter_full_pool(q):
    """The filter of the benchmark step at full size: the 10.24 M cut vectors of
    one bSB and one dSB launch of the headline workload, pooled.  The oracle's
    quadratic filter cannot take the whole pool, so the result is checked by
    properties that define it ("Pareto filtering", Eq. 4) plus a slice:

    * kept rows are pairwise distinct and mutually non-dominated;
    * each kept row is the smallest sample index carrying its vector
      (host lexicographic sort of the whole pool);
    * 10 000 sampled pool rows are each dominated by or equal to a kept row;
    * on the first 200 000 rows the GPU filter equals the oracle bit for bit.
    """
    import torch
    cfg = wl.WORKLOADS["c2_n42_m4"]
    W, R, T = cfg["W"], cfg["R"], cfg["T"]
    inst = wl.workload_instance("c2_n42_m4")
    prob = q.problem_from_instance(inst)
    c = _dev(wl.workload_weights("c2_n42_m4"))
    rows = W * R
    obj = torch.empty((2 * rows, inst.m), dtype=torch.int64, device="cuda")
    for i, v in enumerate(("bsb", "dsb")):
        s = q.make_schedule(v, steps=T, dt=0.5, seed=cfg["seed"] + 3 + i)
        q.qaia_sample(prob, c, R, s, obj=obj[i * rows:(i + 1) * rows])
    keep, num, _ = q.qaia_pareto_filter(obj)
    torch.cuda.synchronize()
    keep = keep[: int(num.item())].cpu().numpy()
    pool = obj.cpu().numpy()
    print(f"pool {pool.shape[0]} rows, front {keep.size}")
    assert keep.size > 100 and np.all(np.diff(keep) > 0)
    front = pool[keep]
    # distinct and mutually non-dominated
    ge = np.ones((keep.size, keep.size), bool)
    for k in range(inst.m):
        ge &= front[:, None, k] >= front[None, :, k]
    np.fill_diagonal(ge, False)
    assert not ge.any()
    # smallest index per vector: first row of each run in a stable lexicographic sort
    order = np.lexsort(tuple(pool[:, k] for k in reversed(range(inst.m))))
    srt = pool[order]
    first = np.ones(order.size, bool)
    first[1:] = (srt[1:] != srt[:-1]).any(axis=1)
    run_start = np.maximum.accumulate(np.where(first, np.arange(order.size), 0))
    pos = np.empty_like(order)
    pos[order] = np.arange(order.size)
    assert np.array_equal(order[run_start[pos[keep]]], keep)
    # sampled rows are dominated by or equal to a kept row
    rng = np.random.default_rng(5)
    for r in rng.choice(pool.shape[0], size=10000, replace=False):
        assert (front >= pool[r]).all(axis=1).any()
    # a slice against the oracle
    sl = torch.from_numpy(pool[:200000].copy()).cuda()
    k2, n2, _ = q.qaia_pareto_filter(sl)
    torch.cuda.synchronize()
    assert np.array_equal(k2[: int(n2.item())].cpu().numpy(), oracle.pareto_filter(pool[:200000]))
