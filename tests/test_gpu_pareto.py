"""GPU non-dominated filter (qaia_pareto_filter) against the oracle: the same
index sets, bit for bit."""
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


def _filter(q, obj):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(obj, np.int64)).cuda()
    keep, num, _ = q.qaia_pareto_filter(t)
    torch.cuda.synchronize()
    return keep[: int(num.item())].cpu().numpy()


@pytest.mark.parametrize("M,m,lo,hi", [
    (1, 3, -5, 5), (2, 2, 0, 1), (7, 4, -3, 3), (1000, 2, -50, 50), (1000, 3, 0, 6),
    (3000, 4, -10, 10), (5000, 1, -100, 100), (4097, 8, -2, 2), (20000, 3, -1000, 1000),
])
def test_filter_matches_oracle_random(q, M, m, lo, hi):
    rng = np.random.default_rng(M * 10 + m)
    obj = rng.integers(lo, hi + 1, size=(M, m)).astype(np.int64)
    assert np.array_equal(_filter(q, obj), oracle.pareto_filter(obj))


def test_filter_empty(q):
    assert _filter(q, np.zeros((0, 3), np.int64)).size == 0


def test_filter_anticorrelated_large_front(q):
    """Points on a hyperplane are mutually non-dominated: the whole set survives
    (spans many chunks in the global pass)."""
    rng = np.random.default_rng(5)
    a = rng.integers(0, 10**9, size=(6000, 2))
    obj = np.stack([a[:, 0], a[:, 1], 3 * 10**9 - a[:, 0] - a[:, 1]], axis=1).astype(np.int64)
    obj = np.concatenate([obj, obj[:100]])  # duplicates
    got = _filter(q, obj)
    assert np.array_equal(got, oracle.pareto_filter(obj))


def test_filter_full_int64_range(q):
    rng = np.random.default_rng(9)
    obj = rng.integers(-2**62, 2**62, size=(3000, 3)).astype(np.int64)
    obj[::7, 0] = np.iinfo(np.int64).max
    obj[::11, 1] = np.iinfo(np.int64).min
    assert np.array_equal(_filter(q, obj), oracle.pareto_filter(obj))


def test_filter_on_sampled_pool(q):
    """The 42-node 3-objective workload: filter the full pool of 3200 sampled cut
    vectors and compare with the oracle; the kept rows carry their own cut values."""
    import torch
    inst = wl.workload_instance("c1_bsb_n42_m3")
    c = wl.workload_weights("c1_bsb_n42_m3")
    prob = q.problem_from_instance(inst)
    spins, obj, _ = q.qaia_sample(prob, torch.from_numpy(c).cuda(), 16, q.make_schedule(steps=1000, seed=7))
    obj_t = obj
    keep, num, _ = q.qaia_pareto_filter(obj_t)
    torch.cuda.synchronize()
    got = keep[: int(num.item())].cpu().numpy()
    o = obj.cpu().numpy()
    assert np.array_equal(got, oracle.pareto_filter(o))
    s = unpack_spins(spins.cpu().numpy()[got], inst.n)
    assert np.array_equal(oracle.cut_values(inst, s), o[got])
    # exact hypervolume of that front: library vs oracle
    ref = np.zeros(3, np.int64)
    assert q.qaia_hypervolume(o[got], ref) == oracle.hypervolume(o[got], ref)
