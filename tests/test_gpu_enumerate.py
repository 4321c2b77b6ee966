"""GPU enumeration of cut values (brute-force reference fronts) and the
random-spin baseline generator, through the C ABI, against the CPU oracle."""
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


def _codes_to_spins(codes, n):
    codes = np.asarray(codes, np.uint64)
    bits = (codes[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)
    return np.where(bits == 1, -1, 1).astype(np.int8)


def test_enumerate_all_codes_small_graph(q):
    import torch
    inst = wl.random_instance(11, 3, "p0.5", seed=1101)
    prob = q.problem_from_instance(inst)
    obj = q.qaia_enumerate_cuts(prob, 0, 1 << 11)
    torch.cuda.synchronize()
    ref = oracle.cut_values(inst, _codes_to_spins(np.arange(1 << 11), 11))
    assert np.array_equal(obj.cpu().numpy(), ref)
    # C(s) = C(-s): the upper half mirrors the lower half
    ob = obj.cpu().numpy()
    mirror = (np.arange(1 << 10) ^ ((1 << 11) - 1))
    assert np.array_equal(ob[: 1 << 10], ob[mirror])


def test_enumerate_high_codes_wide_graph(q):
    import torch
    inst = wl.random_instance(40, 4, "p0.2", seed=1102)
    prob = q.problem_from_instance(inst)
    first = (1 << 38) + 987654321
    obj = q.qaia_enumerate_cuts(prob, first, 3000)
    torch.cuda.synchronize()
    ref = oracle.cut_values(inst, _codes_to_spins(first + np.arange(3000, dtype=np.uint64), 40))
    assert np.array_equal(obj.cpu().numpy(), ref)


def test_enumerate_argument_bounds(q):
    inst = wl.random_instance(12, 2, "p0.5", seed=1103)
    prob = q.problem_from_instance(inst)
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_enumerate_cuts(prob, (1 << 12) - 5, 6)
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT
    assert q.qaia_enumerate_cuts(prob, (1 << 12) - 5, 5).shape == (5, 2)
    big = wl.random_instance(64, 2, "deg3", seed=1104)
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_enumerate_cuts(q.problem_from_instance(big), 0, 4)
    assert ei.value.status == q.QAIA_UNSUPPORTED


@pytest.mark.parametrize("chunk", [1 << 20, 1 << 9])
def test_exact_front_matches_oracle_bruteforce(q, chunk):
    """Appendix-E-shaped correlated instance, n = 14: the enumerated front (one
    representative code per vector, the smallest) equals the oracle's filter
    over all 2^13 cuts; a small chunk exercises the running-front merge."""
    inst = wl.appendix_e_instance(14, 0.8, seed=1105)
    prob = q.problem_from_instance(inst)
    codes, front = q.exact_front(prob, chunk=chunk)
    all_obj = oracle.cut_values(inst, _codes_to_spins(np.arange(1 << 13), 14))
    keep = oracle.pareto_filter(all_obj)
    assert np.array_equal(codes, keep)
    assert np.array_equal(front, all_obj[keep])


def test_random_spins_properties(q):
    import torch
    n, count = 100, 20000
    a = q.qaia_random_spins(n, count, seed=5)
    b = q.qaia_random_spins(n, count, seed=5)
    c = q.qaia_random_spins(n, 500, seed=5, offset=1000)
    torch.cuda.synchronize()
    a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(a[1000:1500], c)
    s = unpack_spins(a, n)
    # bits >= n are zero, every spin is fair and uncorrelated with its neighbour
    assert (a.view(np.uint64)[:, 1] >> np.uint64(n - 64)).max() == 0
    frac = (s < 0).mean(axis=0)
    assert np.abs(frac - 0.5).max() < 0.02
    corr = np.mean(s[:, :-1].astype(np.float64) * s[:, 1:])
    assert abs(corr) < 0.01
    # the spins evaluate like any other
    inst = wl.random_instance(n, 3, "p0.1", seed=1106)
    prob = q.problem_from_instance(inst)
    obj = q.qaia_evaluate(prob, torch.from_numpy(a[:500]).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(obj.cpu().numpy(), oracle.cut_values(inst, s[:500]))


@pytest.mark.parametrize("n,kind,count", [(700, "p0.05", 150), (300, "complete", 64), (6100, "deg3", 40)])
def test_evaluate_large_edge_sets(q, n, kind, count):
    """Exact cut values through the large-graph evaluators: the replica-tiled
    kernel (ragged last tile of 64 replicas, several edge chunks) and, past its
    LDS budget (n > 5952), the one-block-per-replica kernel."""
    import torch
    inst = wl.random_instance(n, 3, kind, seed=1107, num_edges=(n * 8) // 7 if kind == "deg3" else None)
    assert inst.num_edges > 4096
    prob = q.problem_from_instance(inst)
    spins = q.qaia_random_spins(n, count, seed=9)
    obj = q.qaia_evaluate(prob, spins)
    torch.cuda.synchronize()
    ref = oracle.cut_values(inst, unpack_spins(spins.cpu().numpy(), n))
    assert np.array_equal(obj.cpu().numpy(), ref)


@pytest.mark.parametrize("m", [2, 3, 4, 8])
def test_dirichlet_weights_uniform_on_simplex(q, m):
    """Rows lie on the simplex, are reproducible and continue with offset, and
    each coordinate follows the Beta(1, m - 1) marginal of the uniform law
    (Kolmogorov-Smirnov distance well inside the 1e-3 level for 200 000 rows)."""
    import torch
    n = 200_000
    w = q.qaia_dirichlet_weights(m, n, seed=12)
    w2 = q.qaia_dirichlet_weights(m, 1000, seed=12, offset=5000)
    torch.cuda.synchronize()
    w, w2 = w.cpu().numpy().astype(np.float64), w2.cpu().numpy()
    assert np.all(w > 0) and np.allclose(w.sum(axis=1), 1.0, atol=1e-5)
    assert np.array_equal(w[5000:6000].astype(np.float32), w2)
    for k in range(m):
        x = np.sort(w[:, k])
        cdf = 1.0 - (1.0 - x) ** (m - 1)
        ks = np.max(np.abs(cdf - np.arange(1, n + 1) / n))
        assert ks < 1.95 / np.sqrt(n), (k, ks)
    assert abs(w.mean() - 1.0 / m) < 1e-3
