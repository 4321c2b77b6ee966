"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a
printed example (tests/golden), a closed form, an independent brute force, an
algebraic identity computed by a different route, or an invariant.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl


# --------------------------------------------------------------------------
# helpers written independently of the oracle
# --------------------------------------------------------------------------

def _instance(n, m, edges, weights):
    u = np.array([a for a, _ in edges], np.int32)
    v = np.array([b for _, b in edges], np.int32)
    return wl.Instance(n, m, u, v, np.asarray(weights, np.int32).reshape(m, len(edges)))


def _all_spins(n, fix_first=False):
    """Every configuration in {+1,-1}^n (optionally with s_0 = +1) as int8 rows."""
    k = n - 1 if fix_first else n
    codes = np.arange(2 ** k, dtype=np.int64)
    bits = ((codes[:, None] >> np.arange(k)[None, :]) & 1).astype(np.int8)
    s = 1 - 2 * bits
    if fix_first:
        s = np.concatenate([np.ones((s.shape[0], 1), np.int8), s], axis=1)
    return s


def _cut_identity(inst, spins):
    """C_k = 1/2 sum_E W (1 - s_u s_v): the algebraic form of Eq. (1)."""
    su = spins[:, inst.edge_u].astype(np.int64)
    sv = spins[:, inst.edge_v].astype(np.int64)
    ones_minus = 1 - su * sv  # 0 or 2
    return (ones_minus @ inst.weights.T.astype(np.int64)) // 2


def _nondominated_bruteforce(vecs):
    """Unique non-dominated rows by all-pairs comparison (numpy), as a set of tuples."""
    uniq = np.unique(vecs, axis=0)
    ge = (uniq[:, None, :] >= uniq[None, :, :]).all(axis=2)  # ge[a, b]: a >= b everywhere
    np.fill_diagonal(ge, False)
    dominated = ge.any(axis=0)  # some other unique row a >= b  => b dominated
    return {tuple(r) for r in uniq[~dominated]}


def _hv_inclusion_exclusion(points, ref):
    """Union volume by inclusion-exclusion over all non-empty subsets (Python ints)."""
    pts = [tuple(max(int(p[k]), int(ref[k])) for k in range(len(ref))) for p in points]
    total = 0
    for size in range(1, len(pts) + 1):
        sign = 1 if size % 2 else -1
        for sub in itertools.combinations(pts, size):
            vol = 1
            for k in range(len(ref)):
                vol *= min(p[k] for p in sub) - int(ref[k])
            total += sign * vol
    return total


def _hv_grid(points, ref):
    """Count unit cells [z, z+1) covered by some box, for small integer coordinates."""
    pts = np.asarray(points, np.int64)
    ref = np.asarray(ref, np.int64)
    hi = pts.max(axis=0)
    axes = [np.arange(ref[k], max(hi[k], ref[k])) for k in range(len(ref))]
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, len(ref))
    covered = np.zeros(grid.shape[0], bool)
    for p in pts:
        covered |= (grid < p[None, :]).all(axis=1)
    return int(covered.sum())


# --------------------------------------------------------------------------
# counter-based generator
# --------------------------------------------------------------------------

def test_splitmix64_reference_outputs(golden_dir):
    for line in open(os.path.join(golden_dir, "splitmix64_seed0.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, idx, val = line.split()
        assert oracle.splitmix64(int(seed), int(idx)) == int(val, 16)


def test_init_values_range_and_moments():
    vals = np.array([oracle.init_value(7, i, 0.1) for i in range(20000)])
    assert vals.min() >= -0.1 and vals.max() < 0.1
    # U(-0.1, 0.1): mean 0, variance 0.01/3 (4-sigma bounds)
    assert abs(vals.mean()) < 4 * math.sqrt(0.01 / 3 / vals.size)
    assert abs(vals.var() - 0.01 / 3) < 4 * 0.01 / 3 * math.sqrt(0.8 / vals.size)
    # every value is float32(amp * (k - 2^23) / 2^23) for an integer k
    k = np.round(vals.astype(np.float64) / np.float64(np.float32(0.1)) * 2**23)
    back = (np.float32(0.1) * ((k - 0) / 2**23).astype(np.float32)).astype(np.float32)
    assert np.array_equal(back, vals.astype(np.float32))


def test_noise_moments():
    eta = np.array([oracle.noise_value(3, i) for i in range(40000)])
    assert abs(eta.mean()) < 4 / math.sqrt(eta.size)
    assert abs(eta.var() - 1.0) < 4 * math.sqrt(2.0 / eta.size)
    # fourth moment of N(0,1) is 3
    assert abs((eta ** 4).mean() - 3.0) < 0.15
    # the whole distribution (Kolmogorov-Smirnov against N(0,1)) and
    # independence of successive counter positions (lag-1 correlation)
    from scipy import stats
    assert stats.kstest(eta, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(eta[:-1], eta[1:])[0, 1]) < 4 / math.sqrt(eta.size)


# --------------------------------------------------------------------------
# cut values, Eq. (1)
# --------------------------------------------------------------------------

def test_cut_identity_and_flip_invariance():
    inst = wl.random_instance(12, 3, "deg3", seed=11, num_edges=16)
    spins = _all_spins(12)[::7]
    obj = oracle.cut_values(inst, spins)
    assert np.array_equal(obj, _cut_identity(inst, spins))
    assert np.array_equal(obj, oracle.cut_values(inst, -spins))
    allplus = np.ones((1, 12), np.int8)
    assert np.array_equal(oracle.cut_values(inst, allplus), np.zeros((1, 3), np.int64))


def test_bipartite_max_cut_is_total_weight():
    # a 3x3 grid is bipartite; with positive weights the max cut takes every edge
    edges = []
    for r in range(3):
        for c in range(3):
            i = 3 * r + c
            if c < 2:
                edges.append((i, i + 1))
            if r < 2:
                edges.append((i, i + 3))
    rng = np.random.default_rng(0)
    w = rng.integers(1, 1000, size=(2, len(edges)))
    inst = _instance(9, 2, sorted(edges), w)
    obj = oracle.cut_values(inst, _all_spins(9))
    assert obj[:, 0].max() == w[0].sum() and obj[:, 1].max() == w[1].sum()


# --------------------------------------------------------------------------
# Pareto filter (section "Pareto filtering", Eq. (4) in cut space)
# --------------------------------------------------------------------------

def _check_filter(obj):
    keep = oracle.pareto_filter(obj)
    assert np.all(np.diff(keep) > 0)
    got = {tuple(obj[i]) for i in keep}
    assert got == _nondominated_bruteforce(obj)
    # representative is the smallest index carrying that vector
    for i in keep:
        first = np.flatnonzero((obj == obj[i]).all(axis=1))[0]
        assert first == i
    return keep


@pytest.mark.parametrize("n,m,seed", [(8, 2, 1), (10, 3, 2), (11, 4, 3)])
def test_filter_matches_bruteforce_front(n, m, seed):
    inst = wl.random_instance(n, m, "p0.6", seed=seed)
    spins = _all_spins(n, fix_first=True)
    obj = oracle.cut_values(inst, spins)
    _check_filter(obj)


def test_filter_properties_random_vectors():
    rng = np.random.default_rng(5)
    for trial in range(20):
        m = int(rng.integers(2, 5))
        M = int(rng.integers(1, 300))
        obj = rng.integers(-6, 7, size=(M, m)).astype(np.int64)
        keep = _check_filter(obj)
        front = obj[keep]
        # idempotent
        assert len(oracle.pareto_filter(front)) == len(front)
        # order invariance of the front as a set of vectors
        perm = rng.permutation(M)
        k2 = oracle.pareto_filter(obj[perm])
        assert {tuple(r) for r in obj[perm][k2]} == {tuple(r) for r in front}
        # merge law: ND(A u B) = ND(ND(A) u ND(B))
        half = M // 2
        a, b = obj[:half], obj[half:]
        parts = [x[oracle.pareto_filter(x)] for x in (a, b) if len(x)]
        merged = np.concatenate(parts) if parts else obj[:0]
        assert {tuple(r) for r in merged[oracle.pareto_filter(merged)]} == {tuple(r) for r in front}


def test_filter_empty_and_single():
    assert oracle.pareto_filter(np.zeros((0, 3), np.int64)).size == 0
    assert list(oracle.pareto_filter(np.array([[1, 2, 3]]))) == [0]
    assert list(oracle.pareto_filter(np.array([[1, 2], [1, 2], [0, 0]]))) == [0]


# --------------------------------------------------------------------------
# hypervolume, Eq. (6) and Appendix A
# --------------------------------------------------------------------------

def _read_hv_cases(path):
    cases, cur = [], None
    for line in open(path):
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "ref":
            cur = {"ref": [int(x) for x in t[1:]], "pts": []}
        elif t[0] == "pt":
            cur["pts"].append([int(x) for x in t[1:]])
        elif t[0] == "hv":
            cur["hv"] = int(t[1])
            cases.append(cur)
    return cases


def test_hv_appendix_a_worked_example(golden_dir):
    cases = _read_hv_cases(os.path.join(golden_dir, "hv_appendix_a.txt"))
    assert len(cases) == 2
    for c in cases:
        assert oracle.hypervolume(np.array(c["pts"]), c["ref"]) == c["hv"]


def test_hv_single_box_and_invariances():
    rng = np.random.default_rng(9)
    for m in (2, 3, 4):
        p = rng.integers(1, 10**6, size=m)
        assert oracle.hypervolume(p[None, :], np.zeros(m, np.int64)) == math.prod(int(x) for x in p)
    for trial in range(30):
        m = int(rng.integers(2, 5))
        P = int(rng.integers(1, 9))
        pts = rng.integers(-50, 200, size=(P, m))
        ref = rng.integers(-60, 10, size=m)
        hv = oracle.hypervolume(pts, ref)
        assert hv == _hv_inclusion_exclusion(pts, ref)
        # dominated and duplicate points do not change the union
        extra = np.concatenate([pts, pts[:1], np.minimum(pts[:1], pts[-1:])])
        assert oracle.hypervolume(extra, ref) == hv
        # permutation of points and of objectives
        perm = rng.permutation(m)
        assert oracle.hypervolume(pts[rng.permutation(P)][:, perm], ref[perm]) == hv
        # translation and per-axis integer scaling
        shift = rng.integers(-1000, 1000, size=m)
        assert oracle.hypervolume(pts + shift, ref + shift) == hv
        sc = rng.integers(1, 5, size=m)
        assert oracle.hypervolume(pts * sc, ref * sc) == hv * math.prod(int(x) for x in sc)


def test_hv_grid_count_small_coordinates():
    rng = np.random.default_rng(4)
    for trial in range(15):
        m = int(rng.integers(2, 5))
        pts = rng.integers(0, 7, size=(int(rng.integers(1, 12)), m))
        assert oracle.hypervolume(pts, np.zeros(m, np.int64)) == _hv_grid(pts, np.zeros(m, np.int64))


def test_hv_wide_range_exact():
    # 4 objectives near 2^40 each: volume ~ 2^160, beyond 128-bit arithmetic
    big = 2**40
    pts = np.array([[big, big - 3, big - 5, big - 7], [big - 11, big, big, big - 1]], np.int64)
    assert oracle.hypervolume(pts, np.zeros(4, np.int64)) == _hv_inclusion_exclusion(pts, [0] * 4)


# --------------------------------------------------------------------------
# coupling scale c0 and the SB dynamics (Eq. 9)
# --------------------------------------------------------------------------

def test_c0_closed_form_star_graph():
    # star: centre 0 with leaves 1..4, one objective; row sums are sum(w) at the
    # centre and w_i at leaf i, so c0 = 1 / max(|sum w|, max |w_i|)
    w = [3, -5, 2, 7]
    inst = _instance(5, 1, [(0, i) for i in range(1, 5)], [w])
    want = 1.0 / max(abs(sum(w)), max(abs(x) for x in w)) * 2**16
    assert oracle.c0(inst, np.array([1.0], np.float32)) == pytest.approx(want, rel=1e-15)
    # balanced weights: every row sum at the centre cancels -> still the leaf max
    inst2 = _instance(3, 1, [(0, 1), (0, 2)], [[4, -4]])
    assert oracle.c0(inst2, np.array([1.0], np.float32)) == pytest.approx(2**16 / 4.0, rel=1e-15)
    # all row sums zero (a 4-cycle with alternating signs) -> fallback to sum |J|
    inst3 = _instance(4, 1, [(0, 1), (0, 3), (1, 2), (2, 3)], [[2, -2, -2, 2]])
    assert oracle.c0(inst3, np.array([1.0], np.float32)) == pytest.approx(2**16 / 4.0, rel=1e-15)
    # no edges -> c0 = 0
    inst4 = _instance(3, 1, [], np.zeros((1, 0)))
    assert oracle.c0(inst4, np.array([1.0], np.float32)) == 0.0


def _exact_init(seed, g, n, i, comp, amp):
    return Fraction(oracle.init_value(seed, ((g * n + i) << 1) | comp, amp))


@pytest.mark.parametrize("jsign", [1, -1])
def test_two_spin_normal_modes_exact(jsign):
    """n = 2 with one edge: the sum and difference of the spins decouple.

    With c0 = 1/|J| the difference mode d = x1 - x2 has stiffness
    (a0 - a_t) - sgn(J) and the sum mode (a0 - a_t) + sgn(J).  For J > 0
    (a cut edge to be cut) d must grow and the spins end anti-aligned; for
    J < 0 they end aligned.  The mode recursions are run in exact rationals.
    """
    inst = _instance(2, 1, [(0, 1)], [[jsign * 3 * 2**16]])
    T, dt, a0, amp, seed = 400, Fraction(1, 2), Fraction(1), 0.1, 42
    c = np.array([1.0], np.float32)
    spins, trace = oracle.sb_sample(inst, c, R=1, T=T, variant="bsb", dt=0.5, seed=seed,
                                    trace_steps=T, amp=amp)
    x1, x2 = _exact_init(seed, 0, 2, 0, 0, amp), _exact_init(seed, 0, 2, 1, 0, amp)
    y1, y2 = _exact_init(seed, 0, 2, 0, 1, amp), _exact_init(seed, 0, 2, 1, 1, amp)
    d, yd, s, ys = x1 - x2, y1 - y2, x1 + x2, y1 + y2
    for t in range(T):
        at = a0 * Fraction(t, T - 1)
        yd += dt * (-(a0 - at) + jsign) * d
        ys += dt * (-(a0 - at) - jsign) * s
        d += dt * a0 * yd
        s += dt * a0 * ys
        x1n, x2n = (s + d) / 2, (s - d) / 2
        if abs(x1n) > 1 or abs(x2n) > 1:
            break  # the wall couples the modes from here on
        assert trace[0, t, 0] == pytest.approx(float(x1n), rel=1e-9, abs=1e-12)
        assert trace[0, t, 1] == pytest.approx(float(x2n), rel=1e-9, abs=1e-12)
    else:
        pytest.fail("no wall hit within T steps")
    assert t > 5
    assert (spins[0, 0] != spins[0, 1]) == (jsign > 0)


def _exact_sb(x, y, edges, jnorm, T, dt, a0, variant, noise=None):
    """Eq. (9)/(10) in exact rationals, every spin written out.

    x, y: lists of Fractions; edges: [(u, v, c0 J(c)_uv)] with the scaled
    coupling as a Fraction; noise(t, i) -> alpha * eta as a Fraction or None.
    Returns the x trace [T][n] (Fractions).  The force on spin i is
    -(a0 - a_t) x_i - sum_j c0 J(c)_ij phi(x_j) (+ alpha eta_i), phi the
    identity (bSB) or sgn with sgn(0) = +1 (dSB); y is updated first from
    the pre-step x, then x from the new y, then the inelastic wall.
    """
    n = len(x)
    out = []
    for t in range(T):
        at = a0 * Fraction(t, T - 1) if T > 1 else Fraction(0)
        if variant == "dsb":
            phi = [Fraction(1) if v >= 0 else Fraction(-1) for v in x]
        else:
            phi = list(x)
        force = [-(a0 - at) * x[i] for i in range(n)]
        for u, v, j in edges:
            force[u] -= j * phi[v]
            force[v] -= j * phi[u]
        if noise is not None:
            force = [force[i] + noise(t, i) for i in range(n)]
        y = [y[i] + dt * force[i] for i in range(n)]
        x = [x[i] + dt * a0 * y[i] for i in range(n)]
        for i in range(n):
            if abs(x[i]) > 1:
                x[i] = Fraction(1) if x[i] > 0 else Fraction(-1)
                y[i] = Fraction(0)
        out.append(list(x))
    return out


@pytest.mark.parametrize("jsign", [1, -1])
def test_two_spin_discrete_sb_exact(jsign):
    """dSB (phi = sgn) on two spins joined by one edge, in exact rationals.

    With W = 4 * 2^16 and c = 1 the scaled coupling c0 J(c) is exactly 1, so
    the discrete force is piecewise constant; the recursion runs through the
    wall hits to the end.  phi = x (which turns dSB into bSB) or a dropped
    coupling term gives a different trajectory; J > 0 must end cut, J < 0
    uncut (the coupling sign of Eq. 9 under the minimised Ising energy).
    """
    inst = _instance(2, 1, [(0, 1)], [[jsign * 4 * 2**16]])
    T, dt, a0, amp, seed = 60, Fraction(1, 2), Fraction(1), 0.1, 17
    c = np.array([1.0], np.float32)
    spins, trace = oracle.sb_sample(inst, c, R=1, T=T, variant="dsb", dt=0.5, seed=seed,
                                    trace_steps=T, amp=amp)
    x = [_exact_init(seed, 0, 2, i, 0, amp) for i in range(2)]
    y = [_exact_init(seed, 0, 2, i, 1, amp) for i in range(2)]
    want = _exact_sb(x, y, [(0, 1, Fraction(jsign))], None, T, dt, a0, "dsb")
    walls = 0
    for t in range(T):
        for i in range(2):
            assert trace[0, t, i] == pytest.approx(float(want[t][i]), rel=1e-12, abs=1e-14), (t, i)
        walls += sum(abs(v) == 1 for v in want[t])
    assert walls > 0  # the comparison ran through wall hits
    assert (spins[0, 0] != spins[0, 1]) == (jsign > 0)
    # and the discrete trajectory is not the ballistic one
    _, trace_b = oracle.sb_sample(inst, c, R=1, T=T, variant="bsb", dt=0.5, seed=seed, trace_steps=T, amp=amp)
    assert np.abs(trace_b - trace).max() > 0.1


def test_discrete_sb_sign_of_zero_is_plus_one():
    """init_amp = 0: every spin starts at x = y = 0, so the first discrete force
    is -c0 J(c) sgn(0) = -c0 J(c) with sgn(0) = +1 (the read-out convention).
    sgn(0) = 0 would leave x at 0 forever and sgn(0) = -1 would move it the
    other way.  Three spins: an edge 0-1 (J > 0) and a lone spin 2, which has
    no force and stays at 0 (read out as +1)."""
    inst = _instance(3, 1, [(0, 1)], [[2 * 2**16]])
    T, dt, a0 = 40, Fraction(1, 2), Fraction(1)
    c = np.array([1.0], np.float32)
    spins, trace = oracle.sb_sample(inst, c, R=2, T=T, variant="dsb", dt=0.5, seed=3, trace_steps=T, amp=0.0)
    zero = [Fraction(0)] * 3
    want = _exact_sb(list(zero), list(zero), [(0, 1, Fraction(1))], None, T, dt, a0, "dsb")
    assert float(want[0][0]) == -0.25 and float(want[0][1]) == -0.25
    for r in range(2):
        for t in range(T):
            for i in range(3):
                assert trace[r, t, i] == pytest.approx(float(want[t][i]), rel=1e-12, abs=1e-14), (r, t, i)
    assert (spins[:, 2] == 1).all()
    # ballistic SB from the origin never moves (phi(0) = 0)
    _, trace_b = oracle.sb_sample(inst, c, R=1, T=T, variant="bsb", dt=0.5, seed=3, trace_steps=T, amp=0.0)
    assert not trace_b.any()


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_noise_injection_exact_on_free_spins(variant):
    """Eq. (10) on spins without couplings (c0 = 0): each spin is a driven
    oscillator y += dt (-(a0 - a_t) x + alpha eta), x += dt a0 y, with the wall.

    eta comes from the test's own SplitMix64 + Box-Muller (tests/noise_model),
    counter (g T + t) n + i of the stream keyed seed ^ 0xd1b54a32d192ed03, and
    the recursion runs in exact rationals.  Noise added to x instead of y, a
    missing dt factor, a wrong sign or a wrong counter (replica, step or spin
    index) each give a different trajectory.  Two weight vectors x three
    replicas x two spins cover the counter layout."""
    import noise_model as nm
    inst = _instance(2, 1, [], np.zeros((1, 0)))
    W, R, T, alpha, seed, amp = 2, 3, 40, 0.3, 29, 0.1
    dt, a0 = Fraction(1, 2), Fraction(1)
    c = np.array([[1.0], [0.5]], np.float32)
    _, trace = oracle.sb_sample(inst, c, R=R, T=T, variant=variant, dt=0.5, seed=seed, alpha=alpha,
                                trace_steps=T, amp=amp)
    hits = 0
    for g in range(W * R):
        x = [_exact_init(seed, g, 2, i, 0, amp) for i in range(2)]
        y = [_exact_init(seed, g, 2, i, 1, amp) for i in range(2)]

        def noise(t, i, g=g):
            return Fraction(alpha) * Fraction(nm.noise(seed, nm.noise_counter(g, T, t, 2, i))[0])
        want = _exact_sb(x, y, [], None, T, dt, a0, variant, noise=noise)
        for t in range(T):
            for i in range(2):
                assert trace[g, t, i] == pytest.approx(float(want[t][i]), rel=1e-12, abs=1e-14), (g, t, i)
            hits += sum(abs(v) == 1 for v in want[t])
    assert hits > 0  # the noise drives spins into the wall within T steps


def test_python_splitmix_matches_published_outputs(golden_dir):
    import noise_model as nm
    with open(os.path.join(golden_dir, "splitmix64_seed0.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, idx, val = line.split()
            assert nm.splitmix64(int(seed), int(idx)) == int(val, 16)


def test_wall_is_inelastic_and_bounds_x():
    inst = wl.random_instance(10, 2, "deg3", seed=3, num_edges=12)
    c = wl.dirichlet_weights(4, 2, 1)
    _, tr = oracle.sb_sample(inst, c, R=3, T=300, variant="bsb", trace_steps=300, seed=1)
    assert np.abs(tr).max() <= 1.0
    assert np.any(np.abs(tr) == 1.0)  # x projected exactly onto the wall


def test_scale_invariance_of_spins():
    """c0 normalises J(c): scaling c or every weight by 2^p leaves spins unchanged (bitwise)."""
    inst = wl.random_instance(14, 3, "deg3", seed=8, num_edges=18)
    c = wl.dirichlet_weights(5, 3, 2)
    for variant in ("bsb", "dsb"):
        base = oracle.sb_sample(inst, c, R=4, T=200, variant=variant, seed=5)
        scaled_c = oracle.sb_sample(inst, (c * 8).astype(np.float32), R=4, T=200, variant=variant, seed=5)
        inst2 = wl.Instance(inst.n, inst.m, inst.edge_u, inst.edge_v, inst.weights * 4)
        scaled_w = oracle.sb_sample(inst2, c, R=4, T=200, variant=variant, seed=5)
        assert np.array_equal(base, scaled_c) and np.array_equal(base, scaled_w)


def test_replica_offset_continues_streams():
    inst = wl.random_instance(10, 2, "deg3", seed=4, num_edges=12)
    c = wl.dirichlet_weights(4, 2, 3)
    full = oracle.sb_sample(inst, c, R=2, T=50, seed=9)
    second = oracle.sb_sample(inst, c[2:], R=2, T=50, seed=9, replica_offset=4)
    assert np.array_equal(full[4:], second)


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_sampler_recovers_bruteforce_front(variant):
    """On a 12-node instance the sampled front must cover most of the true front.

    The true front comes from enumerating all 2^11 configurations with s_0
    fixed.  A sign error in the coupling would steer SB to *minimum* cuts and
    recover almost nothing.
    """
    inst = wl.random_instance(12, 3, "p0.5", seed=21)
    true_front = _nondominated_bruteforce(oracle.cut_values(inst, _all_spins(12, fix_first=True)))
    c = wl.dirichlet_weights(300, 3, 22)
    spins = oracle.sb_sample(inst, c, R=4, T=300, variant=variant, seed=23)
    obj = oracle.cut_values(inst, spins)
    found = {tuple(obj[i]) for i in oracle.pareto_filter(obj)}
    # every sampled non-dominated vector is attainable, hence dominated-or-equal
    tf = np.array(sorted(true_front))
    for v in found:
        assert ((tf >= np.array(v)).all(axis=1)).any()
    recall = len(found & true_front) / len(true_front)
    # plain SB recovers about 0.3 here; the sign-flipped dynamics recover 0
    assert recall >= 0.2, recall
    # noise injection (Eq. 10) diversifies the samples and raises recall
    spins_n = oracle.sb_sample(inst, c, R=4, T=300, variant=variant, seed=23, alpha=0.15)
    obj_n = oracle.cut_values(inst, spins_n)
    found_n = {tuple(obj_n[i]) for i in oracle.pareto_filter(obj_n)}
    assert len(found_n & true_front) > len(found & true_front)


def test_objective_fields_match_dense_matmul():
    inst = wl.random_instance(16, 3, "p0.4", seed=13)
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((5, 16))
    out = oracle.objective_fields(inst, phi)
    for k in range(3):
        J = np.zeros((16, 16))
        J[inst.edge_u, inst.edge_v] = inst.weights[k]
        J[inst.edge_v, inst.edge_u] = inst.weights[k]
        np.testing.assert_allclose(out[:, k, :], phi @ J.T, rtol=1e-12, atol=1e-6)


# --------------------------------------------------------------------------
# input generators
# --------------------------------------------------------------------------

def test_degree_bounded_graph_shape():
    for seed in range(5):
        u, v = wl.degree_bounded_graph(42, 48, 3, seed)
        assert len(u) == 48 and np.all(u < v)
        assert len({(a, b) for a, b in zip(u, v)}) == 48
        deg = np.bincount(np.concatenate([u, v]), minlength=42)
        assert deg.max() <= 3


def test_weight_and_dirichlet_moments():
    w = wl.gaussian_weights(4, 20000, seed=1).astype(np.float64)
    assert abs(w.mean()) < 4 * 2**16 / math.sqrt(w.size)
    assert abs(w.std() / 2**16 - 1.0) < 4 * math.sqrt(0.5 / w.size)
    for m in (3, 4):
        c = wl.dirichlet_weights(50000, m, seed=2).astype(np.float64)
        np.testing.assert_allclose(c.sum(axis=1), 1.0, atol=1e-6)
        assert np.all(c >= 0)
        var = (m - 1) / (m * m * (m + 1))
        assert np.all(np.abs(c.mean(axis=0) - 1.0 / m) < 4 * math.sqrt(var / c.shape[0]))
        assert np.all(np.abs(c.var(axis=0) - var) < 0.05 * var)


def test_das_dennis_counts():
    assert wl.das_dennis_interior(3, 21).shape == (190, 3)
    assert wl.das_dennis_interior(4, 13).shape == (220, 4)
    d = wl.das_dennis_interior(3, 21).astype(np.float64)
    assert np.all(d > 0) and np.allclose(d.sum(axis=1), 1.0, atol=1e-6)


def test_appendix_e_correlation_closed_form():
    """Cut-value correlation of the Appendix E construction.

    For uniformly random spins the edge indicators are pairwise independent
    Bernoulli(1/2), so corr(C1, C2) = sum J1 J2 / sqrt(sum J1^2 sum J2^2),
    whose expectation is -4.8 / sqrt(2 * 25.04) = -0.678 (the paper quotes
    about -0.7), while C3 is uncorrelated.
    """
    inst = wl.appendix_e_instance(40, 1.0, seed=3)
    rng = np.random.default_rng(0)
    s = (1 - 2 * rng.integers(0, 2, size=(20000, 40))).astype(np.int8)
    obj = oracle.cut_values(inst, s).astype(np.float64)
    r12 = np.corrcoef(obj[:, 0], obj[:, 1])[0, 1]
    r13 = np.corrcoef(obj[:, 0], obj[:, 2])[0, 1]
    assert abs(r12 - (-4.8 / math.sqrt(2 * 25.04))) < 0.05
    assert abs(r13) < 0.1


# --------------------------------------------------------------------------
# Non-dominated ranks (non-dominated sorting of the sample pool)
# --------------------------------------------------------------------------

def _longest_chain_ranks(obj):
    """Independent characterisation: rank(y) = 1 + max rank of the rows that
    dominate y (0 if none), by dynamic programming in an order where every
    dominator comes first (descending coordinate sum)."""
    M = obj.shape[0]
    order = np.argsort(-obj.sum(axis=1), kind="stable")
    rank = np.zeros(M, np.int64)
    for a_pos, a in enumerate(order):
        best = -1
        for b in order[:a_pos]:
            if np.all(obj[b] >= obj[a]) and np.any(obj[b] > obj[a]):
                best = max(best, rank[b])
        rank[a] = best + 1
    return rank


@pytest.mark.parametrize("m,seed", [(2, 1), (3, 2), (4, 3)])
def test_ranks_match_longest_dominance_chain(m, seed):
    rng = np.random.default_rng(seed)
    obj = rng.integers(0, 6, size=(120, m)).astype(np.int64)
    ranks = oracle.pareto_ranks(obj)
    assert np.array_equal(ranks, _longest_chain_ranks(obj))


def test_ranks_front_duplicates_and_permutation():
    rng = np.random.default_rng(4)
    obj = rng.integers(-3, 4, size=(200, 3)).astype(np.int64)
    ranks = oracle.pareto_ranks(obj)
    # rank 0 is exactly the set of non-dominated vectors of the filter
    front = {tuple(v) for v in obj[oracle.pareto_filter(obj)]}
    assert {tuple(v) for v in obj[ranks == 0]} == front
    # equal rows share a rank; ranks are contiguous from 0
    for v in {tuple(r) for r in obj}:
        assert len(set(ranks[(obj == v).all(axis=1)])) == 1
    assert set(ranks) == set(range(ranks.max() + 1))
    # a permutation of the rows permutes the ranks
    perm = rng.permutation(len(obj))
    assert np.array_equal(oracle.pareto_ranks(obj[perm]), ranks[perm])


def test_ranks_chain_and_antichain():
    chain = np.array([[i, i] for i in range(7)], np.int64)  # totally ordered: 7 ranks
    assert list(oracle.pareto_ranks(chain)) == [6, 5, 4, 3, 2, 1, 0]
    anti = np.array([[i, 6 - i] for i in range(7)], np.int64)  # mutually non-dominated
    assert list(oracle.pareto_ranks(anti)) == [0] * 7
    assert oracle.pareto_ranks(np.zeros((0, 3), np.int64)).size == 0
