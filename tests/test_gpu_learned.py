"""GPU parity of the learned weight proposer's kernels against the float64
oracle (oracle/mlp.py), and what the trained network gains."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import mlp as omlp

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


def _bf16_round(a):
    """float32 -> bf16 (round half to even) -> float64, and the bit patterns."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return vals, bits


def _params(D, seed=0):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(omlp.n_params(D)) * 0.25).astype(np.float32)
    vals, bits = _bf16_round(theta)
    return theta, vals, bits


def test_forward_matches_oracle(q):
    D = 12
    _, vals, bits = _params(D, 1)
    for N in (1000, 31, 65536):
        X = np.random.default_rng(2).standard_normal((N, D)).astype(np.float32)
        got = q.qaia_mlp_forward(_dev(bits.view(np.int16)), D, _dev(X)).cpu().numpy()
        want, _ = omlp.forward(vals, X.astype(np.float64), D)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"forward N={N} rel err {err:.2e}")
        assert err < 1e-4


def _grad_magnitude(vals, X, y, D):
    """Running error magnitudes of the float32 forward and backward passes:
    every quantity is replaced by the sum of the magnitudes of the terms it is
    computed from, carried through the forward pass (so a pre-activation that
    cancels keeps the size of its terms) and then through the backward pass
    (first-order: a factor f(z) contributes |f'(z)| times the magnitude of z).
    Per parameter this is the scale to which float32 rounding along the whole
    chain is relative."""
    W1, b1, W2, b2, w3, b3 = (np.abs(p) for p in omlp.unpack(vals, D))
    z3, (X, z1, a1, z2, a2) = omlp.forward(vals, X, D)
    B = X.shape[0]
    phi = lambda z: np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)  # noqa: E731
    g1, g2 = np.abs(omlp.gelu_grad(z1)), np.abs(omlp.gelu_grad(z2))
    h1, h2 = np.abs(phi(z1) * (2.0 - z1 * z1)), np.abs(phi(z2) * (2.0 - z2 * z2))  # |gelu''|
    Xm = np.abs(X)
    Z1m = Xm @ W1.T + b1
    A1m = g1 * Z1m + np.abs(a1)
    Z2m = A1m @ W2.T + b2
    A2m = g2 * Z2m + np.abs(a2)
    Z3m = A2m @ w3 + b3[0]
    sig = 1.0 / (1.0 + np.exp(-z3))
    d3 = (sig * (1.0 - sig) * Z3m + np.abs(sig - y)) / B
    d2 = np.outer(d3, w3) * (g2 + h2 * Z2m)
    d1 = (d2 @ W2) * (g1 + h1 * Z1m)
    parts = [d1.T @ Xm, d1.sum(axis=0), d2.T @ A1m, d2.sum(axis=0), A2m.T @ d3, np.array([d3.sum()])]
    return np.concatenate([p.ravel() for p in parts])


@pytest.mark.parametrize("D,B", [(12, 1024), (11, 77), (12, 1), (16, 4097)])
def test_backward_matches_oracle(q, D, B):
    """Element by element: |g - g_ref| <= 1e-3 |g_ref| + 1e-5 S, with S the
    element's running error magnitude (_grad_magnitude).  1e-5 is about the
    float32 unit roundoff times the longest chain of operations (a 128-term
    sum plus the 12-term input layer and the activations), so an element that
    cancels to nearly zero is held to float32 rounding of its terms instead of
    a relative bound no float32 evaluation can meet."""
    _, vals, bits = _params(D, 3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((B, D)).astype(np.float32)
    y = rng.integers(0, 2, size=B).astype(np.float32)
    got = q.qaia_mlp_backward(_dev(bits.view(np.int16)), D, _dev(X), _dev(y)).cpu().numpy()
    want = omlp.backward(vals, X.astype(np.float64), y.astype(np.float64), D)
    scale = _grad_magnitude(vals, X.astype(np.float64), y.astype(np.float64), D)
    bound = 1e-3 * np.abs(want) + 1e-5 * scale
    excess = np.abs(got - want) / bound
    worst = int(np.argmax(excess))
    print(f"backward (D={D}, B={B}): worst element {worst} at {excess[worst]:.3f} of its bound, "
          f"max relative error {np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-30)):.2e}")
    assert excess.max() <= 1.0
    # the output-bias gradient is mean(sigmoid(z) - y)
    assert got[-1] == pytest.approx(want[-1], rel=1e-3, abs=1e-6)


def test_adam_matches_oracle(q):
    import torch
    n = 5000
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(n).astype(np.float32)
    g = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    m1 = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    m2 = (np.abs(rng.standard_normal(n)) * 1e-5).astype(np.float32)
    master, params = _dev(theta.copy()), torch.zeros(n, dtype=torch.int16, device="cuda")
    dm1, dm2 = _dev(m1.copy()), _dev(m2.copy())
    q.qaia_mlp_adam(master, params, dm1, dm2, _dev(g), step=3, lr=1e-3)
    want, wm, wv = omlp.adam(theta.astype(np.float64), g.astype(np.float64), m1.astype(np.float64),
                             m2.astype(np.float64), 3, lr=1e-3)
    got = master.cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-6)
    np.testing.assert_allclose(dm1.cpu().numpy(), wm, rtol=1e-5, atol=1e-9)
    # the bf16 copy is the round-to-nearest-even of the new master weights
    assert np.array_equal(params.cpu().numpy().view(np.uint16), _bf16_round(got)[1])


def test_training_loop_equals_its_steps(q):
    """qaia_mlp_train (the whole round's loop queued by the library) equals the
    same steps made one by one through qaia_topk, qaia_gather_rows,
    qaia_mlp_backward and qaia_mlp_adam, bit for bit, across a permutation
    boundary (n = 3000 rows, minibatches of 1024: two windows per pass)."""
    import torch
    D, n, B, steps, first = 12, 3000, 1024, 5, 7
    theta, _, bits = _params(D, 9)
    rng = np.random.default_rng(10)
    X = _dev(rng.standard_normal((n, D)).astype(np.float32))
    y = _dev(rng.integers(0, 2, size=n).astype(np.float32))
    m1 = _dev((rng.standard_normal(theta.size) * 1e-3).astype(np.float32))
    m2 = _dev((np.abs(rng.standard_normal(theta.size)) * 1e-5).astype(np.float32))
    A = [_dev(theta.copy()), _dev(bits.view(np.int16).copy()), m1.clone(), m2.clone()]
    Bv = [_dev(theta.copy()), _dev(bits.view(np.int16).copy()), m1.clone(), m2.clone()]
    q.qaia_mlp_train(A[0], A[1], A[2], A[3], D, X, y, B, steps, first, lr=1e-3, seed=1234)
    per_pass = n // B
    cnt = _dev(np.array([n], np.int64))
    zeros = torch.zeros(n, dtype=torch.float32, device="cuda")
    for t in range(steps):
        win = t % per_pass
        if win == 0:
            perm = q.qaia_topk(zeros, n, temperature=1.0, seed=1234 + 104729 * (first + t))
            xp = torch.empty((n, D), dtype=torch.float32, device="cuda")
            yp = torch.empty(n, dtype=torch.float32, device="cuda")
            q.qaia_gather_rows(X, perm, cnt, xp, n)
            q.qaia_gather_rows(y, perm, cnt, yp, n)
        g = q.qaia_mlp_backward(Bv[1], D, xp[win * B:(win + 1) * B], yp[win * B:(win + 1) * B])
        q.qaia_mlp_adam(Bv[0], Bv[1], Bv[2], Bv[3], g, first + t, lr=1e-3)
    torch.cuda.synchronize()
    for a, b in zip(A, Bv):
        assert torch.equal(a, b)
    assert not torch.equal(A[0], _dev(theta))


def test_features_match_oracle(q):
    rng = np.random.default_rng(6)
    m = 4
    front = rng.integers(-10**6, 10**7, size=(300, m)).astype(np.int64)
    cands = rng.dirichlet(np.ones(m), size=500).astype(np.float32)
    hits = rng.dirichlet(np.ones(m), size=5).astype(np.float32)
    misses = rng.dirichlet(np.ones(m), size=7).astype(np.float32)
    got = q.qaia_front_features(_dev(front), _dev(cands), _dev(hits), _dev(misses)).cpu().numpy()
    want = omlp.features(front, cands.astype(np.float64), hits.astype(np.float64), misses.astype(np.float64))
    np.testing.assert_array_equal(got[:, :m], cands)
    np.testing.assert_allclose(got[:, m:], want, rtol=0, atol=2e-5)
    # empty archive and no hits / misses
    got0 = q.qaia_front_features(_dev(front[:0]), _dev(cands), _dev(hits[:0]), _dev(misses[:0])).cpu().numpy()
    want0 = omlp.features(front[:0], cands.astype(np.float64), hits[:0], misses[:0])
    np.testing.assert_allclose(got0[:, m:], want0, rtol=0, atol=2e-6)


def test_topk_gather_and_labels(q):
    import torch
    rng = np.random.default_rng(7)
    scores = rng.standard_normal(65536).astype(np.float32)
    idx = q.qaia_topk(_dev(scores), 1024).cpu().numpy()
    assert np.array_equal(idx, np.argsort(-scores, kind="stable")[:1024])
    ties = np.repeat(np.arange(10, dtype=np.float32), 7)
    assert np.array_equal(q.qaia_topk(_dev(ties), 9).cpu().numpy(), np.argsort(-ties, kind="stable")[:9])
    # signed zeros tie, infinities at the ends, every item returned
    mix = np.array([0.0, -0.0, -np.inf, 1.5, -0.0, np.inf, -2.0, 0.0, 1.5, -np.inf], np.float32)
    mix = np.tile(mix, 1000)
    assert np.array_equal(q.qaia_topk(_dev(mix), len(mix)).cpu().numpy(), np.argsort(-mix, kind="stable"))
    # gather of float rows
    src = rng.standard_normal((100, 6)).astype(np.float32)
    pick = np.array([5, 0, 99, 42], np.int64)
    dst = torch.zeros((4, 6), dtype=torch.float32, device="cuda")
    q.qaia_gather_rows(_dev(src), _dev(pick), _dev(np.array([4], np.int64)), dst, 4)
    assert np.array_equal(dst.cpu().numpy(), src[pick])
    # labels: archive of 10 rows, then W = 5 weight rows x R = 3 replicas
    keep = np.array([2, 7, 10, 11, 18, 24], np.int64)  # new rows 10,11 -> w0; 18 -> w2; 24 -> w4
    lab = q.qaia_new_point_labels(_dev(keep), _dev(np.array([6], np.int64)), 10, 3, 5).cpu().numpy()
    assert np.array_equal(lab, [1, 0, 1, 0, 1])


def _race_rounds(q, prob, base, ref_rounds, contenders, seeds, cap=1.6):
    from paper_2604_26477_amd.learned import ProposerLoop, reference_run, time_to_hypervolume
    ref_hv, ref_s, _ = reference_run(prob, ref_rounds, 777, **base)
    out = {}
    for name, extra in contenders:
        kw = dict(base)
        kw.update(extra)
        ProposerLoop(prob, seed=5, judge="record", **kw).round()  # kernels built on first use
        out[name] = [time_to_hypervolume(ProposerLoop(prob, seed=sd, judge="record", **kw), ref_hv,
                                         int(ref_rounds * cap) + 1, max_seconds=ref_s * 4) for sd in seeds]
    return out


def test_trained_network_needs_fewer_rounds(q):
    """What the trained network gains over the method without it: on the
    42-node 4-objective instance (rounds of 1024 weight vectors x 256 replicas,
    bSB FP32) the learned proposer reaches the hypervolume of the uniform
    loop's 200th round (seed 777) in fewer rounds than uniform Dirichlet
    weight vectors, median over five seeds (a run that does not reach it
    within 1.6x the rounds counts as 1.6x)."""
    inst = wl.instance_42_node(4, seed=2000)
    prob = q.problem_from_instance(inst)
    runs = _race_rounds(q, prob, dict(R=256, steps=2000, n_cand=65536, n_sel=1024), 200,
                        (("uniform", dict(learned=False)), ("learned", dict(learned=True))), (11, 12, 13, 14, 15))
    rounds = {k: [r["rounds"] if r["reached"] else 321 for r in v] for k, v in runs.items()}
    secs = {k: [r["seconds"] for r in v] for k, v in runs.items()}
    print(f"rounds to the reference: {rounds}; seconds: {secs}")
    assert np.median(rounds["learned"]) < np.median(rounds["uniform"])


def test_combined_form_reaches_reference_first(q):
    """The batched low-precision + learned-proposal form (discrete SB on the
    BF16 matrix-core path, weight vectors from the learned proposer, each round
    one launch of 1024 weight vectors x 8 replicas) reaches the hypervolume of
    plain FP32 bSB's 10th round on a complete 512-node 4-objective graph in
    less wall time than plain FP32 bSB with uniform weight vectors."""
    inst = wl.random_instance(512, 4, "complete", seed=5000)
    prob = q.problem_from_instance(inst)
    base = dict(R=8, steps=1000, n_cand=65536, n_sel=1024, variant="bsb", precision="fp32")
    runs = _race_rounds(q, prob, base, 10,
                        (("plain_fp32", dict(learned=False)),
                         ("learned_dsb_bf16", dict(learned=True, variant="dsb", precision="bf16"))), (11,))
    plain, form = runs["plain_fp32"][0], runs["learned_dsb_bf16"][0]
    print(f"plain FP32: {plain['rounds']} rounds {plain['seconds']} s; learned + dSB BF16: {form['rounds']} rounds "
          f"{form['seconds']} s")
    assert form["reached"]
    assert not plain["reached"] or form["seconds"] < plain["seconds"]
