"""GPU tests of the batching form: a ragged batch sampled by one graph launch
must reproduce per-item qaia_sample calls bit for bit, on every replay."""
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


SPECS = [  # (n, m, kind, W, R, path)
    (42, 3, "deg3", 13, 5, "sparse_reg"),
    (42, 4, "deg3", 7, 9, "sparse_lds"),
    (200, 4, "deg3", 5, 32, "sparse_lds"),
    (90, 3, "p0.1", 6, 11, "dense"),
    (150, 4, "p0.5", 3, 40, "dense_staged"),
    (70, 3, "complete", 4, 8, "dense"),
    (260, 3, "p0.3", 5, 30, "dense_staged"),
    (300, 3, "deg3", 2, 3, "sparse_lds"),
    (180, 2, "p0.4", 4, 20, "dense_staged"),  # m <= 2: the grouped kernel's epilogue prefetch
]


def _build(q, variant):
    import torch
    probs, items = [], []
    for i, (n, m, kind, W, R, path) in enumerate(SPECS):
        inst = wl.random_instance(n, m, kind, seed=700 + i)
        p = q.problem_from_instance(inst)
        c = _dev(wl.dirichlet_weights(W, m, 800 + i))
        probs.append((inst, p, c, R, path))
        items.append(q.BatchItem(p, c, R, path))
    return probs, items


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_batch_matches_per_item_calls(q, variant):
    import torch
    probs, items = _build(q, variant)
    s = q.make_schedule(variant, steps=300, dt=0.5, seed=91)
    ref = []
    for inst, p, c, R, path in probs:
        sp, ob, _ = q.qaia_sample(p, c, R, q.make_schedule(variant, steps=300, dt=0.5, seed=91, path=path))
        ref.append((sp.clone(), ob.clone()))
    torch.cuda.synchronize()
    ws = None
    for replay in range(3):
        for it in items:
            it.spins.fill_(-1)
            it.obj.fill_(-1)
        ws = q.qaia_sample_batch(items, s, workspace=ws)
        torch.cuda.synchronize()
        for (inst, p, c, R, path), it, (sp, ob) in zip(probs, items, ref):
            assert torch.equal(it.spins, sp), (replay, inst.name, path)
            assert torch.equal(it.obj, ob), (replay, inst.name, path)
        # eager work between replays
        _ = q.qaia_sample(probs[0][1], probs[0][2], 2, q.make_schedule(variant, steps=10, seed=1))
        torch.cuda.synchronize()
    # and the cut values are exact for the returned spins
    for (inst, p, c, R, path), it in zip(probs, items):
        assert np.array_equal(it.obj.cpu().numpy(), oracle.cut_values(inst, unpack_spins(it.spins.cpu().numpy(), inst.n)))


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_batch_empty_single_and_no_items(q, variant):
    """Items with no weight vectors on every path sit beside full ones and are
    skipped; a one-item batch and a batch with only empty items work; an empty
    list is a no-op.  Full items match per-item calls bit for bit."""
    import torch
    specs = [  # (n, m, kind, W, R, path)
        (42, 3, "deg3", 0, 5, "sparse_reg"),
        (42, 4, "deg3", 6, 7, "sparse_lds"),
        (150, 3, "p0.5", 0, 8, "dense_staged"),
        (90, 2, "p0.2", 5, 9, "dense"),
        (60, 3, "deg3", 0, 4, "sparse_lds"),
        (42, 3, "deg3", 3, 6, "sparse_reg"),
        (80, 3, "p0.3", 0, 3, "dense"),
        (130, 3, "p0.4", 4, 10, "dense_staged"),
    ]
    s = q.make_schedule(variant, steps=200, dt=0.5, seed=93)
    probs, items = [], []
    for i, (n, m, kind, W, R, path) in enumerate(specs):
        inst = wl.random_instance(n, m, kind, seed=900 + i)
        p = q.problem_from_instance(inst)
        c = _dev(wl.dirichlet_weights(W, m, 950 + i)) if W else torch.zeros((0, m), dtype=torch.float32,
                                                                               device="cuda")
        probs.append((inst, p, c, R, path))
        items.append(q.BatchItem(p, c, R, path))

    def per_item(p, c, R, path):
        sp, ob, _ = q.qaia_sample(p, c, R, q.make_schedule(variant, steps=200, dt=0.5, seed=93, path=path))
        return sp, ob

    q.qaia_sample_batch(items, s)
    torch.cuda.synchronize()
    for (inst, p, c, R, path), it in zip(probs, items):
        if c.shape[0] == 0:
            assert it.spins.numel() == 0 and it.obj.numel() == 0
            continue
        sp, ob = per_item(p, c, R, path)
        torch.cuda.synchronize()
        assert torch.equal(it.spins, sp) and torch.equal(it.obj, ob), (inst.name, path)

    one = q.BatchItem(probs[7][1], probs[7][2], probs[7][3], "dense_staged")
    q.qaia_sample_batch([one], s)
    torch.cuda.synchronize()
    assert torch.equal(one.spins, items[7].spins) and torch.equal(one.obj, items[7].obj)

    q.qaia_sample_batch([it for it, spec in zip(items, specs) if spec[3] == 0], s)
    q.qaia_sample_batch([], s)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_batch_low_precision_dense(q, prec):
    import torch
    specs = [(90, 3, "p0.1", "dense"), (150, 4, "p0.5", "dense_staged"), (130, 3, "complete", "dense"),
             (200, 3, "complete", "dense_staged"), (160, 2, "complete", "dense_staged")]
    items, refs = [], []
    for i, (n, m, kind, path) in enumerate(specs):
        inst = wl.random_instance(n, m, kind, seed=900 + i)
        p = q.problem_from_instance(inst)
        c = _dev(wl.dirichlet_weights(5, m, 950 + i))
        items.append(q.BatchItem(p, c, 16, path))
        sp, ob, _ = q.qaia_sample(p, c, 16, q.make_schedule("dsb", precision=prec, steps=200, seed=3, path=path))
        refs.append((sp, ob))
    q.qaia_sample_batch(items, q.make_schedule("dsb", precision=prec, steps=200, seed=3))
    torch.cuda.synchronize()
    for it, (sp, ob) in zip(items, refs):
        assert torch.equal(it.spins, sp) and torch.equal(it.obj, ob)


def test_autotune_picks_valid_paths(q):
    import torch
    probs, items = _build(q, "bsb")
    for it in items:
        it.path = "auto"
    s = q.make_schedule("bsb", steps=400, dt=0.5, seed=5)
    est = q.qaia_plan_autotune(items, s, probe_steps=20)
    print([(spec[:3], it.path, it.tile, f"{e * 1e3:.2f} ms") for spec, it, e in zip(SPECS, items, est)])
    assert all(it.tile == 0 or it.path == "sparse_lds" for it in items)
    assert all(e > 0 for e in est)
    assert all(it.path in ("sparse_reg", "sparse_lds", "dense", "dense_staged") for it in items)
    # a small sparse graph never goes to the matrix cores, a 50%-dense one never to the LDS kernel
    assert items[0].path in ("sparse_reg", "sparse_lds")
    q.qaia_sample_batch(items, s)
    torch.cuda.synchronize()
    for (inst, p, c, R, path), it in zip(probs, items):
        sp, ob, _ = q.qaia_sample(p, c, R, q.make_schedule("bsb", steps=400, dt=0.5, seed=5, path=it.path))
        torch.cuda.synchronize()
        assert torch.equal(it.spins, sp) and torch.equal(it.obj, ob)


@pytest.mark.parametrize("variant", ["bsb", "dsb"])
def test_sparse_tiles_and_queue_match_per_item_calls(q, variant):
    """The generic sparse kernel with 2x and 4x its default replicas per block
    (several spins per lane), and many items of different sizes sharing one
    persistent work-queue launch: outputs equal per-item qaia_sample calls at
    the default tile, bit for bit, on two replays."""
    import torch
    specs = [  # (n, m, kind, W, R, tile multiplier)
        (42, 4, "deg3", 9, 7, 1), (42, 4, "deg3", 5, 13, 2), (42, 3, "deg3", 3, 30, 4),
        (100, 3, "deg3", 4, 17, 2), (64, 4, "deg3", 11, 3, 4), (250, 2, "deg3", 2, 9, 1),
        (120, 3, "deg3", 6, 8, 2), (33, 4, "deg3", 1, 50, 4),
    ]
    s = q.make_schedule(variant, steps=250, dt=0.5, seed=97)
    probs, items, refs = [], [], []
    for i, (n, m, kind, W, R, mult) in enumerate(specs):
        inst = wl.random_instance(n, m, kind, seed=1100 + i)
        p = q.problem_from_instance(inst)
        c = _dev(wl.dirichlet_weights(W, m, 1200 + i))
        probs.append((inst, p, c, R))
        items.append(q.BatchItem(p, c, R, "sparse_lds", tile=(256 // n) * mult if mult > 1 else 0))
        sp, ob, _ = q.qaia_sample(p, c, R, q.make_schedule(variant, steps=250, dt=0.5, seed=97, path="sparse_lds"))
        refs.append((sp, ob))
    ws = None
    for replay in range(2):
        for it in items:
            it.spins.fill_(-1)
            it.obj.fill_(-1)
        ws = q.qaia_sample_batch(items, s, workspace=ws)
        torch.cuda.synchronize()
        for spec, it, (sp, ob) in zip(specs, items, refs):
            assert torch.equal(it.spins, sp) and torch.equal(it.obj, ob), (replay, spec)


def test_tile_knob_rejected_where_it_does_not_apply(q):
    inst = wl.random_instance(42, 3, "deg3", seed=1300)
    p = q.problem_from_instance(inst)
    c = _dev(wl.dirichlet_weights(2, 3, 1301))
    s = q.make_schedule("bsb", steps=10, seed=1)
    with pytest.raises(q.QaiaError) as e:
        q.qaia_sample_batch([q.BatchItem(p, c, 4, "dense_staged", tile=8)], s)
    assert e.value.status == q.QAIA_INVALID_ARGUMENT
    with pytest.raises(q.QaiaError) as e:  # 100 replicas x 42 spins > 16 spins per lane
        q.qaia_sample_batch([q.BatchItem(p, c, 4, "sparse_lds", tile=100)], s)
    assert e.value.status == q.QAIA_UNSUPPORTED
