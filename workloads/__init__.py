"""Seeded synthetic inputs for multi-objective MaxCut.

This module is shared by the CPU oracle, the GPU library's tests and the
benchmark.  It only *draws inputs*: graphs, fixed-point edge weights and
scalarisation weight vectors.  It holds none of the sampler's arithmetic (no
dynamics, no cut evaluation, no filtering, no hypervolume), so the oracle and
the HIP path share no method code through it.

The paper's own instances (the IBM 42-node heavy-hex graphs and the Appendix E
instances with unpublished seeds) are not available; the generators below
reproduce their *shapes*: 42 nodes with degree <= 3, K in {3, 4} objectives,
dense complete graphs, Bernoulli density masks, and the Appendix E correlated
weight construction (Eq. 11).

Conventions
-----------
* Edges are pairs ``u < v`` sorted lexicographically; the edge index is the
  position in that order (the paper's edge set E holds i < j pairs,
  section "Hamiltonian formulation of multi-objective MaxCut").
* Edge weights are int32 fixed point: ``W = rint(g * 2**frac_bits)``,
  round-half-even, with ``g`` drawn in float64.
* Weight vectors are float32 rows on the simplex (``c_k >= 0``, sum 1),
  section "Scalarization via the weighted sum method".
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

FRAC_BITS = 16


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Instance:
    """A multi-objective MaxCut instance in edge-list form."""

    n: int
    m: int
    edge_u: np.ndarray  # int32 [E], u < v
    edge_v: np.ndarray  # int32 [E]
    weights: np.ndarray  # int32 [m, E], fixed point with FRAC_BITS fraction bits
    frac_bits: int = FRAC_BITS
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.edge_u.shape[0])


def _sorted_edges(pairs) -> tuple[np.ndarray, np.ndarray]:
    pairs = sorted((min(a, b), max(a, b)) for a, b in pairs)
    if not pairs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    arr = np.asarray(pairs, dtype=np.int32)
    return np.ascontiguousarray(arr[:, 0]), np.ascontiguousarray(arr[:, 1])


def degree_bounded_graph(n: int, num_edges: int, max_degree: int, seed: int):
    """Random graph with exactly ``num_edges`` edges and every degree <= ``max_degree``.

    Seeded random pairing of nodes with free degree: draw ``u`` uniformly among
    nodes whose degree is below the bound, then ``v`` uniformly among the other
    such nodes not yet joined to ``u``; restart from scratch on a dead end.
    Connectivity is not enforced.
    """
    if num_edges > n * max_degree // 2:
        raise ValueError("too many edges for the degree bound")
    rng = _rng(seed)
    while True:
        deg = np.zeros(n, np.int64)
        edges: set[tuple[int, int]] = set()
        dead = False
        while len(edges) < num_edges:
            free = np.flatnonzero(deg < max_degree)
            if free.size < 2:
                dead = True
                break
            u = int(free[rng.integers(free.size)])
            cand = [int(v) for v in free if v != u and (min(u, v), max(u, v)) not in edges]
            if not cand:
                dead = True
                break
            v = cand[int(rng.integers(len(cand)))]
            edges.add((min(u, v), max(u, v)))
            deg[u] += 1
            deg[v] += 1
        if not dead:
            return _sorted_edges(edges)


def complete_graph(n: int):
    """All pairs i < j in lexicographic order."""
    iu = np.triu_indices(n, k=1)
    return iu[0].astype(np.int32), iu[1].astype(np.int32)


def bernoulli_graph(n: int, density: float, seed: int):
    """Each pair i < j is an edge independently with probability ``density``."""
    rng = _rng(seed)
    iu, iv = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < density
    return iu[keep].astype(np.int32), iv[keep].astype(np.int32)


def fixed_point(g: np.ndarray, frac_bits: int = FRAC_BITS) -> np.ndarray:
    """``rint(g * 2**frac_bits)`` with round-half-even, as int32."""
    w = np.rint(np.asarray(g, np.float64) * float(2 ** frac_bits))
    if np.any(np.abs(w) > 2**31 - 1):
        raise ValueError("weight out of int32 range")
    return w.astype(np.int32)


def gaussian_weights(m: int, num_edges: int, seed: int, frac_bits: int = FRAC_BITS) -> np.ndarray:
    """i.i.d. N(0,1) per objective and edge, in int32 fixed point, shape [m, E]."""
    rng = _rng(seed)
    return fixed_point(rng.standard_normal((m, num_edges)), frac_bits)


def dirichlet_weights(count: int, m: int, seed: int) -> np.ndarray:
    """``count`` Dirichlet(1,...,1) weight vectors (uniform on the simplex), float32 [count, m]."""
    rng = _rng(seed)
    return np.ascontiguousarray(rng.dirichlet(np.ones(m), size=count).astype(np.float32))


def das_dennis_interior(m: int, h: int) -> np.ndarray:
    """Interior points of the Das-Dennis simplex lattice of resolution ``h``.

    All vectors with components in {1/h, ..., (h-1)/h} summing to one; the
    paper drops lattice points on the simplex vertices and edges (section
    "Scalarization via the weighted sum method", Appendix B).  There are
    C(h-1, m-1) of them: 190 for (m=3, h=21) and 220 for (m=4, h=13).
    """
    rows = []
    for comp in itertools.product(range(1, h), repeat=m - 1):
        last = h - sum(comp)
        if last >= 1:
            rows.append(list(comp) + [last])
    arr = np.asarray(rows, dtype=np.float64) / h
    return np.ascontiguousarray(arr.astype(np.float32))


def random_instance(n: int, m: int, kind: str, seed: int, num_edges: int | None = None,
                    frac_bits: int = FRAC_BITS) -> Instance:
    """Instance with Gaussian fixed-point weights.

    ``kind`` is ``"deg3"`` (degree <= 3, ``num_edges`` edges, default
    round(8n/7) -- 48 edges at n = 42), ``"complete"``, or a density such as
    ``"p0.1"`` / ``"p0.5"`` (Bernoulli mask).  The weight seed is ``seed + 1``.
    """
    if kind == "deg3":
        e = num_edges if num_edges is not None else int(round(8 * n / 7))
        u, v = degree_bounded_graph(n, e, 3, seed)
    elif kind == "complete":
        u, v = complete_graph(n)
    elif kind.startswith("p"):
        u, v = bernoulli_graph(n, float(kind[1:]), seed)
    else:
        raise ValueError(kind)
    w = gaussian_weights(m, u.shape[0], seed + 1, frac_bits)
    return Instance(n, m, u, v, w, frac_bits, name=f"{kind}-n{n}-m{m}-s{seed}")


def appendix_e_instance(n: int, density: float, seed: int, frac_bits: int = FRAC_BITS) -> Instance:
    """Correlated three-objective instance shaped like Appendix E (Eq. 11).

    A and B have integer entries uniform on [-25, 25]; J1 = A + B and
    J2 = 0.2 A - 5 B (so C1 and C2 are negatively correlated), J3 is drawn
    independently like A; a Bernoulli(density) mask picks the edges.  Only the
    upper triangle i < j is used.
    """
    rng = _rng(seed)
    iu, iv = np.triu_indices(n, k=1)
    npair = iu.shape[0]
    a = rng.integers(-25, 26, size=npair).astype(np.float64)
    b = rng.integers(-25, 26, size=npair).astype(np.float64)
    c = rng.integers(-25, 26, size=npair).astype(np.float64)
    keep = rng.random(npair) < density if density < 1.0 else np.ones(npair, bool)
    j = np.stack([a + b, 0.2 * a - 5.0 * b, c])[:, keep]
    return Instance(n, 3, iu[keep].astype(np.int32), iv[keep].astype(np.int32),
                    fixed_point(j, frac_bits), frac_bits, name=f"appE-n{n}-d{density}-s{seed}")


# --- the benchmark workloads (sizes from the paper-shaped configurations) ---

def instance_42_node(m: int, seed: int) -> Instance:
    """42 nodes, max degree 3, 48 edges, N(0,1) weights at scale 2^16."""
    return random_instance(42, m, "deg3", seed, num_edges=48)


WORKLOADS = {
    # name: (instance factory, weight-vector count, replicas, steps)
    "c1_bsb_n42_m3": dict(n=42, m=3, kind="deg3", edges=48, W=200, R=16, T=1000, seed=1000),
    "c2_n42_m4": dict(n=42, m=4, kind="deg3", edges=48, W=20000, R=256, T=2000, seed=2000),
    "c3_dsb_complete2048_m3": dict(n=2048, m=3, kind="complete", W=512, R=8, T=1000, seed=3000),
}


def workload_instance(name: str) -> Instance:
    cfg = WORKLOADS[name]
    return random_instance(cfg["n"], cfg["m"], cfg["kind"], cfg["seed"], num_edges=cfg.get("edges"))


def workload_weights(name: str, count: int | None = None) -> np.ndarray:
    cfg = WORKLOADS[name]
    return dirichlet_weights(cfg["W"] if count is None else count, cfg["m"], cfg["seed"] + 2)


def ragged_batch(count: int = 64, seed: int = 4000):
    """The batching workload: ``count`` instances with N uniform on [42, 1024],
    m uniform on {3, 4} and the edge class uniform on {degree-3 sparse, 10 %,
    50 % density}; instance i uses seed ``seed + 10 i`` (graph), ``+1``
    (weights), ``+2`` (its 1024 Dirichlet weight vectors)."""
    rng = _rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.integers(42, 1025))
        m = int(rng.integers(3, 5))
        kind = ("deg3", "p0.1", "p0.5")[int(rng.integers(0, 3))]
        specs.append((n, m, kind, seed + 10 * i))
    return specs
