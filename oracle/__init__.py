"""CPU oracle for simulated-bifurcation sampling of multi-objective MaxCut.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links or
runs anything here, and nothing here imports the library.

Python wrappers over ``liboracle.so`` (``qaia_oracle.c``): float64 dynamics,
exact int64 cut values, the O(U^2 m) non-dominated filter and the exact
slicing hypervolume.  The small-MLP oracle lives in ``oracle.mlp``.
Spins are int8 arrays of +1/-1, one row per sample.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_init_value.restype = C.c_float
        L.orc_init_value.argtypes = [C.c_uint64, C.c_uint64, C.c_float]
        L.orc_noise_value.restype = C.c_double
        L.orc_noise_value.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_cut_values.restype = None
        L.orc_cut_values.argtypes = [C.c_int, C.c_int, C.c_int64, P, P, P, C.c_int64, P, P]
        L.orc_c0.restype = C.c_double
        L.orc_c0.argtypes = [C.c_int, C.c_int, C.c_int64, P, P, P, C.c_double, P]
        L.orc_sb_sample.restype = C.c_int
        L.orc_sb_sample.argtypes = [C.c_int, C.c_int, C.c_int64, P, P, P, C.c_int, P, C.c_int64,
                                    C.c_int32, C.c_int, C.c_int32, C.c_float, C.c_float, C.c_float,
                                    C.c_double, C.c_uint64, C.c_uint64, P, P, C.c_int32, C.c_int]
        L.orc_objective_fields.restype = None
        L.orc_objective_fields.argtypes = [C.c_int, C.c_int, C.c_int64, P, P, P, C.c_int64, P, P]
        L.orc_pareto_filter.restype = C.c_int64
        L.orc_pareto_filter.argtypes = [P, C.c_int64, C.c_int, P]
        L.orc_pareto_ranks.restype = C.c_int32
        L.orc_pareto_ranks.argtypes = [P, C.c_int64, C.c_int, P]
        L.orc_hypervolume.restype = C.c_int
        L.orc_hypervolume.argtypes = [P, C.c_int64, C.c_int, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def splitmix64(seed: int, idx: int) -> int:
    """The ``idx``-th draw of the counter-based SplitMix64 stream ``seed``."""
    return int(lib().orc_splitmix64(seed & (2**64 - 1), idx & (2**64 - 1)))


def init_value(seed: int, idx: int, amp: float) -> float:
    return float(lib().orc_init_value(seed, idx, amp))


def noise_value(seed: int, idx: int) -> float:
    return float(lib().orc_noise_value(seed, idx))


def cut_values(inst, spins: np.ndarray) -> np.ndarray:
    """Eq. (1) for every row of ``spins`` (int8 +1/-1, [count, n]) -> int64 [count, m]."""
    spins = _c(spins, np.int8)
    count = spins.shape[0]
    out = np.zeros((count, inst.m), np.int64)
    eu, ev, w = _c(inst.edge_u, np.int32), _c(inst.edge_v, np.int32), _c(inst.weights, np.int32)
    lib().orc_cut_values(inst.n, inst.m, inst.num_edges, _p(eu), _p(ev), _p(w), count, _p(spins), _p(out))
    return out


def c0(inst, c: np.ndarray) -> float:
    c = _c(c, np.float32)
    eu, ev, w = _c(inst.edge_u, np.int32), _c(inst.edge_v, np.int32), _c(inst.weights, np.int32)
    return float(lib().orc_c0(inst.n, inst.m, inst.num_edges, _p(eu), _p(ev), _p(w),
                              2.0 ** -inst.frac_bits, _p(c)))


def sb_sample(inst, weights: np.ndarray, R: int, T: int, variant: str = "bsb", dt: float = 0.5,
              a0: float = 1.0, amp: float = 0.1, alpha: float = 0.0, seed: int = 0,
              replica_offset: int = 0, trace_steps: int = 0, nthreads: int = 0):
    """Run SB for every (weight vector, replica); rows are ``w * R + r``.

    Returns ``spins`` (int8 [W*R, n]) and, when ``trace_steps`` > 0, the
    float64 x trace [W*R, trace_steps, n].
    """
    weights = _c(weights, np.float32)
    nw = weights.shape[0]
    spins = np.zeros((nw * R, inst.n), np.int8)
    trace = np.zeros((nw * R, trace_steps, inst.n), np.float64) if trace_steps > 0 else None
    eu, ev, w = _c(inst.edge_u, np.int32), _c(inst.edge_v, np.int32), _c(inst.weights, np.int32)
    var = {"bsb": 0, "dsb": 1}[variant]
    rc = lib().orc_sb_sample(inst.n, inst.m, inst.num_edges, _p(eu), _p(ev), _p(w), inst.frac_bits,
                             _p(weights), nw, R, var, T, dt, a0, amp, alpha, seed & (2**64 - 1),
                             replica_offset, _p(spins), _p(trace) if trace is not None else None,
                             trace_steps, nthreads)
    if rc != 0:
        raise ValueError(f"orc_sb_sample failed with status {rc}")
    return (spins, trace) if trace is not None else spins


def objective_fields(inst, phi: np.ndarray) -> np.ndarray:
    """Per-objective force sum_j J^(k)_ij phi_j in weight units: float64 [count, m, n]."""
    phi = _c(phi, np.float64)
    count = phi.shape[0]
    out = np.zeros((count, inst.m, inst.n), np.float64)
    eu, ev, w = _c(inst.edge_u, np.int32), _c(inst.edge_v, np.int32), _c(inst.weights, np.int32)
    lib().orc_objective_fields(inst.n, inst.m, inst.num_edges, _p(eu), _p(ev), _p(w), count,
                               _p(phi), _p(out))
    return out


def pareto_filter(obj: np.ndarray) -> np.ndarray:
    """Ascending sample indices representing the non-dominated unique vectors."""
    obj = _c(obj, np.int64)
    M, m = obj.shape
    keep = np.zeros(max(M, 1), np.int64)
    P = lib().orc_pareto_filter(_p(obj), M, m, _p(keep))
    return keep[:P].copy()


def pareto_ranks(obj: np.ndarray) -> np.ndarray:
    """Non-dominated rank of every row (0 = non-dominated), int32 [M]."""
    obj = _c(obj, np.int64)
    M, m = obj.shape
    rank = np.zeros(max(M, 1), np.int32)
    lib().orc_pareto_ranks(_p(obj), M, m, _p(rank))
    return rank[:M].copy()


class HypervolumeOverflow(ArithmeticError):
    pass


def hypervolume(points: np.ndarray, ref) -> int:
    """Exact hypervolume (Python int) of the union of boxes [ref, y]."""
    points = _c(points, np.int64)
    if points.ndim == 1:
        points = points.reshape(1, -1) if points.size else points.reshape(0, len(ref))
    P, m = points.shape
    ref = _c(ref, np.int64)
    out = np.zeros(4, np.uint64)
    rc = lib().orc_hypervolume(_p(points), P, m, _p(ref), _p(out))
    if rc == 5:
        raise HypervolumeOverflow("hypervolume range exceeds 2^256")
    if rc != 0:
        raise ValueError(f"orc_hypervolume failed with status {rc}")
    return sum(int(out[i]) << (64 * i) for i in range(4))
