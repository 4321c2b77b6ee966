"""Python binding of libqaia (simulated-bifurcation sampling of multi-objective
MaxCut on AMD Instinct MI355X).

Thin ctypes layer over the C ABI declared in ``include/qaia.h``: the functions
carry the ABI's names and only marshal arguments.  PyTorch provides device
memory (tensors) and streams; every step of the computation runs in the
library's HIP kernels (or, for the exact hypervolume, its host C++).  Importing
this module fails loudly when ``libqaia.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np
import torch  # loaded first so that libqaia binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqaia.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2604_26477_amd/build.py` "
                      "(or __graft_entry__.build())")

_lib = C.CDLL(LIB_PATH)

QAIA_OK, QAIA_INVALID_ARGUMENT, QAIA_UNSUPPORTED, QAIA_OUT_OF_MEMORY = 0, 1, 2, 3
QAIA_DEVICE_ERROR, QAIA_OVERFLOW, QAIA_WORKSPACE_TOO_SMALL = 4, 5, 6
VARIANTS = {"bsb": 0, "dsb": 1}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2, "fp16": 3}
PATHS = {"auto": 0, "sparse_reg": 1, "sparse_lds": 2, "dense": 3, "dense_staged": 4}


class qaia_schedule(C.Structure):
    _fields_ = [("variant", C.c_int32), ("precision", C.c_int32), ("steps", C.c_int32),
                ("path", C.c_int32), ("dt", C.c_float), ("a0", C.c_float),
                ("init_amp", C.c_float), ("noise_alpha", C.c_float),
                ("seed", C.c_uint64), ("replica_offset", C.c_uint64)]


class qaia_batch_item(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("weights", C.c_void_p), ("W", C.c_int64), ("R", C.c_int32),
                ("path", C.c_int32), ("spins", C.c_void_p), ("obj", C.c_void_p), ("tile", C.c_int32),
                ("reserved", C.c_int32)]


_P, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_SIGS = {
    "qaia_abi_version": (_i32, []),
    "qaia_status_string": (C.c_char_p, [_i32]),
    "qaia_last_error": (C.c_char_p, []),
    "qaia_problem_create": (_i32, [_i32, _i32, _i64, _P, _P, _P, _i32, _i32, C.POINTER(_P)]),
    "qaia_problem_destroy": (_i32, [_P]),
    "qaia_problem_info": (_i32, [_P, _P, _P, _P, _P]),
    "qaia_sample_workspace_bytes": (_i32, [_P, _i64, _i32, C.POINTER(qaia_schedule), C.POINTER(_sz)]),
    "qaia_sample": (_i32, [_P, _P, _i64, _i32, C.POINTER(qaia_schedule), _P, _P, _P, _sz, _P]),
    "qaia_sample_trace": (_i32, [_P, _P, _i64, _i32, C.POINTER(qaia_schedule), _P, _P, _P, _sz, _P,
                                 _i32, _P]),
    "qaia_sample_noalloc": (_i32, [_P, _P, _i64, _i32, C.POINTER(qaia_schedule), _P, _P, _P, _P]),
    "qaia_workspace_status": (_i32, [_P, C.POINTER(_i64)]),
    "qaia_evaluate": (_i32, [_P, _P, _i64, _P, _P]),
    "qaia_enumerate_cuts": (_i32, [_P, C.c_uint64, _i64, _P, _P]),
    "qaia_random_spins": (_i32, [_i32, _i64, C.c_uint64, C.c_uint64, _P, _P]),
    "qaia_dirichlet_weights": (_i32, [_i32, _i64, C.c_uint64, C.c_uint64, _P, _P]),
    "qaia_pareto_filter_workspace_bytes": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "qaia_pareto_filter": (_i32, [_P, _i64, _i32, _P, _P, _P, _sz, _P]),
    "qaia_hypervolume": (_i32, [_P, _i64, _i32, _P, _P, _P]),
    "qaia_objective_min": (_i32, [_P, _i64, _i32, _P, _i32, _P]),
    "qaia_pareto_ranks_workspace_bytes": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "qaia_pareto_ranks": (_i32, [_P, _i64, _i32, _i32, _P, C.POINTER(_i32), _P, _sz, _P]),
    "qaia_dense_field_workspace_bytes": (_i32, [_P, _i32, _i64, C.POINTER(_sz)]),
    "qaia_dense_field": (_i32, [_P, _i32, _P, _i64, _P, _P, _sz, _P]),
    "qaia_mlp_param_count": (_i32, [_i32, C.POINTER(_i64)]),
    "qaia_mlp_forward_workspace_bytes": (_i32, [_i64, C.POINTER(_sz)]),
    "qaia_mlp_forward": (_i32, [_P, _i32, _P, _i64, _P, _P, _sz, _P]),
    "qaia_mlp_backward_workspace_bytes": (_i32, [_i32, _i64, C.POINTER(_sz)]),
    "qaia_mlp_backward": (_i32, [_P, _i32, _P, _P, _i64, _P, _P, _P, _sz, _P]),
    "qaia_mlp_adam": (_i32, [_P, _P, _P, _P, _P, _i64, _i32, C.c_float, C.c_float, C.c_float,
                             C.c_float, _P]),
    "qaia_mlp_train_workspace_bytes": (_i32, [_i32, _i64, _i32, C.POINTER(_sz)]),
    "qaia_mlp_train": (_i32, [_P, _P, _P, _P, _i32, _P, _P, _i64, _i32, _i32, _i32, C.c_float, C.c_uint64, _P, _sz,
                              _P]),
    "qaia_front_features_workspace_bytes": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "qaia_front_features": (_i32, [_P, _i64, _i32, _P, _i64, _P, _i64, _P, _i64, _P, _P, _sz, _P]),
    "qaia_topk_workspace_bytes": (_i32, [_i64, C.POINTER(_sz)]),
    "qaia_topk": (_i32, [_P, _i64, _i64, C.c_float, C.c_uint64, _P, _P, _sz, _P]),
    "qaia_new_point_labels": (_i32, [_P, _P, _i64, _i32, _i64, _P, _P]),
    "qaia_gather_rows": (_i32, [_P, _i32, _P, _P, _i64, _P, _P]),
    "qaia_sample_batch_workspace_bytes": (_i32, [_P, _i32, C.POINTER(qaia_schedule), C.POINTER(_sz)]),
    "qaia_sample_batch": (_i32, [_P, _i32, C.POINTER(qaia_schedule), _P, _sz, _P]),
    "qaia_plan_autotune_workspace_bytes": (_i32, [_P, _i32, C.POINTER(qaia_schedule), _i32, C.POINTER(_sz)]),
    "qaia_plan_autotune": (_i32, [_P, _i32, C.POINTER(qaia_schedule), _i32, _P, _P, _sz, _P]),
    "qaia_peak_fma": (_i32, [_i64, _i32, C.c_float, C.c_float, _P, _P]),
    "qaia_peak_mfma": (_i32, [_i32, _i64, _i32, _P, _P]),
    "qaia_peak_copy": (_i32, [_P, _P, _sz, _P]),
    "qaia_peak_valu": (_i32, [_i64, _i32, C.c_float, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class QaiaError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{qaia_status_string(status)} ({status}): {detail}")


def _check(rc: int):
    if rc != QAIA_OK:
        raise QaiaError(rc, qaia_last_error())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    raise TypeError(type(t))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_tensor(t, dtype, shape, device):
    if t is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < int(np.prod(shape)):
        raise ValueError(f"expected a contiguous {dtype} tensor with at least {int(np.prod(shape))} elements")
    return t


# ------------------------------------------------------------------ basics

def qaia_abi_version() -> int:
    return int(_lib.qaia_abi_version())


def qaia_status_string(status: int) -> str:
    return _lib.qaia_status_string(status).decode()


def qaia_last_error() -> str:
    return _lib.qaia_last_error().decode()


# ------------------------------------------------------------------ problem

class Problem:
    """Owning handle of a ``qaia_problem``."""

    def __init__(self, handle, n, m, num_edges, device):
        self.handle, self.n, self.m, self.num_edges, self.device = handle, n, m, num_edges, device
        self.words = (n + 63) // 64

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps sys.is_finalizing reachable while modules
        # are torn down at interpreter exit, when the process frees everything
        h = getattr(self, "handle", None)
        if h and not _finalizing():
            _lib.qaia_problem_destroy(h)
            self.handle = None

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)


def qaia_problem_create(n, m, edge_u, edge_v, weights, frac_bits=16, device=0) -> Problem:
    eu = np.ascontiguousarray(edge_u, np.int32)
    ev = np.ascontiguousarray(edge_v, np.int32)
    w = np.ascontiguousarray(weights, np.int32).ravel()
    if eu.shape != ev.shape or w.size < max(m, 0) * eu.shape[0]:
        raise ValueError("edge_u/edge_v lengths differ or weights hold fewer than m * num_edges values")
    h = C.c_void_p()
    _check(_lib.qaia_problem_create(n, m, eu.shape[0], _ptr(eu), _ptr(ev), _ptr(w), frac_bits,
                                    device, C.byref(h)))
    return Problem(h, n, m, eu.shape[0], device)


def problem_from_instance(inst, device=0) -> Problem:
    return qaia_problem_create(inst.n, inst.m, inst.edge_u, inst.edge_v, inst.weights,
                               inst.frac_bits, device)


def qaia_problem_destroy(p: Problem):
    if p.handle:
        _check(_lib.qaia_problem_destroy(p.handle))
        p.handle = None


def qaia_problem_info(p: Problem):
    n, m, e = C.c_int32(), C.c_int32(), C.c_int64()
    tot = np.zeros(p.m, np.int64)
    _check(_lib.qaia_problem_info(p.handle, C.byref(n), C.byref(m), C.byref(e), _ptr(tot)))
    return {"n": n.value, "m": m.value, "num_edges": e.value, "total_weight": tot}


# ------------------------------------------------------------------ sampling

def make_schedule(variant="bsb", precision="fp32", steps=1000, dt=0.5, a0=1.0, init_amp=0.1,
                  noise_alpha=0.0, seed=0, replica_offset=0, path="auto") -> qaia_schedule:
    return qaia_schedule(VARIANTS[variant], PRECISIONS[precision], steps, PATHS[path], dt, a0,
                         init_amp, noise_alpha, seed & (2**64 - 1), replica_offset)


def qaia_sample_workspace_bytes(p: Problem, W: int, R: int, s: qaia_schedule) -> int:
    b = C.c_size_t()
    _check(_lib.qaia_sample_workspace_bytes(p.handle, W, R, C.byref(s), C.byref(b)))
    return b.value


def qaia_sample(p: Problem, weights: torch.Tensor, R: int, s: qaia_schedule, spins=None, obj=None,
                workspace=None, stream=None):
    """Returns (spins uint64-as-int64 [W*R, words], obj int64 [W*R, m], workspace)."""
    return _sample(p, weights, R, s, spins, obj, workspace, stream, None, 0)


def qaia_sample_trace(p: Problem, weights: torch.Tensor, R: int, s: qaia_schedule, trace_steps: int,
                      spins=None, obj=None, workspace=None, trace=None, stream=None):
    """As qaia_sample, plus x after each of the first trace_steps steps [W*R, trace_steps, n]."""
    W = weights.shape[0]
    trace = _dev_tensor(trace, torch.float32, (W * R, trace_steps, p.n), p.torch_device)
    out = _sample(p, weights, R, s, spins, obj, workspace, stream, trace, trace_steps)
    return (*out, trace)


def _sample(p, weights, R, s, spins, obj, workspace, stream, trace, trace_steps):
    if weights.dtype != torch.float32 or not weights.is_cuda or not weights.is_contiguous():
        raise ValueError("weights must be a contiguous float32 CUDA tensor [W, m]")
    W = weights.shape[0]
    dev = p.torch_device
    spins = _dev_tensor(spins, torch.int64, (W * R, p.words), dev)
    obj = _dev_tensor(obj, torch.int64, (W * R, p.m), dev)
    need = qaia_sample_workspace_bytes(p, W, R, s)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if trace is None:
        rc = _lib.qaia_sample(p.handle, _ptr(weights), W, R, C.byref(s), _ptr(spins), _ptr(obj),
                              _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream(stream))
    else:
        rc = _lib.qaia_sample_trace(p.handle, _ptr(weights), W, R, C.byref(s), _ptr(spins),
                                    _ptr(obj), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), _ptr(trace),
                                    trace_steps, _stream(stream))
    _check(rc)
    return spins, obj, workspace


NOALLOC_SCRATCH_BYTES = 16 << 20  # QAIA_NOALLOC_SCRATCH_BYTES


def qaia_sample_noalloc(p: Problem, weights: torch.Tensor, R: int, s: qaia_schedule, spins: torch.Tensor,
                        obj: torch.Tensor, bad_row: torch.Tensor | None = None, stream=None):
    """qaia_sample with the library's static scratch as workspace: allocates
    nothing, so spins [W*R, words] int64, obj [W*R, m] int64 and the optional
    bad_row (int64 [1]) are caller-provided device tensors."""
    if weights.dtype != torch.float32 or not weights.is_cuda or not weights.is_contiguous():
        raise ValueError("weights must be a contiguous float32 CUDA tensor [W, m]")
    if spins is None or obj is None:
        raise ValueError("qaia_sample_noalloc takes caller-provided spins and obj tensors")
    W = weights.shape[0]
    dev = p.torch_device
    spins = _dev_tensor(spins, torch.int64, (W * R, p.words), dev)
    obj = _dev_tensor(obj, torch.int64, (W * R, p.m), dev)
    if bad_row is not None:
        bad_row = _dev_tensor(bad_row, torch.int64, (1,), dev)
    _check(_lib.qaia_sample_noalloc(p.handle, _ptr(weights), W, R, C.byref(s), _ptr(spins), _ptr(obj),
                                    _ptr(bad_row), _stream(stream)))
    return spins, obj


def qaia_workspace_status(workspace: torch.Tensor):
    """None if every weight row was valid, else the smallest invalid row."""
    bad = C.c_int64(-1)
    rc = _lib.qaia_workspace_status(_ptr(workspace), C.byref(bad))
    if rc == QAIA_INVALID_ARGUMENT and bad.value >= 0:
        return bad.value
    _check(rc)
    return None


def qaia_evaluate(p: Problem, spins: torch.Tensor, obj=None, stream=None) -> torch.Tensor:
    count = spins.shape[0]
    obj = _dev_tensor(obj, torch.int64, (count, p.m), p.torch_device)
    _check(_lib.qaia_evaluate(p.handle, _ptr(spins), count, _ptr(obj), _stream(stream)))
    return obj


def qaia_enumerate_cuts(p: Problem, first: int, count: int, obj=None, stream=None) -> torch.Tensor:
    """Cut values of the configurations with spin words first .. first + count - 1."""
    obj = _dev_tensor(obj, torch.int64, (count, p.m), p.torch_device)
    _check(_lib.qaia_enumerate_cuts(p.handle, first, count, _ptr(obj), _stream(stream)))
    return obj


def qaia_random_spins(n: int, count: int, seed: int, offset: int = 0, spins=None, device=None,
                      stream=None) -> torch.Tensor:
    """count uniformly random spin configurations, packed like qaia_sample's spins."""
    words = (n + 63) // 64
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    spins = _dev_tensor(spins, torch.int64, (count, words), dev)
    _check(_lib.qaia_random_spins(n, count, seed & (2**64 - 1), offset & (2**64 - 1), _ptr(spins),
                                  _stream(stream)))
    return spins


def qaia_dirichlet_weights(m: int, count: int, seed: int, offset: int = 0, out=None, device=None,
                           stream=None) -> torch.Tensor:
    """count weight vectors uniform on the simplex (float32 [count, m] device)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = _dev_tensor(out, torch.float32, (count, m), dev)
    _check(_lib.qaia_dirichlet_weights(m, count, seed & (2**64 - 1), offset & (2**64 - 1), _ptr(out),
                                       _stream(stream)))
    return out


def exact_front(p: Problem, chunk: int = 1 << 26, with_min: bool = False):
    """Pareto front by exhaustive enumeration of the 2^(n-1) cuts (n <= 36 here).

    Enumerates in chunks, filters each chunk together with the running front,
    and returns (codes int64 [P] host, obj int64 [P, m] host): the spin words
    of one representative per non-dominated objective vector (the smallest
    code) and their cut values, in ascending code order.  with_min also
    returns the per-objective minimum cut value over all configurations
    (qaia_objective_min folded over the chunks)."""
    if p.n > 36:
        raise ValueError("exhaustive enumeration is limited to n <= 36")
    total = 1 << (p.n - 1)
    dev = p.torch_device
    front_codes = torch.zeros(0, dtype=torch.int64, device=dev)
    front_obj = torch.zeros((0, p.m), dtype=torch.int64, device=dev)
    lo = torch.empty(p.m, dtype=torch.int64, device=dev)
    first = 0
    while first < total:
        cnt = min(chunk, total - first)
        F = front_obj.shape[0]
        pool = torch.empty((F + cnt, p.m), dtype=torch.int64, device=dev)
        codes = torch.empty(F + cnt, dtype=torch.int64, device=dev)
        pool[:F] = front_obj
        codes[:F] = front_codes
        codes[F:] = torch.arange(first, first + cnt, dtype=torch.int64, device=dev)  # the row's spin word
        qaia_enumerate_cuts(p, first, cnt, obj=pool[F:])
        if with_min:
            qaia_objective_min(pool[F:], out=lo, accumulate=first > 0)
        keep, nkeep, _ = qaia_pareto_filter(pool)
        P = int(nkeep.item())
        front_obj = torch.empty((P, p.m), dtype=torch.int64, device=dev)
        front_codes = torch.empty(P, dtype=torch.int64, device=dev)
        qaia_gather_rows(pool, keep, nkeep, front_obj, P)
        qaia_gather_rows(codes.view(-1, 1), keep, nkeep, front_codes.view(-1, 1), P)
        first += cnt
    out = (front_codes.cpu().numpy(), front_obj.cpu().numpy())
    return out + (lo.cpu().numpy(),) if with_min else out


def qaia_objective_min(obj: torch.Tensor, out=None, accumulate: bool = False, stream=None) -> torch.Tensor:
    """Per-objective minimum of the rows of obj (int64 [M, m] device); with
    accumulate, folded into the values already in out."""
    M, m = obj.shape
    out = _dev_tensor(out, torch.int64, (m,), obj.device)
    _check(_lib.qaia_objective_min(_ptr(obj) if M else None, M, m, _ptr(out), 1 if accumulate else 0,
                                   _stream(stream)))
    return out


# ------------------------------------------------------------------ filtering

def qaia_pareto_filter_workspace_bytes(M: int, m: int) -> int:
    b = C.c_size_t()
    _check(_lib.qaia_pareto_filter_workspace_bytes(M, m, C.byref(b)))
    return b.value


def qaia_pareto_filter(obj: torch.Tensor, keep_idx=None, num_keep=None, workspace=None,
                       stream=None):
    """Returns (keep_idx int64 [M] device, num_keep int64 [1] device, workspace)."""
    if obj.dtype != torch.int64 or not obj.is_contiguous() or obj.dim() != 2:
        raise ValueError("obj must be a contiguous int64 tensor [M, m]")
    M, m = obj.shape
    dev = obj.device
    keep_idx = _dev_tensor(keep_idx, torch.int64, (max(M, 1),), dev)
    num_keep = _dev_tensor(num_keep, torch.int64, (1,), dev)
    need = qaia_pareto_filter_workspace_bytes(M, m)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(_lib.qaia_pareto_filter(_ptr(obj), M, m, _ptr(keep_idx), _ptr(num_keep),
                                   _ptr(workspace), workspace.numel(), _stream(stream)))
    return keep_idx, num_keep, workspace


def pareto_front(obj: torch.Tensor, stream=None) -> torch.Tensor:
    """Representative sample indices of the non-dominated set (synchronises)."""
    keep, num, _ = qaia_pareto_filter(obj, stream=stream)
    return keep[: int(num.item())]


def qaia_pareto_ranks(obj: torch.Tensor, max_rank: int = 2**31 - 1, rank=None, workspace=None, stream=None):
    """Non-dominated rank of every row (int32 [M] device) and the number of ranks peeled."""
    if obj.dtype != torch.int64 or not obj.is_contiguous() or obj.dim() != 2:
        raise ValueError("obj must be a contiguous int64 tensor [M, m]")
    M, m = obj.shape
    b = C.c_size_t()
    _check(_lib.qaia_pareto_ranks_workspace_bytes(M, m, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(b.value, 1), dtype=torch.uint8, device=obj.device)
    rank = _dev_tensor(rank, torch.int32, (max(M, 1),), obj.device)
    n = C.c_int32()
    _check(_lib.qaia_pareto_ranks(_ptr(obj), M, m, max_rank, _ptr(rank), C.byref(n), _ptr(workspace),
                                  workspace.numel(), _stream(stream)))
    return rank[:M], n.value


# ------------------------------------------------------------------ hypervolume

def qaia_hypervolume(points, ref) -> int:
    """Exact hypervolume (Python int) of the union of boxes [ref, y] (host call)."""
    pts = np.ascontiguousarray(points, np.int64)
    ref = np.ascontiguousarray(ref, np.int64)
    if pts.ndim == 1:
        pts = pts.reshape(-1, ref.shape[0])
    P, m = pts.shape if pts.size else (0, ref.shape[0])
    hv = np.zeros(4, np.uint64)
    approx = C.c_double()
    _check(_lib.qaia_hypervolume(_ptr(pts) if P else None, P, m, _ptr(ref), _ptr(hv), C.byref(approx)))
    return sum(int(hv[i]) << (64 * i) for i in range(4))


def unpack_spins(spins: np.ndarray, n: int) -> np.ndarray:
    """Packed rows (bit i set <=> s_i = -1) -> int8 +1/-1 rows [count, n]."""
    words = np.ascontiguousarray(spins).view(np.uint64)
    bits = ((words[:, :, None] >> np.arange(64, dtype=np.uint64)[None, None, :]) & np.uint64(1))
    bits = bits.reshape(words.shape[0], -1)[:, :n].astype(np.int8)
    return (1 - 2 * bits).astype(np.int8)


# ------------------------------------------------------------------ precision form

def qaia_dense_field(p: Problem, precision: str, phi: torch.Tensor, field=None, workspace=None, stream=None):
    """Per-objective products sum_j J^(k)_ij phi_j (float32 [count, m, n]) in the given arithmetic."""
    prec = PRECISIONS[precision]
    count = phi.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_dense_field_workspace_bytes(p.handle, prec, count, C.byref(b)))
    if workspace is None:
        workspace = torch.empty(max(b.value, 1), dtype=torch.uint8, device=p.torch_device)
    field = _dev_tensor(field, torch.float32, (count, p.m, p.n), p.torch_device)
    _check(_lib.qaia_dense_field(p.handle, prec, _ptr(phi), count, _ptr(field), _ptr(workspace),
                                 workspace.numel(), _stream(stream)))
    return field


# ------------------------------------------------------------------ learned form

def qaia_mlp_param_count(in_dim: int) -> int:
    n = C.c_int64()
    _check(_lib.qaia_mlp_param_count(in_dim, C.byref(n)))
    return n.value


def qaia_mlp_forward(params: torch.Tensor, in_dim: int, X: torch.Tensor, logits=None, workspace=None,
                     stream=None) -> torch.Tensor:
    N = X.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_mlp_forward_workspace_bytes(N, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(b.value, 1), dtype=torch.uint8, device=X.device)
    logits = _dev_tensor(logits, torch.float32, (N,), X.device)
    _check(_lib.qaia_mlp_forward(_ptr(params), in_dim, _ptr(X), N, _ptr(logits), _ptr(workspace),
                                 workspace.numel(), _stream(stream)))
    return logits


def qaia_mlp_backward(params: torch.Tensor, in_dim: int, X: torch.Tensor, labels: torch.Tensor,
                      grad=None, logits=None, workspace=None, stream=None):
    B = X.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_mlp_backward_workspace_bytes(in_dim, B, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=X.device)
    grad = _dev_tensor(grad, torch.float32, (qaia_mlp_param_count(in_dim),), X.device)
    _check(_lib.qaia_mlp_backward(_ptr(params), in_dim, _ptr(X), _ptr(labels), B, _ptr(grad),
                                  _ptr(logits), _ptr(workspace), workspace.numel(), _stream(stream)))
    return grad


def qaia_mlp_adam(master, params, moment1, moment2, grad, step, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, stream=None):
    _check(_lib.qaia_mlp_adam(_ptr(master), _ptr(params), _ptr(moment1), _ptr(moment2), _ptr(grad),
                              master.numel(), step, lr, beta1, beta2, eps, _stream(stream)))


def qaia_mlp_train(master, params, moment1, moment2, in_dim: int, X: torch.Tensor, labels: torch.Tensor,
                   batch: int, steps: int, first_step: int, lr: float = 1e-3, seed: int = 0, workspace=None,
                   stream=None):
    """One round's Adam steps on minibatches of (X [n, in_dim], labels [n]); see qaia.h."""
    n = X.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_mlp_train_workspace_bytes(in_dim, n, batch, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=X.device)
    _check(_lib.qaia_mlp_train(_ptr(master), _ptr(params), _ptr(moment1), _ptr(moment2), in_dim, _ptr(X),
                               _ptr(labels), n, batch, steps, first_step, lr, seed & (2**64 - 1), _ptr(workspace),
                               workspace.numel(), _stream(stream)))
    return workspace


def qaia_front_features(front: torch.Tensor, cands: torch.Tensor, hits: torch.Tensor, misses: torch.Tensor,
                        out=None, workspace=None, stream=None) -> torch.Tensor:
    """MLP input rows [N, m + 8] = (c, f1..f8) of candidates c against an int64 front [P, m]."""
    P, m = front.shape[0], cands.shape[1]
    N = cands.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_front_features_workspace_bytes(P, m, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=cands.device)
    out = _dev_tensor(out, torch.float32, (N, m + 8), cands.device)
    _check(_lib.qaia_front_features(_ptr(front) if P else None, P, m, _ptr(cands), N,
                                    _ptr(hits) if hits.shape[0] else None, hits.shape[0],
                                    _ptr(misses) if misses.shape[0] else None, misses.shape[0],
                                    _ptr(out), _ptr(workspace), workspace.numel(), _stream(stream)))
    return out


def qaia_topk(scores: torch.Tensor, k: int, temperature: float = 0.0, seed: int = 0, idx=None, workspace=None,
              stream=None) -> torch.Tensor:
    N = scores.shape[0]
    b = C.c_size_t()
    _check(_lib.qaia_topk_workspace_bytes(N, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=scores.device)
    idx = _dev_tensor(idx, torch.int64, (max(k, 1),), scores.device)
    _check(_lib.qaia_topk(_ptr(scores), N, k, temperature, seed & (2**64 - 1), _ptr(idx), _ptr(workspace),
                          workspace.numel(), _stream(stream)))
    return idx[:k]


def qaia_new_point_labels(keep_idx, num_keep, archive_rows: int, R: int, W: int, labels=None, stream=None):
    labels = _dev_tensor(labels, torch.float32, (max(W, 1),), keep_idx.device)
    _check(_lib.qaia_new_point_labels(_ptr(keep_idx), _ptr(num_keep), archive_rows, R, W, _ptr(labels),
                                      _stream(stream)))
    return labels[:W]


def qaia_gather_rows(src: torch.Tensor, idx: torch.Tensor, count: torch.Tensor, dst: torch.Tensor, cap: int,
                     stream=None):
    """dst[r] = src[idx[r]] for r < min(count, cap); rows of any 4-byte-multiple width."""
    row_bytes = src[0].numel() * src.element_size() if src.dim() > 1 else src.element_size()
    if row_bytes % 4:
        raise ValueError("row size must be a multiple of 4 bytes")
    _check(_lib.qaia_gather_rows(_ptr(src), row_bytes // 4, _ptr(idx), _ptr(count), cap, _ptr(dst),
                                 _stream(stream)))
    return dst


# ------------------------------------------------------------------ measurement kernels

def qaia_peak_fma(blocks: int, iters: int, a: float = 1.0, b: float = 1.0, out=None, device=None,
                  stream=None) -> torch.Tensor:
    """Eight fp32 FMA chains per lane (x <- x a + b); out[t] = sum of the final values."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = _dev_tensor(out, torch.float32, (blocks * 256,), dev)
    _check(_lib.qaia_peak_fma(blocks, iters, a, b, _ptr(out), _stream(stream)))
    return out


def qaia_peak_valu(blocks: int, iters: int, k: float = 0.0, out=None, device=None, stream=None) -> torch.Tensor:
    """Sparse-SB instruction-mix ceiling (60 FMAs + 42 wall operations per lane-iteration)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = _dev_tensor(out, torch.float32, (blocks * 256,), dev)
    _check(_lib.qaia_peak_valu(blocks, iters, k, _ptr(out), _stream(stream)))
    return out


def qaia_peak_mfma(precision, blocks: int, iters: int, out=None, device=None, stream=None) -> torch.Tensor:
    """Four independent 32x32 MFMAs per wave per iteration, operands 1.0; out[t] = 4 K iters."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = _dev_tensor(out, torch.float32, (blocks * 256,), dev)
    _check(_lib.qaia_peak_mfma(prec, blocks, iters, _ptr(out), _stream(stream)))
    return out


def qaia_peak_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> torch.Tensor:
    """dst = src for two equal-sized device buffers (16-byte multiple)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    _check(_lib.qaia_peak_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)))
    return dst


# ------------------------------------------------------------------ batching form

class BatchItem:
    """One item of a ragged batch: a problem, device weights [W, m], replicas R,
    an optional forced path, and its outputs (allocated when not given)."""

    def __init__(self, problem: Problem, weights: torch.Tensor, R: int, path: str = "auto", spins=None, obj=None,
                 tile: int = 0):
        W = weights.shape[0]
        self.problem, self.weights, self.R, self.path, self.tile = problem, weights, R, path, tile
        self.spins = _dev_tensor(spins, torch.int64, (W * R, problem.words), problem.torch_device)
        self.obj = _dev_tensor(obj, torch.int64, (W * R, problem.m), problem.torch_device)

    def c_struct(self):
        return qaia_batch_item(self.problem.handle.value if isinstance(self.problem.handle, C.c_void_p)
                               else self.problem.handle, self.weights.data_ptr(), self.weights.shape[0], self.R,
                               PATHS[self.path], self.spins.data_ptr(), self.obj.data_ptr(), self.tile, 0)


def _items_array(items):
    arr = (qaia_batch_item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it.c_struct()
    return arr


def qaia_sample_batch_workspace_bytes(items, s: qaia_schedule) -> int:
    arr = _items_array(items)
    b = C.c_size_t()
    _check(_lib.qaia_sample_batch_workspace_bytes(C.cast(arr, C.c_void_p), len(items), C.byref(s), C.byref(b)))
    return b.value


def qaia_sample_batch(items, s: qaia_schedule, workspace=None, stream=None):
    """Samples every BatchItem with one graph launch; outputs land in item.spins / item.obj."""
    arr = _items_array(items)
    need = qaia_sample_batch_workspace_bytes(items, s)
    if workspace is None or workspace.numel() < need:
        dev = items[0].problem.torch_device if items else torch.device("cuda", torch.cuda.current_device())
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(_lib.qaia_sample_batch(C.cast(arr, C.c_void_p), len(items), C.byref(s), _ptr(workspace),
                                  workspace.numel(), _stream(stream)))
    return workspace


def qaia_plan_autotune(items, s: qaia_schedule, probe_steps: int = 20, stream=None):
    """Times each kernel family and tile per item; sets item.path and
    item.tile to the fastest and returns the estimated seconds per item at
    s.steps."""
    arr = _items_array(items)
    b = C.c_size_t()
    _check(_lib.qaia_plan_autotune_workspace_bytes(C.cast(arr, C.c_void_p), len(items), C.byref(s), probe_steps,
                                                   C.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=items[0].problem.torch_device)
    est = np.zeros(len(items), np.float64)
    _check(_lib.qaia_plan_autotune(C.cast(arr, C.c_void_p), len(items), C.byref(s), probe_steps, _ptr(est),
                                   _ptr(ws), ws.numel(), _stream(stream)))
    inv = {v: k for k, v in PATHS.items()}
    for i, it in enumerate(items):
        it.path = inv[arr[i].path]
        it.tile = arr[i].tile
    return est
