"""Host-side checks of the C ABI: symbols, status codes, argument validation
and the library's exact hypervolume (pure host code) against the oracle's
independent algorithm.  No GPU needed."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def q():
    import paper_2604_26477_amd as q
    return q


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "qaia.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qaia_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(q):
    import ctypes
    import shutil
    import subprocess
    lib = ctypes.CDLL(q.LIB_PATH)
    names = _declared_symbols()
    assert "qaia_sample" in names and "qaia_hypervolume" in names
    for name in names:
        assert hasattr(lib, name), name
    # and conversely: the library exports no qaia_ entry point the header lacks
    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--defined-only", q.LIB_PATH], capture_output=True, text=True).stdout
        exported = {f for line in out.splitlines() for f in line.split()[2:3] if f.startswith("qaia_")}
        assert exported == set(names), sorted(exported ^ set(names))


def test_version_and_status_strings(q):
    assert q.qaia_abi_version() == 2
    assert q.qaia_status_string(0) == "ok"
    assert q.qaia_status_string(5) == "overflow"
    assert q.qaia_status_string(99) == "unknown status"


@pytest.mark.parametrize("eu,ev,msg", [
    ([0, 1], [1, 1], "violates"),      # u == v
    ([0, 2], [1, 1], "violates"),      # u > v
    ([0, 0], [1, 1], "repeated"),      # duplicate pair
    ([0, 0], [1, 9], "violates"),      # v >= n
])
def test_problem_create_rejects_bad_edges(q, eu, ev, msg):
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_problem_create(4, 2, eu, ev, np.zeros((2, 2), np.int32))
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT and msg in str(ei.value)


def test_problem_create_rejects_bad_sizes(q):
    for n, m in ((0, 2), (4, 0), (4, 9)):
        with pytest.raises(q.QaiaError) as ei:
            q.qaia_problem_create(n, m, [0], [1], np.zeros((max(m, 1), 1), np.int32))
        assert ei.value.status == q.QAIA_INVALID_ARGUMENT


def test_hypervolume_worked_example(q):
    assert q.qaia_hypervolume(np.array([[10, 5], [5, 10]]), [0, 0]) == 75
    assert q.qaia_hypervolume(np.array([[10, 5], [5, 10], [8, 8]]), [0, 0]) == 84


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_hypervolume_matches_oracle(q, m):
    rng = np.random.default_rng(100 + m)
    for trial in range(25):
        P = int(rng.integers(0, 60 if m < 5 else 25))
        pts = rng.integers(-1000, 5000, size=(P, m))
        ref = rng.integers(-500, 100, size=m)
        assert q.qaia_hypervolume(pts, ref) == oracle.hypervolume(pts, ref)


def test_hypervolume_ties_and_duplicates(q):
    rng = np.random.default_rng(7)
    for m in (2, 3, 4):
        for trial in range(30):
            pts = rng.integers(0, 5, size=(int(rng.integers(1, 40)), m))  # many equal coordinates
            assert q.qaia_hypervolume(pts, np.zeros(m)) == oracle.hypervolume(pts, np.zeros(m))


def test_hypervolume_on_sampled_front(q):
    """A front of SB samples (oracle sampler) on a 4-objective instance."""
    inst = wl.random_instance(16, 4, "deg3", seed=31, num_edges=20)
    c = wl.dirichlet_weights(200, 4, 32)
    spins = oracle.sb_sample(inst, c, R=4, T=200, seed=33)
    obj = oracle.cut_values(inst, spins)
    front = obj[oracle.pareto_filter(obj)]
    ref = obj.min(axis=0)
    assert len(front) > 5
    assert q.qaia_hypervolume(front, ref) == oracle.hypervolume(front, ref)
    assert q.qaia_hypervolume(obj, ref) == oracle.hypervolume(front, ref)  # dominated points add nothing


def test_hypervolume_wide_range_and_overflow(q):
    big = 2**62
    pts = np.array([[big, big - 3, big - 5, big - 7], [big - 11, big, big, big - 1]], np.int64)
    ref = np.zeros(4, np.int64)
    assert q.qaia_hypervolume(pts, ref) == oracle.hypervolume(pts, ref)
    # five objectives of 62 bits each need 310 bits: OVERFLOW
    pts5 = np.full((1, 5), big, np.int64)
    with pytest.raises(q.QaiaError) as ei:
        q.qaia_hypervolume(pts5, np.zeros(5, np.int64))
    assert ei.value.status == q.QAIA_OVERFLOW


def test_hypervolume_empty_and_clipped(q):
    assert q.qaia_hypervolume(np.zeros((0, 3), np.int64), [0, 0, 0]) == 0
    # a point below the reference in one objective contributes nothing
    assert q.qaia_hypervolume(np.array([[5, -1, 5], [2, 2, 2]]), [0, 0, 0]) == 8


def test_random_spins_and_enumeration_argument_errors(q):
    for args in ((0, 4, 1, 0), (10, -1, 1, 0)):
        with pytest.raises(q.QaiaError) as ei:
            q._check(q._lib.qaia_random_spins(*args, None, None))
        assert ei.value.status == q.QAIA_INVALID_ARGUMENT
    with pytest.raises(q.QaiaError) as ei:
        q._check(q._lib.qaia_random_spins(10, 4, 1, 0, None, None))
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT
    with pytest.raises(q.QaiaError) as ei:
        q._check(q._lib.qaia_enumerate_cuts(None, 0, 4, None, None))
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT
    # an empty request is valid and touches no device
    q._check(q._lib.qaia_random_spins(10, 0, 1, 0, None, None))


def test_pareto_ranks_argument_errors(q):
    import ctypes
    n = ctypes.c_int32()
    with pytest.raises(q.QaiaError) as ei:
        q._check(q._lib.qaia_pareto_ranks(None, 4, 3, 0, None, ctypes.byref(n), None, 0, None))
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT  # max_rank < 1
    with pytest.raises(q.QaiaError) as ei:
        q._check(q._lib.qaia_pareto_ranks(None, 4, 9, 5, None, ctypes.byref(n), None, 0, None))
    assert ei.value.status == q.QAIA_INVALID_ARGUMENT  # m > 8
    q._check(q._lib.qaia_pareto_ranks(None, 0, 3, 5, None, ctypes.byref(n), None, 0, None))
    assert n.value == 0


def test_peak_kernels_argument_errors(q):
    bad = [
        lambda: q._lib.qaia_peak_fma(0, 10, 1.0, 1.0, 16, None),            # blocks < 1
        lambda: q._lib.qaia_peak_fma(4, 0, 1.0, 1.0, 16, None),             # iters < 1
        lambda: q._lib.qaia_peak_fma(4, 10, 1.0, 1.0, None, None),          # null out
        lambda: q._lib.qaia_peak_mfma(3, 4, 10, 16, None),                  # unknown precision
        lambda: q._lib.qaia_peak_mfma(q.PRECISIONS["fp8"], 4, 1 << 16, 16, None),  # 4 * 64 * iters >= 2^24
        lambda: q._lib.qaia_peak_copy(16, 4096, 40, None),                  # not a multiple of 16
        lambda: q._lib.qaia_peak_copy(16, 32, 64, None),                    # overlapping buffers
        lambda: q._lib.qaia_peak_copy(8, 4096, 64, None),                   # misaligned
    ]
    for call in bad:
        with pytest.raises(q.QaiaError) as ei:
            q._check(call())
        assert ei.value.status == q.QAIA_INVALID_ARGUMENT
    q._check(q._lib.qaia_peak_copy(None, None, 0, None))  # empty copy: nothing enqueued


@pytest.mark.parametrize("threads", ["1", "3", "8"])
def test_hypervolume_threaded_paths_match_oracle(q, threads, monkeypatch):
    """The m = 3 and m = 4 paths with their threaded non-dominated filter and
    (m = 4) threaded sweep: a front with duplicates, dominated points, ties in
    every coordinate and points clipped to zero extent, large enough to split
    over threads."""
    monkeypatch.setenv("QAIA_HV_THREADS", threads)
    rng = np.random.default_rng(300 + int(threads))
    for m in (3, 4):
        d = np.abs(rng.standard_normal((400, m)))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        front = np.round(d * 3000).astype(np.int64)            # mostly non-dominated, some ties
        dominated = front[:120] - rng.integers(0, 40, size=(120, m))
        pts = np.concatenate([front, front[:100], dominated, -front[:20]])  # duplicates, clipped
        pts = pts[rng.permutation(len(pts))]
        ref = np.zeros(m, np.int64)
        assert q.qaia_hypervolume(pts, ref) == oracle.hypervolume(pts, ref), m


def test_header_compiles_as_c99_and_cpp(tmp_path):
    """include/qaia.h is a C ABI: it must compile as pedantic C99 and as C++."""
    import shutil
    import subprocess
    src = tmp_path / "use.c"
    src.write_text('#include "qaia.h"\nint main(void) { return qaia_abi_version() > 0 ? 0 : 1; }\n')
    inc = os.path.join(ROOT, "include")
    for cc, args in (("gcc", ["-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror"]),
                     ("g++", ["-std=c++17", "-Wall", "-Wextra", "-Werror", "-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, *args, "-I", inc, "-c", str(src), "-o", str(tmp_path / "use.o")],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
