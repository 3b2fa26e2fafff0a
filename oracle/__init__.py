"""CPU oracle for exact triangle counting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The device library never loads it and
shares no code with it; the two meet only at the seeded edge lists of
:mod:`graphgen`.

Functions (all take the raw input edge list; cleaning happens inside):

* :func:`count` -- total T and optionally per-vertex t(x), by sorted-merge
  intersection on the (degree, id) orientation (paper Section 2.2: merge-path
  intersection and rank-by-degree orientation; problem statement Sections 1
  and 2.1; cleaning rules Section 2.6).
* :func:`vertex_counts` -- t(x) for queried x from the definition (edges among
  the neighbours of x), orientation-free.
* :func:`oriented` -- the cleaned graph's degrees, out-degrees and sorted
  oriented lists, for checking a device-built CSR.
* :func:`brute_force` -- dense trace(A^3)/6 and diag(A^3)/2 for tiny graphs
  (the matrix form of Section 2.2, used as an independent pin).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_tc.cpp")
_LIB = os.path.join(_HERE, "liboracle_tc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle_tc.so`` (g++ -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint64), ("wedges_plus", ctypes.c_uint64),
                ("max_dplus", ctypes.c_uint64), ("counted_vertices", ctypes.c_uint64),
                ("counted_edges", ctypes.c_uint64), ("counted_wedges", ctypes.c_uint64),
                ("t_clean_s", ctypes.c_double), ("t_count_s", ctypes.c_double),
                ("threads", ctypes.c_int)]


@dataclass
class OracleResult:
    total: int
    per_vertex: np.ndarray | None
    m: int
    wedges_plus: int
    max_dplus: int
    counted_vertices: int
    counted_edges: int
    counted_wedges: int
    t_clean_s: float
    t_count_s: float
    threads: int


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_count.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, ctypes.c_int,
                                     ctypes.c_uint32, u64p, u64p, ctypes.POINTER(_Stats)]
        lib.oracle_vertex_counts.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p,
                                             ctypes.c_uint64, u32p, u64p, ctypes.c_int]
        lib.oracle_oriented.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u32p, u32p,
                                        u32p, u64p]
        for f in (lib.oracle_count, lib.oracle_vertex_counts, lib.oracle_oriented):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


class OracleRangeError(ValueError):
    pass


def count(n, src, dst, per_vertex: bool = False, threads: int = 0, stride: int = 1) -> OracleResult:
    """Exact triangle count of the cleaned undirected graph on ids [0, n)."""
    s, sp = _u32(src)
    d, dp = _u32(dst)
    assert s.shape == d.shape
    tot = ctypes.c_uint64(0)
    pv = np.zeros(n, np.uint64) if per_vertex else None
    pvp = pv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if per_vertex else None
    st = _Stats()
    rc = _load().oracle_count(n, s.shape[0], sp, dp, threads, stride, ctypes.byref(tot), pvp,
                              ctypes.byref(st))
    if rc == 2:
        raise OracleRangeError("vertex id out of range")
    if rc:
        raise RuntimeError(f"oracle_count failed ({rc})")
    return OracleResult(int(tot.value), pv, st.m, st.wedges_plus, st.max_dplus, st.counted_vertices,
                        st.counted_edges, st.counted_wedges, st.t_clean_s, st.t_count_s, st.threads)


def vertex_counts(n, src, dst, queries, threads: int = 0) -> np.ndarray:
    """t(x) for each x in ``queries`` (edges among the neighbours of x)."""
    s, sp = _u32(src)
    d, dp = _u32(dst)
    q, qp = _u32(queries)
    out = np.zeros(q.shape[0], np.uint64)
    rc = _load().oracle_vertex_counts(n, s.shape[0], sp, dp, q.shape[0], qp,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), threads)
    if rc == 2:
        raise OracleRangeError("vertex id out of range")
    if rc:
        raise RuntimeError(f"oracle_vertex_counts failed ({rc})")
    return out


def oriented(n, src, dst):
    """(deg[n], dplus[n], nbr[m]) of the (degree, id)-oriented cleaned graph, lists sorted by id."""
    s, sp = _u32(src)
    d, dp = _u32(dst)
    deg = np.zeros(n, np.uint32)
    dplus = np.zeros(n, np.uint32)
    nbr = np.zeros(max(1, s.shape[0]), np.uint32)
    m = ctypes.c_uint64(0)
    rc = _load().oracle_oriented(n, s.shape[0], sp, dp, _u32(deg)[1], _u32(dplus)[1], _u32(nbr)[1],
                                 ctypes.byref(m))
    if rc == 2:
        raise OracleRangeError("vertex id out of range")
    return deg, dplus, nbr[: m.value].copy()


def brute_force(n, src, dst):
    """Dense pin for tiny graphs: (trace(A^3)/6, diag(A^3)/2) with A the cleaned
    0/1 adjacency matrix (symmetric, zero diagonal)."""
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    if s.size and (s.max() >= n or d.max() >= n):
        raise OracleRangeError("vertex id out of range")
    A = np.zeros((n, n), dtype=np.int64)
    A[s, d] = 1
    A[d, s] = 1
    np.fill_diagonal(A, 0)
    A3 = A @ A @ A
    diag = np.diag(A3).copy()
    return int(diag.sum() // 6), diag // 2
