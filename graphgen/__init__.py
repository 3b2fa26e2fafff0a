"""Seeded synthetic graph inputs shared by the CPU checker and the device path.

This module produces edge lists only (uint32 ``src``/``dst`` arrays plus a
vertex count).  It holds none of the triangle-counting arithmetic: removing
self-loops and duplicates, symmetrising, orienting and counting are the job of
whoever consumes the lists.  The random families (R-MAT, Erdos-Renyi,
Barabasi-Albert) come from ``graphgen.c`` through ctypes; the structured
families used as closed-form cases are built here with numpy.

Workload recipes (sizes, parameters and seeds of the benchmarked inputs) live
in :mod:`graphgen.workloads`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` next to its source (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.gg_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, u32p, u32p]
        lib.gg_er.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p]
        lib.gg_ba.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, u32p, u32p]
        lib.gg_ba_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.gg_ba_edges.restype = ctypes.c_uint64
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
        lib.gg_splitmix64.restype = ctypes.c_uint64
        for f in (lib.gg_rmat, lib.gg_er, lib.gg_ba):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


@dataclass
class EdgeList:
    """An input edge list: ``n`` vertex ids, ``src[i] -- dst[i]`` for each sample."""
    n: int
    src: np.ndarray  # uint32
    dst: np.ndarray  # uint32
    name: str = ""

    @property
    def m_in(self) -> int:
        return int(self.src.shape[0])


def _el(n, src, dst, name):
    return EdgeList(int(n), np.ascontiguousarray(src, dtype=np.uint32),
                    np.ascontiguousarray(dst, dtype=np.uint32), name)


# --------------------------------------------------------------------------- random families

def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, samples: int | None = None) -> EdgeList:
    """R-MAT with ``edge_factor * 2**scale`` samples (or ``samples``) on ``2**scale`` ids."""
    m = int(samples if samples is not None else edge_factor * (1 << scale))
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    q = lambda p: min(int(round(p * 2**32)), 2**32 - 1)
    rc = _load().gg_rmat(scale, m, seed, q(a), q(a + b), q(a + b + c), _ptr(src), _ptr(dst))
    if rc:
        raise ValueError(f"gg_rmat failed ({rc})")
    return EdgeList(1 << scale, src, dst, f"rmat{scale}_ef{edge_factor}_s{seed}")


def erdos_renyi(n: int, m: int, seed: int = 1) -> EdgeList:
    """G(n, M) by sampling ``m`` uniform pairs (repeats and self-loops included)."""
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    if _load().gg_er(n, m, seed, _ptr(src), _ptr(dst)):
        raise ValueError("gg_er failed")
    return EdgeList(n, src, dst, f"er{n}_m{m}_s{seed}")


def barabasi_albert(n: int, k: int, seed: int = 1) -> EdgeList:
    """Preferential attachment, ``k`` distinct targets per new vertex, seed graph K_{k+1}."""
    lib = _load()
    m = int(lib.gg_ba_edges(n, k))
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    if lib.gg_ba(n, k, seed, _ptr(src), _ptr(dst)):
        raise ValueError("gg_ba failed")
    return EdgeList(n, src, dst, f"ba{n}_k{k}_s{seed}")


# --------------------------------------------------------------------------- structured families

def complete(n: int) -> EdgeList:
    i, j = np.triu_indices(n, 1)
    return _el(n, i, j, f"K{n}")


def complete_bipartite(a: int, b: int) -> EdgeList:
    i, j = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return _el(a + b, i.ravel(), j.ravel(), f"K{a},{b}")


def complete_tripartite(a: int, b: int, c: int) -> EdgeList:
    parts = [np.arange(a), a + np.arange(b), a + b + np.arange(c)]
    s, d = [], []
    for x in range(3):
        for y in range(x + 1, 3):
            i, j = np.meshgrid(parts[x], parts[y], indexing="ij")
            s.append(i.ravel()); d.append(j.ravel())
    return _el(a + b + c, np.concatenate(s), np.concatenate(d), f"K{a},{b},{c}")


def cycle(n: int) -> EdgeList:
    i = np.arange(n)
    return _el(n, i, (i + 1) % n, f"C{n}")


def wheel(n: int) -> EdgeList:
    """W_n: hub 0 joined to every vertex of the cycle on 1..n-1 (n vertices in total)."""
    r = np.arange(1, n)
    rim_s, rim_d = r, np.where(r + 1 < n, r + 1, 1)
    return _el(n, np.concatenate([np.zeros(n - 1, np.int64), rim_s]),
               np.concatenate([r, rim_d]), f"W{n}")


def star(n: int) -> EdgeList:
    return _el(n, np.zeros(n - 1, np.int64), np.arange(1, n), f"S{n}")


def random_tree(n: int, seed: int = 1) -> EdgeList:
    """Random recursive tree: vertex i > 0 hangs off a uniform earlier vertex."""
    rng = np.random.default_rng(seed)
    i = np.arange(1, n)
    parent = (rng.random(n - 1) * i).astype(np.int64)
    return _el(n, i, parent, f"tree{n}")


def cocktail_party(k: int) -> EdgeList:
    """K_{2k} minus a perfect matching (vertex 2t is not joined to 2t+1)."""
    i, j = np.triu_indices(2 * k, 1)
    keep = ~((i % 2 == 0) & (j == i + 1))
    return _el(2 * k, i[keep], j[keep], f"CP{k}")


def friendship(k: int) -> EdgeList:
    """F_k: k triangles sharing the centre vertex 0."""
    a = 1 + 2 * np.arange(k)
    s = np.concatenate([np.zeros(k, np.int64), np.zeros(k, np.int64), a])
    d = np.concatenate([a, a + 1, a + 1])
    return _el(2 * k + 1, s, d, f"F{k}")


def torus3d(side: int) -> EdgeList:
    """3-D torus side^3: each vertex joined to its +1 neighbour along x, y and z (mod side)."""
    s = side
    x, y, z = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    vid = lambda a, b, c: (a * s + b) * s + c
    u = vid(x, y, z)
    src = np.concatenate([u, u, u])
    dst = np.concatenate([vid((x + 1) % s, y, z), vid(x, (y + 1) % s, z), vid(x, y, (z + 1) % s)])
    return _el(s ** 3, src, dst, f"torus{s}")


def disjoint_union(graphs: list[EdgeList]) -> EdgeList:
    s, d, base = [], [], 0
    for g in graphs:
        s.append(g.src.astype(np.int64) + base)
        d.append(g.dst.astype(np.int64) + base)
        base += g.n
    return _el(base, np.concatenate(s) if s else np.zeros(0), np.concatenate(d) if d else np.zeros(0),
               "+".join(g.name for g in graphs))


def with_isolated(g: EdgeList, extra: int) -> EdgeList:
    return EdgeList(g.n + extra, g.src, g.dst, g.name + f"+iso{extra}")


# --------------------------------------------------------------------------- input transforms

def dirty(g: EdgeList, seed: int = 1, dup_frac: float = 0.3, loops: int = 5) -> EdgeList:
    """Same undirected edge set, presented badly: duplicated and reversed samples,
    self-loops, shuffled order."""
    rng = np.random.default_rng(seed)
    m = g.m_in
    src, dst = g.src.astype(np.int64), g.dst.astype(np.int64)
    flip = rng.random(m) < 0.5
    s = np.where(flip, dst, src)
    d = np.where(flip, src, dst)
    nd = int(m * dup_frac)
    if m and nd:
        pick = rng.integers(0, m, nd)
        rev = rng.random(nd) < 0.5
        ds = np.where(rev, d[pick], s[pick])
        dd = np.where(rev, s[pick], d[pick])
        s = np.concatenate([s, ds])
        d = np.concatenate([d, dd])
    if g.n and loops:
        lv = rng.integers(0, g.n, loops)
        s = np.concatenate([s, lv]); d = np.concatenate([d, lv])
    perm = rng.permutation(s.shape[0])
    return _el(g.n, s[perm], d[perm], g.name + "+dirty")


def relabel(g: EdgeList, seed: int = 1) -> tuple[EdgeList, np.ndarray]:
    """Apply a random permutation p to the ids; returns (graph, p) with new id = p[old]."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(g.n).astype(np.int64)
    return _el(g.n, p[g.src], p[g.dst], g.name + "+perm"), p


def shuffled(g: EdgeList, seed: int = 1) -> EdgeList:
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.m_in)
    return _el(g.n, g.src[perm], g.dst[perm], g.name + "+shuf")


def log_uniform_int(u: float, lo: int, hi: int) -> int:
    return int(math.floor(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
