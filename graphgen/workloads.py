"""Benchmarked input recipes: every size, parameter and seed in one place.

Each recipe returns edge lists from :mod:`graphgen`; nothing here counts
anything.  The R-MAT quadrant probabilities (0.57, 0.19, 0.19, 0.05) and the
edge factor 16 are those of the Graph500-style R-MAT family; the paper's own
synthetic inputs (its rMat, random and 3-D grid graphs) are replaced by these
seeded stand-ins of the same kind.
"""
from __future__ import annotations

import math

import numpy as np

from . import (EdgeList, barabasi_albert, erdos_renyi, log_uniform_int, rmat, splitmix64)

RMAT_ABC = (0.57, 0.19, 0.19)


def rmat_config(scale: int, seed: int = 1, edge_factor: int = 16) -> EdgeList:
    a, b, c = RMAT_ABC
    return rmat(scale, edge_factor, a, b, c, seed=seed)


def small_rmat() -> EdgeList:
    """R-MAT scale 16, edge factor 16, seed 1 (the small parity case)."""
    return rmat_config(16)


def large_rmat() -> EdgeList:
    """R-MAT scale 22, edge factor 16, seed 1 (the throughput case, per-vertex output on)."""
    return rmat_config(22)


def huge_rmat() -> EdgeList:
    """R-MAT scale 26, edge factor 16, seed 1 (skewed hubs)."""
    return rmat_config(26)


def uniform_er() -> EdgeList:
    """Erdos-Renyi on 2^25 vertices with average degree 32 (M = 16 n samples)."""
    n = 1 << 25
    return erdos_renyi(n, 16 * n, seed=1)


def batch_spec(count: int = 4096, seed: int = 1, n_lo: int = 100, n_hi: int = 50000):
    """Per-graph recipe of the small-graph batch: even index -> Erdos-Renyi,
    odd -> Barabasi-Albert; n log-uniform in [n_lo, n_hi]; k uniform in 4..16;
    the Erdos-Renyi graphs take M = n * k samples (mean degree 2k, matched to
    the Barabasi-Albert half).  Every draw comes from the counter-based
    SplitMix64 stream of (seed, graph index)."""
    out = []
    for g in range(count):
        s = splitmix64((seed << 32) ^ g)
        u = ((s >> 11) & ((1 << 53) - 1)) / float(1 << 53)
        n = max(n_lo, min(n_hi, log_uniform_int(u, n_lo, n_hi)))
        k = 4 + (splitmix64(s) % 13)
        kind = "er" if g % 2 == 0 else "ba"
        out.append((kind, int(n), int(k), int(s & 0x7FFFFFFF)))
    return out


def batch_graph(spec) -> EdgeList:
    kind, n, k, s = spec
    if kind == "er":
        return erdos_renyi(n, n * k, seed=s)
    return barabasi_albert(n, k, seed=s)


def batch_graphs(count: int = 4096, seed: int = 1, **kw) -> list[EdgeList]:
    return [batch_graph(sp) for sp in batch_spec(count, seed, **kw)]


def serving_pool(size: int, seed: int = 7, rmat_scales=(10, 20), ba_n=(1000, 1000000)):
    """Request pool of the serving trace: half R-MAT (scale uniform in the
    given range, edge factor 16), half Barabasi-Albert (n log-uniform, k in 4..16)."""
    specs = []
    for i in range(size):
        s = splitmix64((seed << 40) ^ (i * 2654435761))
        if i % 2 == 0:
            lo, hi = rmat_scales
            scale = lo + int(s % (hi - lo + 1))
            specs.append(("rmat", scale, 16, int((s >> 20) & 0x7FFFFFFF)))
        else:
            u = ((s >> 11) & ((1 << 53) - 1)) / float(1 << 53)
            n = log_uniform_int(u, *ba_n)
            k = 4 + (splitmix64(s) % 13)
            specs.append(("ba", int(n), int(k), int((s >> 24) & 0x7FFFFFFF)))
    return specs


def serving_graph(spec) -> EdgeList:
    kind = spec[0]
    if kind == "rmat":
        _, scale, ef, s = spec
        a, b, c = RMAT_ABC
        return rmat(scale, ef, a, b, c, seed=s)
    _, n, k, s = spec
    return barabasi_albert(n, k, seed=s)


def poisson_arrivals(rate: float, duration_s: float, seed: int = 11) -> np.ndarray:
    """Open-loop arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return t[t < duration_s]
