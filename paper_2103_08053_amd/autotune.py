"""Autotuner for the counting kernel's knobs (bucket layout, bins, workgroup shape).

Every knob in :class:`Params` changes only speed, never a count; the tuner
checks that on every candidate (a differing count raises).  Search is
coordinate descent from the defaults: each knob in turn is set to each of
its candidate values while the others stay at the best so far, keeping any
strict improvement of the measured count-kernel time (HIP events recorded by
the library around the count launches, median of `trials` launches).  Two
passes over the knobs.  Because knobs that size the tables or the bins are
fixed when a graph is built, each candidate rebuilds the graph (or batch).

Prior: the cost estimate of the paper's Equation 2, phi = sum over vertices
of W(u) * max collision(u), computed by the library for the tables a
candidate builds (tc_graph_collisions).  Candidates of the knobs that decide
the tables (slots per bucket, load factor, hash kind, vertex order) whose phi
exceeds `prior_ratio` times the current best's are rejected without timing.
The knob "order" is the hash-id vertex order (Section 4.1): 0 (degree rank),
0x40 (in-degree), 0x80 (collective degree); "intra" the intra-vertex probe
assignment (Section 4.2): 0 (virtual combination), subwaves of 8/16/32 lanes
(0x100/0x200/0x400) or one list per wavefront (0x800); both set in the flags.

Results are cached in a JSON file keyed by coarse features of the workload
(log2 of n, m, the largest out-degree and the mean 2-hop list length W+/m,
per-vertex mode, batch or single graph), so graphs of the same kind reuse a
tuned configuration without searching again.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, replace

from .tc import Batch, Context, Graph, Params

SPACE = {
    "wg_lds_bytes": [16384, 24576, 32768, 40960, 65536],
    "wg_waves": [4, 8, 16],
    "slots_per_bucket": [2, 4],
    "load_factor_pct": [25, 35, 50],
    "light_chunk": [1, 2, 4, 8, 16, 32],
    "hash_kind": [0, 1],
    "wave_max_dplus": [0, 32, 64, 128],
    "order": [0, 0x40, 0x80],
    "intra": [0, 0x100, 0x200, 0x400, 0x800],
}
TABLE_KNOBS = ("slots_per_bucket", "load_factor_pct", "hash_kind", "order")
FLAG_KNOBS = {"order": 0x40 | 0x80, "intra": 0x100 | 0x200 | 0x400 | 0x800}


def _with(p: Params, knob: str, v) -> Params:
    if knob in FLAG_KNOBS:
        return replace(p, flags=(p.flags & ~FLAG_KNOBS[knob]) | v)
    return replace(p, **{knob: v})


def _get(p: Params, knob: str):
    return p.flags & FLAG_KNOBS[knob] if knob in FLAG_KNOBS else getattr(p, knob)


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_2103_08053_amd", "autotune.json")


def feature_key(info, per_vertex: bool, k: int = 1) -> str:
    lg = lambda x: int(round(math.log2(max(1, x))))
    wpm = info.wedges_plus / max(1, info.m)
    return (f"n{lg(info.n)}_m{lg(info.m)}_d{lg(info.max_dplus)}_w{lg(wpm)}_pv{int(per_vertex)}"
            f"_k{lg(k)}")


def _valid(p: Params) -> bool:
    # the library's rule: every wavefront keeps a 256-word probe queue and at least 64 table words
    return 64 * p.wg_waves <= 1024 and p.wg_lds_bytes <= 131072 and p.wg_lds_bytes // 4 >= p.wg_waves * 320


class _Workload:
    """Builds the graph (or batch) under given knobs and times its count."""

    def __init__(self, device: int, graph_args, batch: bool, per_vertex: bool):
        self.device = device
        self.graph_args = graph_args
        self.batch = batch
        self.per_vertex = per_vertex

    def measure(self, params: Params, trials: int, phi_limit: float | None = None):
        """(median ms, totals, info, k, phi); ms and totals are None when phi exceeds phi_limit."""
        import torch
        ctx = Context(self.device, params)
        if self.batch:
            g = Batch(ctx, self.graph_args)
        else:
            src, dst, n = self.graph_args
            g = Graph(ctx, src, dst, n)
        phi = g.collisions(per_vertex=self.per_vertex)["phi"]
        if phi_limit is not None and phi > phi_limit:
            info, k = g.info(), g.k
            g.release()
            ctx.close()
            return None, None, info, k, phi
        pv = torch.empty(max(g.n, 1), dtype=torch.int64, device=g.storage.device) if self.per_vertex else None
        ctx.timing(True)
        g.count_async(pv)  # warm-up (first launch resolves the launch shape)
        times = []
        for _ in range(trials):
            g.count_async(pv)
            times.append(ctx.last_times_ms()[1])
        ctx.timing(False)
        totals = g.totals_dev.cpu().tolist()
        info = g.info()
        k = g.k
        g.release()
        ctx.close()
        times.sort()
        return times[len(times) // 2], totals, info, k, phi


def tune(graph_args, batch: bool = False, per_vertex: bool = False, device: int = 0, trials: int = 3,
         space: dict | None = None, passes: int = 2, start: Params | None = None, cache_path: str | None = None,
         use_cache: bool = True, verbose: bool = False, prior_ratio: float = 1.5):
    """Tune the knobs for one workload.

    graph_args: (src, dst, n) for a single graph, or a list of (n_g, src_g, dst_g)
    with ``batch=True``.  Returns (best Params, report dict)."""
    space = space or SPACE
    wl = _Workload(device, graph_args, batch, per_vertex)
    best = start or Params()
    t0 = time.time()
    best_ms, ref, info, k, best_phi = wl.measure(best, trials)
    key = feature_key(info, per_vertex, k)
    cache_path = cache_path or default_cache_path()
    if use_cache and os.path.exists(cache_path):
        cached = json.load(open(cache_path)).get(key)
        if cached:
            p = Params(**cached["params"])
            ms, tot, _, _, _ = wl.measure(p, trials)
            if tot != ref:
                raise AssertionError(f"cached params changed the count: {tot} vs {ref}")
            return p, {"key": key, "cached": True, "ms": ms, "default_ms": best_ms}
    history = [(asdict(best), best_ms, best_phi)]
    skipped = 0
    for _ in range(passes):
        improved = False
        for knob, values in space.items():
            for v in values:
                if _get(best, knob) == v:
                    continue
                cand = _with(best, knob, v)
                if not _valid(cand):
                    continue
                limit = prior_ratio * best_phi if knob in TABLE_KNOBS else None
                ms, tot, _, _, phi = wl.measure(cand, trials, limit)
                if ms is None:
                    skipped += 1
                    if verbose:
                        print(f"[tune] {knob}={v}: phi {phi:.4g} > {limit:.4g}, not timed", flush=True)
                    continue
                if tot != ref:
                    raise AssertionError(f"{knob}={v} changed the count: {tot} vs {ref}")
                history.append((asdict(cand), ms, phi))
                if verbose:
                    print(f"[tune] {knob}={v}: {ms:.3f} ms phi {phi:.4g} (best {best_ms:.3f})", flush=True)
                if ms < best_ms * 0.995:
                    best, best_ms, best_phi, improved = cand, ms, phi, True
        if not improved:
            break
    report = {"key": key, "cached": False, "ms": best_ms, "default_ms": history[0][1],
              "params": asdict(best), "evaluated": len(history), "skipped_by_prior": skipped,
              "phi": best_phi, "default_phi": history[0][2], "seconds": round(time.time() - t0, 1)}
    if use_cache:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        data[key] = {"params": asdict(best), "ms": best_ms}
        json.dump(data, open(cache_path, "w"), indent=1)
    return best, report
