"""Continuous-batching triangle-count server (single GPU).

Requests (graphs as edge lists in pinned host memory) arrive over time.  The
loop, on one host thread:

* admits waiting requests into the next batch, first come first served,
  while the batch's device footprint (union build storage + temp + count
  scratch, from the library's size queries) fits the free HBM budget and the
  batch has fewer than `max_batch` requests;
* copies a new batch to the device and builds it (tc_batch_build: clean,
  orient, bin, as one disjoint union) on the *build* stream, while earlier
  batches count on the *count* stream (one persistent launch per batch,
  per-graph totals, asynchronous copy of the totals back to pinned memory);
  so requests that arrive while others are on the GPU are admitted as soon
  as budget and pipeline slots free up, and their build overlaps the count
  of the batches ahead of them;
* retires a batch when its count event has completed: every request in it
  is answered, its device memory returns to the budget;
* when the device is idle and exactly one request waits, answers it directly
  through tc_count (no batch set-up: at low load this is the lower-latency
  path), unless ``direct_when_idle`` is off.

Latency of a request = time its answer is available on the host - its
scheduled arrival time.  :func:`serve_fifo` is the plain baseline: one
request at a time through tc_count, same arrival trace.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .tc import Batch, Context, Params


@dataclass
class Request:
    rid: int
    n: int
    src: "object"  # pinned host uint32/int32 tensor
    dst: "object"
    arrival: float = 0.0
    done: float = -1.0
    total: int = -1


@dataclass
class _Flight:
    reqs: list
    batch: object
    bytes: int
    ev_count: object
    host_totals: object
    keep: list = field(default_factory=list)


def _pinned(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int32))
    return t.pin_memory()


def make_request(rid: int, n: int, src, dst) -> Request:
    return Request(rid, int(n), _pinned(src), _pinned(dst))


class Server:
    def __init__(self, device: int = 0, params: Params | None = None, hbm_budget: int = 64 << 30,
                 max_batch: int = 256, max_inflight: int = 2, direct_when_idle: bool = True):
        import torch
        self.torch = torch
        self.ctx = Context(device, params)
        self.dev = torch.device("cuda", device)
        self.build_stream = torch.cuda.Stream(device=self.dev)
        self.count_stream = torch.cuda.Stream(device=self.dev)
        self.hbm_budget = hbm_budget
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.direct_when_idle = direct_when_idle

    def footprint(self, n_total: int, m_total: int, k: int) -> int:
        s, t = self.ctx.batch_footprint(max(k, 1), n_total, m_total)
        return s + t + self.ctx.scratch_bytes(n_total, m_total) + 8 * (k + 1) * 3 + 8 * m_total

    def _launch(self, reqs):
        torch = self.torch
        with torch.cuda.stream(self.build_stream):
            graphs = [(r.n, r.src.to(self.dev, non_blocking=True), r.dst.to(self.dev, non_blocking=True))
                      for r in reqs]
            b = Batch(self.ctx, graphs, stream=self.build_stream, sync=False)
            ev_built = torch.cuda.Event()
            ev_built.record(self.build_stream)
        self.count_stream.wait_event(ev_built)
        host = torch.empty(len(reqs), dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(self.count_stream):
            b.count_async(None, stream=self.count_stream)
            host.copy_(b.totals_dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.count_stream)
        return b, ev, host, graphs

    def run(self, requests: list[Request], arrivals: np.ndarray, idle_sleep: float = 50e-6):
        """Serve `requests` arriving at `arrivals` (seconds from start). Returns stats."""
        order = np.argsort(arrivals, kind="stable")
        pending: deque = deque()
        inflight: deque = deque()
        used = 0
        nxt = 0
        done = 0
        batches = 0
        direct = 0
        busy = 0.0  # host-observed time with at least one batch on the device
        t0 = time.perf_counter()
        last = 0.0
        while done < len(requests):
            now = time.perf_counter() - t0
            if inflight:
                busy += now - last
            last = now
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                r = requests[order[nxt]]
                r.arrival = float(arrivals[order[nxt]])
                pending.append(r)
                nxt += 1
            # retire finished batches (in launch order)
            while inflight and inflight[0].ev_count.query():
                f = inflight.popleft()
                t = time.perf_counter() - t0
                tots = f.host_totals.tolist()
                for r, v in zip(f.reqs, tots):
                    r.total = int(v)
                    r.done = t
                done += len(f.reqs)
                used -= f.bytes
                f.batch.release()
            # idle device, one waiting request: answer it directly
            if self.direct_when_idle and not inflight and len(pending) == 1:
                r = pending.popleft()
                t_start = time.perf_counter()
                r.total, _ = self.ctx.count(r.src.to(self.dev, non_blocking=True),
                                            r.dst.to(self.dev, non_blocking=True), r.n)
                r.done = time.perf_counter() - t0
                busy += r.done - (t_start - t0)
                last = r.done
                done += 1
                direct += 1
                continue
            # admit a new batch
            if pending and len(inflight) < self.max_inflight:
                take, n_tot, m_tot = [], 0, 0
                while pending and len(take) < self.max_batch:
                    r = pending[0]
                    need = self.footprint(n_tot + r.n, m_tot + r.src.numel(), len(take) + 1)
                    if used + need > self.hbm_budget and take:
                        break
                    if used + need > self.hbm_budget and inflight:
                        break  # wait for memory to free up
                    take.append(pending.popleft())
                    n_tot += r.n
                    m_tot += r.src.numel()
                if take:
                    need = self.footprint(n_tot, m_tot, len(take))
                    b, ev, host, keep = self._launch(take)
                    inflight.append(_Flight(take, b, need, ev, host, keep))
                    used += need
                    batches += 1
                    continue
            if not inflight and nxt < len(order) and not pending:
                # nothing to do until the next arrival
                wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            else:
                time.sleep(idle_sleep)
        wall = time.perf_counter() - t0
        out = summarize(requests, wall, batches + direct)
        out["direct"] = direct
        out["device_busy_frac"] = busy / wall
        return out


def serve_fifo(ctx: Context, requests: list[Request], arrivals: np.ndarray):
    """Plain baseline: each request alone through tc_count, in arrival order."""
    import torch
    dev = torch.device("cuda", ctx.device)
    order = np.argsort(arrivals, kind="stable")
    t0 = time.perf_counter()
    for i in order:
        r = requests[i]
        r.arrival = float(arrivals[i])
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        r.total, _ = ctx.count(r.src.to(dev, non_blocking=True), r.dst.to(dev, non_blocking=True), r.n)
        r.done = time.perf_counter() - t0
    wall = time.perf_counter() - t0
    return summarize(requests, wall, len(requests))


def summarize(requests, wall: float, batches: int):
    lat = np.array([r.done - r.arrival for r in requests])
    edges = sum(int(r.src.numel()) for r in requests)
    return {
        "requests": len(requests), "batches": batches, "wall_s": wall,
        "throughput_rps": len(requests) / wall, "input_edges_per_s": edges / wall,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
    }
