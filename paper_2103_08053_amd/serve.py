"""Continuous-batching triangle-count server (single GPU).

Requests (graphs as edge lists in pinned host memory) arrive over time.  The
loop, on one host thread:

* admits waiting requests first come first served while their device
  footprint (storage, build memory and the edge list copy, from the
  library's size queries) fits the free HBM budget and the count has fewer
  than `max_batch` requests;
* whenever fewer than `max_inflight` counts are on the device, copies the
  admitted requests to the device and builds them on the *build* stream as
  one disjoint union (tc_batch_build: one set of preprocessing launches for
  all of them), then counts them on the *count* stream with ONE
  tc_count_graphs call replayed from a HIP graph captured once per workspace
  (the launches read k and the graph descriptors from the workspace),
  followed by an asynchronous copy of the totals to pinned host memory; so
  requests that arrive while others are on the GPU join the next count, and
  its build overlaps the counts ahead of it;
* retires a count when its event has completed: every request in it is
  answered and its device memory returns to the budget;
* when the device is idle and exactly one request waits, answers it directly
  through tc_count (no pipeline set-up), unless ``direct_when_idle`` is off.

With ``build="each"`` every request is instead built on its own as soon as it
is admitted (tc_graph_build), and all built or building requests are counted
together: a request's preprocessing starts earlier, but each build pays its
own ~35 launches, which caps the rate (measured below the union server's).

Latency of a request = time its answer is available on the host - its
scheduled arrival time.  :func:`serve_fifo` is the plain baseline: one
request at a time through tc_count, same arrival trace.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .tc import Batch, Context, Graph, Params


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
class _Built:
    req: Request
    graph: object
    bytes: int


@dataclass
class _Flight:
    reqs: list
    handles: list
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
                 max_batch: int = 256, max_inflight: int = 2, direct_when_idle: bool = True, build: str = "union"):
        import torch
        if build not in ("each", "union"):
            raise ValueError("build is 'each' or 'union'")
        self.torch = torch
        self.ctx = Context(device, params)
        self.dev = torch.device("cuda", device)
        self.build_stream = torch.cuda.Stream(device=self.dev)
        self.count_stream = torch.cuda.Stream(device=self.dev)
        self.hbm_budget = hbm_budget
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.direct_when_idle = direct_when_idle
        self.build_mode = build
        self.temp = None            # build temp, reused by every build on the build stream
        self.ws = [None] * max_inflight   # count workspaces, one per count in flight
        self.ws_m = [0] * max_inflight    # the largest edge-sample count each was sized for
        self.ws_free = list(range(max_inflight))

    # ------------------------------------------------------------------ sizes
    def request_bytes(self, r: Request) -> int:
        s, _ = self.ctx.footprint(r.n, r.src.numel())
        return s + 8 * r.src.numel()

    def _temp_for(self, n: int, m_in: int):
        torch = self.torch
        _, t = self.ctx.footprint(n, m_in)
        if self.temp is None or self.temp.numel() < t:
            with torch.cuda.stream(self.build_stream):
                self.temp = torch.empty(max(t, 1 << 20) * 5 // 4, dtype=torch.uint8, device=self.dev)
        return self.temp

    def _workspace(self, slot: int, m_max: int):
        torch = self.torch
        if self.ws[slot] is None or self.ws_m[slot] < m_max:
            m_cap = 1 << max(10, (max(m_max, 1) - 1).bit_length())
            need = self.ctx.count_graphs_bytes(self.max_batch, 1 << 31, min(m_cap, (1 << 31) - 1), per_vertex=False)
            with torch.cuda.stream(self.count_stream):
                self.ws[slot] = torch.empty(need, dtype=torch.uint8, device=self.dev)
            self.ws_m[slot] = m_cap
        return self.ws[slot]

    # ------------------------------------------------------------------ device steps
    def _build_one(self, r: Request) -> _Built:
        torch = self.torch
        with torch.cuda.stream(self.build_stream):
            s = r.src.to(self.dev, non_blocking=True)
            d = r.dst.to(self.dev, non_blocking=True)
            g = Graph(self.ctx, s, d, r.n, stream=self.build_stream, temp=self._temp_for(r.n, s.numel()),
                      sync=False, scratch=False)
        return _Built(r, g, self.request_bytes(r))

    def _count(self, built: list, slot: int) -> _Flight:
        torch = self.torch
        ev_built = torch.cuda.Event()
        ev_built.record(self.build_stream)
        self.count_stream.wait_event(ev_built)
        handles = [b.graph for b in built]
        ws = self._workspace(slot, max(h.m_in for h in handles))
        nt = sum(h.k for h in handles)
        with torch.cuda.stream(self.count_stream):
            totals = torch.empty(nt, dtype=torch.int64, device=self.dev)
            self.ctx.count_graphs_async(handles, totals, None, workspace=ws, stream=self.count_stream, replay=True)
            host = torch.empty(nt, dtype=torch.int64, pin_memory=True)
            host.copy_(totals, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.count_stream)
        reqs = [b.req for b in built]
        return _Flight(reqs, handles, sum(b.bytes for b in built), ev, host, [totals, slot])

    def _count_union(self, reqs: list, slot: int) -> _Flight:
        torch = self.torch
        with torch.cuda.stream(self.build_stream):
            graphs = [(r.n, r.src.to(self.dev, non_blocking=True), r.dst.to(self.dev, non_blocking=True))
                      for r in reqs]
            b = Batch(self.ctx, graphs, stream=self.build_stream, sync=False)
        ev_built = torch.cuda.Event()
        ev_built.record(self.build_stream)
        self.count_stream.wait_event(ev_built)
        ws = self._workspace(slot, b.m_in)
        with torch.cuda.stream(self.count_stream):
            totals = torch.empty(len(reqs), dtype=torch.int64, device=self.dev)
            self.ctx.count_graphs_async([b], totals, None, workspace=ws, stream=self.count_stream, replay=True)
            host = torch.empty(len(reqs), dtype=torch.int64, pin_memory=True)
            host.copy_(totals, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.count_stream)
        need = sum(self.request_bytes(r) for r in reqs) + sum(self.ctx.batch_footprint(len(reqs), b.n, b.m_in))
        return _Flight(reqs, [b], need, ev, host, [totals, slot, graphs])

    # ------------------------------------------------------------------ loop
    def run(self, requests: list[Request], arrivals: np.ndarray, idle_sleep: float = 50e-6,
            stop_after: float | None = None):
        """Serve `requests` arriving at `arrivals` (seconds from start).  With `stop_after`, the loop
        ends at that time even if requests are unanswered (they keep done = -1).  Returns stats."""
        order = np.argsort(arrivals, kind="stable")
        for r, a in zip(requests, arrivals):
            r.arrival = float(a)
        pending: deque = deque()
        built: list = []
        inflight: deque = deque()
        used = 0
        nxt = 0
        done = 0
        counts = 0
        direct = 0
        busy = 0.0  # host-observed time with device work outstanding
        t0 = time.perf_counter()
        last = 0.0
        while done < len(requests):
            now = time.perf_counter() - t0
            if stop_after is not None and now > stop_after:
                break
            if inflight or built:
                busy += now - last
            last = now
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                pending.append(requests[order[nxt]])
                nxt += 1
            # retire finished counts (in launch order)
            while inflight and inflight[0].ev_count.query():
                f = inflight.popleft()
                t = time.perf_counter() - t0
                tots = f.host_totals.tolist()
                for r, v in zip(f.reqs, tots):
                    r.total = int(v)
                    r.done = t
                done += len(f.reqs)
                used -= f.bytes
                for h in f.handles:
                    h.release()
                self.ws_free.append(f.keep[1])
            # idle device, one waiting request: answer it directly
            if self.direct_when_idle and not inflight and not built and len(pending) == 1:
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
            progressed = False
            # admit and build (per-request mode): every waiting request that fits the budget
            if self.build_mode == "each":
                while pending and len(built) < self.max_batch:
                    need = self.request_bytes(pending[0])
                    if used + need > self.hbm_budget and (built or inflight):
                        break  # wait for memory to free up
                    r = pending.popleft()
                    built.append(self._build_one(r))
                    used += need
                    progressed = True
                if built and self.ws_free:
                    f = self._count(built, self.ws_free.pop())
                    inflight.append(f)
                    built = []
                    counts += 1
                    progressed = True
            elif pending and self.ws_free:
                take, need = [], 0
                while pending and len(take) < self.max_batch:
                    r = pending[0]
                    nb = self.request_bytes(r) * 3
                    if used + need + nb > self.hbm_budget and (take or inflight):
                        break
                    take.append(pending.popleft())
                    need += nb
                if take:
                    f = self._count_union(take, self.ws_free.pop())
                    inflight.append(f)
                    used += f.bytes
                    counts += 1
                    progressed = True
            if progressed:
                continue
            if not inflight and not built and nxt < len(order) and not pending:
                # nothing to do until the next arrival
                wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            else:
                time.sleep(idle_sleep)
        wall = time.perf_counter() - t0
        self.torch.cuda.synchronize()
        out = summarize(requests, wall, counts + direct)
        out["direct"] = direct
        out["device_busy_frac"] = busy / wall
        return out


def serve_fifo(ctx: Context, requests: list[Request], arrivals: np.ndarray, stop_after: float | None = None):
    """Plain baseline: each request alone through tc_count, in arrival order.  With `stop_after`,
    requests not started by then stay unanswered (done = -1)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    order = np.argsort(arrivals, kind="stable")
    for r, a in zip(requests, arrivals):
        r.arrival = float(a)
    t0 = time.perf_counter()
    for i in order:
        r = requests[i]
        now = time.perf_counter() - t0
        if stop_after is not None and now > stop_after:
            break
        if now < r.arrival:
            time.sleep(r.arrival - now)
        r.total, _ = ctx.count(r.src.to(dev, non_blocking=True), r.dst.to(dev, non_blocking=True), r.n)
        r.done = time.perf_counter() - t0
    wall = time.perf_counter() - t0
    return summarize(requests, wall, sum(1 for r in requests if r.done >= 0))


def summarize(requests, wall: float, batches: int, window: tuple[float, float] | None = None):
    """Latency percentiles and throughput.  `window` = (t_lo, t_hi): only requests scheduled to
    arrive in it count (warm-up excluded); unanswered ones are reported apart and their latency
    is at least wall - arrival."""
    sel = list(requests)
    if window is not None:
        sel = [r for r in requests if window[0] <= r.arrival < window[1]]
    answered = [r for r in sel if r.done >= 0]
    lat = np.array([r.done - r.arrival for r in answered]) if answered else np.zeros(1)
    edges = sum(int(r.src.numel()) for r in answered)
    span = wall if window is None else (window[1] - window[0])
    return {
        "requests": len(sel), "answered": len(answered), "unanswered": len(sel) - len(answered),
        "batches": batches, "wall_s": wall,
        "throughput_rps": len(answered) / span, "input_edges_per_s": edges / span,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
    }
