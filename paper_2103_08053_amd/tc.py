"""Thin ctypes binding of ``libtrust_tc.so`` (declared in ``include/trust_tc.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (workspace, outputs) and the stream.
If the library is not built this module raises on import of its entry points;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtrust_tc.so")

TC_OK, TC_E_INVALID, TC_E_RANGE, TC_E_NOMEM, TC_E_DEVICE, TC_E_UNSUPPORTED, TC_E_BUSY = range(7)
TC_F_NO_LPT, TC_F_FORCE_WG, TC_F_FORCE_HUB, TC_F_SCATTER_CSR, TC_F_WIDE_ADDR = 0x1, 0x2, 0x4, 0x8, 0x10
TC_F_FORCE_BIG, TC_F_NO_PACK, TC_F_NO_MID, TC_F_RECORDS = 0x20, 0x1000, 0x2000, 0x4000

EXPORTS = [
    "tc_default_params", "tc_create", "tc_destroy", "tc_set_params", "tc_get_params", "tc_status_str",
    "tc_last_error", "tc_workspace_bytes", "tc_count", "tc_graph_footprint", "tc_graph_build",
    "tc_count_scratch_bytes", "tc_graph_count", "tc_graph_info_get", "tc_graph_release",
    "tc_timing_enable", "tc_timing_last", "tc_batch_footprint", "tc_batch_build", "tc_graph_count_each",
    "tc_graph_count_replay", "tc_graph_k", "tc_graph_count_shard", "tc_graph_collisions",
    "tc_graph_count_simple", "tc_graph_bin_work", "tc_vc_locate", "tc_wide_list_addressing",
    "tc_count_graphs_bytes", "tc_count_graphs", "tc_count_graphs_replay", "tc_graph_count_static",
]
TC_STATIC_SCRATCH_BYTES = 128 << 20


class TCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class RangeError(TCError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "struct_size", "wg_waves", "wg_lds_bytes", "wave_max_dplus", "slots_per_bucket", "load_factor_pct",
        "hash_kind", "light_chunk", "grid_wgs", "flags")]


class _CollisionStats(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_uint64), ("sum_max_collision", ctypes.c_uint64), ("tables", ctypes.c_uint64),
                ("max_collision", ctypes.c_uint64)]


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("wedges_plus", ctypes.c_uint64),
                ("max_dplus", ctypes.c_uint32), ("n_hub", ctypes.c_uint32), ("n_wg", ctypes.c_uint32),
                ("n_wave", ctypes.c_uint32), ("wave_cap", ctypes.c_uint32), ("wg_cap", ctypes.c_uint32),
                ("n_big", ctypes.c_uint32), ("big_cap", ctypes.c_uint32), ("n_packed", ctypes.c_uint32),
                ("n_mid", ctypes.c_uint32), ("mid_cap", ctypes.c_uint32), ("records", ctypes.c_uint32)]


@dataclass
class Params:
    """Tuning knobs (see ``tc_params`` in the header); none changes any count."""
    wg_waves: int = 8
    wg_lds_bytes: int = 49152
    wave_max_dplus: int = 0
    slots_per_bucket: int = 4
    load_factor_pct: int = 50
    hash_kind: int = 0
    light_chunk: int = 16
    grid_wgs: int = 0
    flags: int = 0

    def to_c(self) -> _Params:
        p = _Params()
        p.struct_size = ctypes.sizeof(_Params)
        for f in fields(self):
            setattr(p, f.name, int(getattr(self, f.name)))
        return p

    @classmethod
    def from_c(cls, p: _Params) -> "Params":
        return cls(**{f.name: int(getattr(p, f.name)) for f in fields(cls)})


@dataclass
class GraphInfo:
    n: int
    m: int
    wedges_plus: int
    max_dplus: int
    n_hub: int
    n_wg: int
    n_wave: int
    wave_cap: int
    wg_cap: int
    n_big: int = 0
    big_cap: int = 0
    n_packed: int = 0
    n_mid: int = 0      # large-LDS-bin vertices counted by the half-LDS launch (included in n_big)
    mid_cap: int = 0
    records: int = 0    # 1: the graph carries the record layout (TC_F_RECORDS)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2103_08053_amd.build`")
    lib = ctypes.CDLL(path)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    pp = ctypes.POINTER(_Params)
    sig = {
        "tc_default_params": [pp],
        "tc_create": [i32, pp, ctypes.POINTER(vp)],
        "tc_destroy": [vp],
        "tc_set_params": [vp, pp],
        "tc_get_params": [vp, pp],
        "tc_workspace_bytes": [vp, u32, u64, ctypes.POINTER(u64)],
        "tc_count": [vp, u32, u64, vp, vp, vp, vp, u64, vp, ctypes.POINTER(u64)],
        "tc_graph_footprint": [vp, u32, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "tc_graph_build": [vp, u32, u64, vp, vp, vp, u64, vp, u64, vp, ctypes.POINTER(vp)],
        "tc_count_scratch_bytes": [vp, u32, u64, ctypes.POINTER(u64)],
        "tc_graph_count": [vp, vp, vp, vp, vp, u64, vp],
        "tc_graph_info_get": [vp, vp, ctypes.POINTER(_GraphInfo)],
        "tc_graph_release": [vp],
        "tc_timing_enable": [vp, i32],
        "tc_batch_footprint": [vp, u32, u32, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "tc_batch_build": [vp, u32, u32, u64, vp, vp, vp, vp, vp, u64, vp, u64, vp, ctypes.POINTER(vp)],
        "tc_graph_count_each": [vp, vp, vp, vp, vp, u64, vp],
        "tc_graph_count_replay": [vp, vp, vp, vp, vp, u64, vp],
        "tc_graph_count_shard": [vp, vp, u32, u32, vp, vp, vp, u64, vp],
        "tc_graph_collisions": [vp, vp, i32, vp, u64, vp, ctypes.POINTER(_CollisionStats)],
        "tc_graph_count_simple": [vp, vp, u32, vp, vp, u64, vp],
        "tc_graph_bin_work": [vp, vp, ctypes.POINTER(u64)],
        "tc_graph_k": [vp, ctypes.POINTER(u32)],
        "tc_timing_last": [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "tc_vc_locate": [ctypes.POINTER(u32), u32, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)],
        "tc_wide_list_addressing": [u64, u32, ctypes.POINTER(i32)],
        "tc_count_graphs_bytes": [vp, u32, u64, u64, i32, ctypes.POINTER(u64)],
        "tc_count_graphs": [vp, u32, ctypes.POINTER(vp), vp, ctypes.POINTER(vp), vp, u64, vp],
        "tc_count_graphs_replay": [vp, u32, ctypes.POINTER(vp), vp, ctypes.POINTER(vp), vp, u64, vp],
        "tc_graph_count_static": [vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.tc_status_str.argtypes = [ctypes.c_int]
    lib.tc_status_str.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = [vp]
    lib.tc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status == TC_OK:
        return
    lib = load_library()
    msg = lib.tc_status_str(status).decode()
    if ctx is not None:
        detail = lib.tc_last_error(ctx).decode()
        if detail:
            msg = f"{msg}: {detail}"
    raise (RangeError if status == TC_E_RANGE else TCError)(status, msg)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _edge_tensor(x, device):
    torch = _torch()
    t = torch.as_tensor(x)
    if t.dtype != torch.int32 and t.dtype != torch.uint32:
        t = t.to(torch.int64)
        if t.numel() and (int(t.min()) < 0 or int(t.max()) > 0xFFFFFFFF):
            raise ValueError("vertex ids must fit in uint32")
        t = t.to(torch.uint32) if hasattr(torch, "uint32") else t.to(torch.int32)
    return t.to(device).contiguous()


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device: int = 0, params: Params | None = None):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        p = (params or Params()).to_c()
        _check(self.lib.tc_create(device, ctypes.byref(p), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> Params:
        p = _Params()
        _check(self.lib.tc_get_params(self.h, ctypes.byref(p)), self.h)
        return Params.from_c(p)

    @params.setter
    def params(self, params: Params):
        p = params.to_c()
        _check(self.lib.tc_set_params(self.h, ctypes.byref(p)), self.h)

    def timing(self, on: bool = True):
        """Record HIP events around the build and the count kernel of every call."""
        _check(self.lib.tc_timing_enable(self.h, 1 if on else 0), self.h)

    def last_times_ms(self) -> tuple[float, float]:
        """(build ms, count-kernel ms) of the last timed calls (-1 if none)."""
        b, c = ctypes.c_float(), ctypes.c_float()
        _check(self.lib.tc_timing_last(self.h, ctypes.byref(b), ctypes.byref(c)), self.h)
        return b.value, c.value

    def workspace_bytes(self, n: int, m_in: int) -> int:
        b = ctypes.c_uint64()
        _check(self.lib.tc_workspace_bytes(self.h, n, m_in, ctypes.byref(b)), self.h)
        return b.value

    def footprint(self, n: int, m_in: int) -> tuple[int, int]:
        s, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.tc_graph_footprint(self.h, n, m_in, ctypes.byref(s), ctypes.byref(t)), self.h)
        return s.value, t.value

    def batch_footprint(self, k: int, n_total: int, m_total: int) -> tuple[int, int]:
        s, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.tc_batch_footprint(self.h, k, n_total, m_total, ctypes.byref(s), ctypes.byref(t)), self.h)
        return s.value, t.value

    def scratch_bytes(self, n: int, m_in: int) -> int:
        b = ctypes.c_uint64()
        _check(self.lib.tc_count_scratch_bytes(self.h, n, m_in, ctypes.byref(b)), self.h)
        return b.value

    def count(self, src, dst, n: int, per_vertex: bool = False, workspace=None, stream=None):
        """Triangle count of the undirected graph given by edge samples src[i] -- dst[i].

        Returns (total, per_vertex int64 tensor or None).  src/dst: device or host
        integer tensors/arrays (copied to the device if needed)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        s = _edge_tensor(src, dev)
        d = _edge_tensor(dst, dev)
        if s.shape != d.shape:
            raise ValueError("src and dst differ in length")
        m_in = s.numel()
        need = self.workspace_bytes(n, m_in)
        ws = workspace
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        pv = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if per_vertex else None
        tot = ctypes.c_uint64()
        _check(self.lib.tc_count(self.h, n, m_in, _ptr(s), _ptr(d), _ptr(pv), _ptr(ws), ws.numel(),
                                 _stream_ptr(stream), ctypes.byref(tot)), self.h)
        return tot.value, (pv[:n] if per_vertex else None)

    def build(self, src, dst, n: int, stream=None) -> "Graph":
        return Graph(self, src, dst, n, stream=stream)

    def count_graphs_bytes(self, k: int, n_total: int, m_max: int, per_vertex: bool = True) -> int:
        """Workspace bytes of :meth:`count_graphs` for up to k handles, n_total vertices, m_max samples each."""
        b = ctypes.c_uint64()
        _check(self.lib.tc_count_graphs_bytes(self.h, k, n_total, m_max, int(per_vertex), ctypes.byref(b)), self.h)
        return b.value

    def count_graphs_async(self, graphs, totals, per_vertex_outs=None, workspace=None, stream=None,
                           replay: bool = False):
        """Enqueue one count of built handles ``graphs`` (tc_count_graphs / tc_count_graphs_replay):
        ``totals`` is a device int64 tensor with one entry per graph (batch handles hold several);
        ``per_vertex_outs`` None or one device int64 tensor per handle.  Returns the workspace used."""
        torch = _torch()
        k = len(graphs)
        hs = (ctypes.c_void_p * k)(*[g.h.value for g in graphs])
        ws = workspace
        if ws is None:
            need = self.count_graphs_bytes(k, sum(g.n for g in graphs), max(g.m_in for g in graphs),
                                           per_vertex_outs is not None)
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=totals.device)
        pvs = None
        if per_vertex_outs is not None:
            pvs = (ctypes.c_void_p * k)(*[t.data_ptr() if t is not None else 0 for t in per_vertex_outs])
        fn = self.lib.tc_count_graphs_replay if replay else self.lib.tc_count_graphs
        _check(fn(self.h, k, hs, _ptr(totals), pvs, _ptr(ws), ws.numel(), _stream_ptr(stream)), self.h)
        return ws

    def count_graphs(self, graphs, per_vertex: bool = False, workspace=None, stream=None, replay: bool = False):
        """Count built handles (:class:`Graph` / :class:`Batch`) together.  Returns (totals, per-vertex):
        totals[g] is an int for a single graph and a list for a batch handle; per-vertex is None or a
        list of device tensors."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        nt = sum(g.k for g in graphs)
        totals = torch.empty(max(nt, 1), dtype=torch.int64, device=dev)
        pvs = [torch.empty(max(g.n, 1), dtype=torch.int64, device=dev) for g in graphs] if per_vertex else None
        self.count_graphs_async(graphs, totals, pvs, workspace=workspace, stream=stream, replay=replay)
        flat = totals.cpu().tolist()
        out, t0 = [], 0
        for g in graphs:
            out.append(flat[t0] if g.k == 1 else flat[t0:t0 + g.k])
            t0 += g.k
        return out, ([p[: g.n] for p, g in zip(pvs, graphs)] if per_vertex else None)


class Graph:
    """A graph (or a batch of graphs) cleaned, oriented and binned once on the
    device; count it many times.  Use :meth:`Context.build` or :class:`Batch`."""

    def __init__(self, ctx: Context, src, dst, n: int, stream=None, storage=None, temp=None, _batch=None,
                 sync: bool = True, scratch: bool = True):
        torch = _torch()
        self.ctx = ctx
        self.n = n
        dev = torch.device("cuda", ctx.device)
        s = _edge_tensor(src, dev)
        d = _edge_tensor(dst, dev)
        self.m_in = s.numel()
        if _batch is None:
            sb, tb = ctx.footprint(n, self.m_in)
        else:
            sb, tb = ctx.batch_footprint(_batch[0], n, self.m_in)
        self.storage = storage if storage is not None else torch.empty(max(sb, 1), dtype=torch.uint8, device=dev)
        tmp = temp if temp is not None else torch.empty(max(tb, 1), dtype=torch.uint8, device=dev)
        # count scratch of this graph's own count calls (not needed when it is only counted through
        # Context.count_graphs, which brings its own workspace)
        self.scratch = (torch.empty(max(ctx.scratch_bytes(n, self.m_in), 1), dtype=torch.uint8, device=dev)
                        if scratch else None)
        h = ctypes.c_void_p()
        if _batch is None:
            _check(ctx.lib.tc_graph_build(ctx.h, n, self.m_in, _ptr(s), _ptr(d), _ptr(self.storage),
                                          self.storage.numel(), _ptr(tmp), tmp.numel(), _stream_ptr(stream),
                                          ctypes.byref(h)), ctx.h)
        else:
            k, voff, eoff = _batch
            _check(ctx.lib.tc_batch_build(ctx.h, k, n, self.m_in, _ptr(voff), _ptr(eoff), _ptr(s), _ptr(d),
                                          _ptr(self.storage), self.storage.numel(), _ptr(tmp), tmp.numel(),
                                          _stream_ptr(stream), ctypes.byref(h)), ctx.h)
        self.h = h
        kk = ctypes.c_uint32()
        _check(ctx.lib.tc_graph_k(self.h, ctypes.byref(kk)))
        self.k = kk.value
        self.totals_dev = torch.zeros(self.k, dtype=torch.int64, device=dev)
        self.total_dev = self.totals_dev[:1]
        self._keep = (s, d, tmp, _batch)  # alive until the build has run on the stream
        if sync:
            self.info(stream)  # synchronises; raises RangeError on bad ids
            self._keep = None

    def info(self, stream=None) -> GraphInfo:
        gi = _GraphInfo()
        _check(self.ctx.lib.tc_graph_info_get(self.h, _stream_ptr(stream), ctypes.byref(gi)), self.ctx.h)
        return GraphInfo(**{k: int(getattr(gi, k)) for k, _ in _GraphInfo._fields_})

    def count_async(self, per_vertex_out=None, stream=None, replay: bool = False, shard=None):
        """Launch the count; totals land in ``self.totals_dev`` (device int64[k]).
        With ``replay`` the device work is captured once into a HIP graph and replayed.
        ``shard=(r, g)`` counts only workload partition r of g (tc_graph_count_shard)."""
        lib = self.ctx.lib
        if shard is not None:
            if replay:
                raise ValueError("replay counts the whole graph")
            r, g = shard
            _check(lib.tc_graph_count_shard(self.ctx.h, self.h, r, g, _ptr(self.totals_dev), _ptr(per_vertex_out),
                                            _ptr(self.scratch), self.scratch.numel(), _stream_ptr(stream)), self.ctx.h)
            return
        fn = lib.tc_graph_count_replay if replay else lib.tc_graph_count_each
        _check(fn(self.ctx.h, self.h, _ptr(self.totals_dev), _ptr(per_vertex_out), _ptr(self.scratch),
                  self.scratch.numel(), _stream_ptr(stream)), self.ctx.h)

    def count(self, per_vertex: bool = False, stream=None, replay: bool = False, shard=None):
        """(total, per-vertex tensor or None) for a single graph; (totals list, ...) for a batch."""
        torch = _torch()
        pv = torch.empty(max(self.n, 1), dtype=torch.int64, device=self.storage.device) if per_vertex else None
        self.count_async(pv, stream, replay=replay, shard=shard)
        tot = self.totals_dev.cpu().tolist()
        return (tot[0] if self.k == 1 else tot), (pv[: self.n] if per_vertex else None)

    def bin_work(self, stream=None) -> list[int]:
        """Sum of W(u) per bin: global table, large LDS, workgroup, wavefront, packed, skipped."""
        arr = (ctypes.c_uint64 * 6)()
        _check(self.ctx.lib.tc_graph_bin_work(self.h, _stream_ptr(stream), arr), self.ctx.h)
        return [int(x) for x in arr]

    def count_simple(self, edge_centric: bool = False, build_only: bool = False, stream=None) -> int:
        """Total from the plain vertex- or edge-centric design of Section 3.3 (construction ablation)."""
        mode = (1 if edge_centric else 0) | (2 if build_only else 0)
        _check(self.ctx.lib.tc_graph_count_simple(self.ctx.h, self.h, mode, _ptr(self.totals_dev), _ptr(self.scratch),
                                                  self.scratch.numel(), _stream_ptr(stream)), self.ctx.h)
        return int(self.totals_dev[0].item())

    def collisions(self, per_vertex: bool = True, stream=None) -> dict:
        """Collision statistics of the tables a count builds (Equation 2's phi and friends)."""
        st = _CollisionStats()
        _check(self.ctx.lib.tc_graph_collisions(self.ctx.h, self.h, int(per_vertex), _ptr(self.scratch),
                                                self.scratch.numel(), _stream_ptr(stream), ctypes.byref(st)),
               self.ctx.h)
        return {k: int(getattr(st, k)) for k, _ in _CollisionStats._fields_}

    def release(self):
        if getattr(self, "h", None):
            self.ctx.lib.tc_graph_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Batch(Graph):
    """k graphs counted together: one build and one persistent count launch.

    ``graphs`` is a list of (n_g, src_g, dst_g) with local ids in [0, n_g);
    src_g / dst_g are host arrays or device tensors.  With ``sync=False`` the
    build is only enqueued on ``stream`` (range errors then surface at the
    next :meth:`info`)."""

    def __init__(self, ctx: Context, graphs, stream=None, sync: bool = True):
        import numpy as np
        torch = _torch()
        dev = torch.device("cuda", ctx.device)
        ns = np.array([int(g[0]) for g in graphs], dtype=np.int64)
        ms = np.array([len(g[1]) for g in graphs], dtype=np.int64)
        voff = np.zeros(len(graphs) + 1, np.int64)
        eoff = np.zeros(len(graphs) + 1, np.int64)
        np.cumsum(ns, out=voff[1:])
        np.cumsum(ms, out=eoff[1:])
        if graphs and all(isinstance(g[1], torch.Tensor) and g[1].is_cuda for g in graphs):
            src = torch.cat([g[1].view(torch.int32) for g in graphs])
            dst = torch.cat([g[2].view(torch.int32) for g in graphs])
        else:
            src = np.concatenate([np.asarray(g[1], dtype=np.uint32) for g in graphs]) if graphs \
                else np.zeros(0, np.uint32)
            dst = np.concatenate([np.asarray(g[2], dtype=np.uint32) for g in graphs]) if graphs \
                else np.zeros(0, np.uint32)
            src, dst = src.view(np.int32), dst.view(np.int32)
        self.voff = voff
        vo = torch.from_numpy(voff).to(dev, non_blocking=True)
        eo = torch.from_numpy(eoff).to(dev, non_blocking=True)
        super().__init__(ctx, src, dst, int(voff[-1]), stream=stream, _batch=(len(graphs), vo, eo), sync=sync)


def vc_locate(incl_prefix, index: int) -> tuple[int, int]:
    """(list k, position in it) of flattened index ``index`` under virtual combination, computed by
    the library's own index-map code on the host (``tc_vc_locate``)."""
    lib = load_library()
    arr = (ctypes.c_uint32 * len(incl_prefix))(*[int(x) for x in incl_prefix])
    k, off = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.tc_vc_locate(arr, len(incl_prefix), int(index), ctypes.byref(k), ctypes.byref(off)))
    return k.value, off.value


def wide_list_addressing(m_in: int, flags: int = 0) -> bool:
    """Whether a count over m_in edge samples uses 64-bit list addressing (``tc_wide_list_addressing``)."""
    w = ctypes.c_int()
    _check(load_library().tc_wide_list_addressing(int(m_in), int(flags), ctypes.byref(w)))
    return bool(w.value)


_default_ctx = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx


def count(src, dst, n: int, per_vertex: bool = False):
    """Triangle count (and optional per-vertex counts) on device 0."""
    return default_context().count(src, dst, n, per_vertex=per_vertex)
