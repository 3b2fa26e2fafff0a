"""tc_graph_count_static (count scratch in the library's static device buffer, no allocation)
against tc_graph_count with a caller workspace, called through the C-ABI."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def count_static(ctx, graph, per_vertex, torch):
    from paper_2103_08053_amd.tc import _check, _ptr, _stream_ptr
    tot = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    pv = torch.full((max(graph.n, 1),), -1, dtype=torch.int64, device="cuda:0") if per_vertex else None
    _check(ctx.lib.tc_graph_count_static(ctx.h, graph.h, _ptr(tot), _ptr(pv), _stream_ptr(None)), ctx.h)
    torch.cuda.synchronize()
    return int(tot[0]), (pv[: graph.n] if per_vertex else None)


def count_workspace(ctx, graph, per_vertex, torch):
    from paper_2103_08053_amd.tc import _check, _ptr, _stream_ptr
    tot = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    pv = torch.full((max(graph.n, 1),), -1, dtype=torch.int64, device="cuda:0") if per_vertex else None
    ws = torch.empty(max(ctx.scratch_bytes(graph.n, graph.m_in), 1), dtype=torch.uint8, device="cuda:0")
    _check(ctx.lib.tc_graph_count(ctx.h, graph.h, _ptr(tot), _ptr(pv), _ptr(ws), ws.numel(), _stream_ptr(None)),
           ctx.h)
    torch.cuda.synchronize()
    return int(tot[0]), (pv[: graph.n] if per_vertex else None)


@pytest.mark.parametrize("kw", [{}, dict(flags=4), dict(flags=32)], ids=["default", "hub", "big"])
def test_static_scratch_equals_workspace_twice(torch, kw):
    """Two calls in a row, the second on a smaller graph: each equals the workspace entry point's
    result (total and per-vertex) and the oracle."""
    from paper_2103_08053_amd import Context, Params
    ctx = Context(0, Params(**kw))
    big = gg.dirty(gg.rmat(15, 16, seed=21), seed=4)
    small = gg.barabasi_albert(3000, 7, seed=5)
    for g in (big, small):
        say(f"[gpu] static scratch: {g.name} n={g.n} m_in={g.m_in} params={kw}")
        graph = ctx.build(g.src, g.dst, g.n)
        r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
        for pv_on in (True, False):
            t_s, pv_s = count_static(ctx, graph, pv_on, torch)
            t_w, pv_w = count_workspace(ctx, graph, pv_on, torch)
            assert t_s == t_w == r.total, (g.name, pv_on, t_s, t_w, r.total)
            if pv_on:
                assert torch.equal(pv_s, pv_w), g.name
                assert (pv_s.cpu().numpy().astype(np.uint64) == r.per_vertex).all(), g.name
        graph.release()


def test_static_scratch_limit(torch):
    """A graph whose count scratch (its per-vertex staging alone) exceeds the static buffer is
    refused before any launch; a small graph on the same context passes."""
    from paper_2103_08053_amd import Context, TCError
    from paper_2103_08053_amd.tc import TC_STATIC_SCRATCH_BYTES
    ctx = Context(0)
    n = TC_STATIC_SCRATCH_BYTES // 8 + 1024  # 8 n bytes of staging alone exceed the buffer
    src = np.array([0, 1, 2], np.uint32)
    dst = np.array([1, 2, 0], np.uint32)
    assert ctx.scratch_bytes(n, 3) > TC_STATIC_SCRATCH_BYTES
    graph = ctx.build(src, dst, n)
    with pytest.raises(TCError):
        count_static(ctx, graph, True, torch)
    ok = ctx.build(src, dst, 10)
    assert count_static(ctx, ok, True, torch)[0] == 1
