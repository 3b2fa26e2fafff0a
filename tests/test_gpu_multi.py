"""Many independently built graphs counted by one launch sequence (tc_count_graphs), eager and
replayed from one capture.

Each graph's total (and per-vertex counts) must equal the oracle's on that graph alone, bit for
bit, whatever else shares the call, and one capture must serve calls with other graphs and other k.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import graphgen.workloads as W
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2103_08053_amd import Context
    return Context(0)


def mixed(seed=0, count=10):
    gs = [gg.complete(30), gg.wheel(50), gg.EdgeList(0, np.zeros(0, np.uint32), np.zeros(0, np.uint32), "empty0"),
          gg.friendship(20), gg.EdgeList(7, np.zeros(0, np.uint32), np.zeros(0, np.uint32), "iso7"),
          gg.torus3d(6), gg.complete_tripartite(4, 5, 6), gg.dirty(gg.rmat(11, 16, seed=2 + seed), seed=3)]
    for s in range(count):
        rng = np.random.default_rng(100 + s + 1000 * seed)
        n = int(rng.integers(2, 2000))
        gs.append(gg.dirty(gg.erdos_renyi(n, int(rng.integers(1, 12 * n)), seed=s + seed), seed=s))
        gs.append(gg.barabasi_albert(int(rng.integers(10, 3000)), int(rng.integers(2, 12)), seed=s + seed))
    return gs


_ref_cache = {}


def ref(g):
    key = (g.name, g.n, g.m_in, int(g.src[:8].sum()) if g.m_in else 0)
    if key not in _ref_cache:
        _ref_cache[key] = oracle.count(g.n, g.src, g.dst, per_vertex=True)
    return _ref_cache[key]


def build_all(ctx, graphs):
    return [ctx.build(g.src, g.dst, g.n) for g in graphs]


def check(graphs, totals, pvs=None):
    for i, g in enumerate(graphs):
        r = ref(g)
        assert totals[i] == r.total, (i, g.name, totals[i], r.total)
        if pvs is not None:
            got = pvs[i].cpu().numpy().astype(np.uint64)
            assert (got == r.per_vertex).all(), (i, g.name)


def test_count_graphs_matches_oracle(ctx):
    graphs = mixed()
    say(f"[gpu] tc_count_graphs over {len(graphs)} built graphs")
    hs = build_all(ctx, graphs)
    totals, pvs = ctx.count_graphs(hs, per_vertex=True)
    check(graphs, totals, pvs)
    totals2, _ = ctx.count_graphs(hs)
    assert totals2 == totals


def test_count_graphs_single_equals_plain(ctx):
    g = gg.dirty(gg.rmat(13, 16, seed=7), seed=8)
    h = ctx.build(g.src, g.dst, g.n)
    (t,), (pv,) = ctx.count_graphs([h], per_vertex=True)
    t0, pv0 = h.count(per_vertex=True)
    assert t == t0 == ref(g).total
    assert bool((pv == pv0).all())


def test_count_graphs_with_batch_handles(ctx):
    """Batch handles (disjoint-union builds) mixed with single graphs: totals land handle after handle."""
    from paper_2103_08053_amd import Batch
    graphs = mixed(seed=1, count=6)
    a, b = graphs[:9], graphs[9:]
    say(f"[gpu] tc_count_graphs: batch of {len(a)} + {len(b)} single graphs")
    batch = Batch(ctx, [(g.n, g.src, g.dst) for g in a])
    hs = [batch] + build_all(ctx, b)
    totals, pvs = ctx.count_graphs(hs, per_vertex=True)
    assert len(totals[0]) == len(a)
    check(a, totals[0])
    check(b, totals[1:], pvs[1:])
    pvb = pvs[0].cpu().numpy().astype(np.uint64)
    for i, g in enumerate(a):
        assert (pvb[batch.voff[i]:batch.voff[i + 1]] == ref(g).per_vertex).all(), g.name


@pytest.mark.parametrize("kw", [dict(flags=2), dict(flags=4), dict(flags=32), dict(wg_lds_bytes=4096, wg_waves=2),
                                dict(slots_per_bucket=1, load_factor_pct=100), dict(hash_kind=1),
                                dict(flags=0x40), dict(flags=0x1000), dict(light_chunk=1), dict(grid_wgs=3),
                                dict(flags=0x10), dict(flags=0x4000)],
                         ids=["wg", "hub", "big", "tinylds", "s1full", "hash1", "order_in", "nopack", "chunk1",
                              "grid3", "wide", "records"])
def test_count_graphs_forced_paths(kw):
    from paper_2103_08053_amd import Context, Params
    c = Context(0, Params(**kw))
    graphs = mixed(seed=2, count=4)
    say(f"[gpu] tc_count_graphs forced path {kw}")
    totals, pvs = c.count_graphs(build_all(c, graphs), per_vertex=True)
    check(graphs, totals, pvs)


def test_count_graphs_packed_light_vertices(ctx):
    """Graphs whose light vertices go to the packed bin (sparse Erdos-Renyi), several per call."""
    graphs = [gg.erdos_renyi(3000 + 500 * s, 16 * (3000 + 500 * s), seed=s) for s in range(6)]
    hs = build_all(ctx, graphs)
    assert any(h.info().n_packed > 0 for h in hs)
    totals, pvs = ctx.count_graphs(hs, per_vertex=True)
    check(graphs, totals, pvs)


def test_one_capture_serves_other_batches(ctx, torch):
    """One workspace, one capture: replays with different graphs and different k (larger and
    smaller than the first), eager work and synchronisations in between, every graph equal to the
    oracle each time."""
    from paper_2103_08053_amd import Batch
    sets = [mixed(seed=3, count=5), mixed(seed=4, count=2)[:6], mixed(seed=5, count=9)]
    handles = [build_all(ctx, s) for s in sets]
    # a batch handle in the last set too
    extra = mixed(seed=6, count=1)
    handles[2].append(Batch(ctx, [(g.n, g.src, g.dst) for g in extra]))
    kmax = max(len(h) for h in handles)
    nmax = max(sum(x.n for x in h) for h in handles)
    mmax = max(max(x.m_in for x in h) for h in handles)
    ws = torch.empty(ctx.count_graphs_bytes(kmax, nmax, mmax), dtype=torch.uint8, device="cuda:0")
    other = gg.rmat(12, 16, seed=4)
    other_tot = ctx.count(other.src, other.dst, other.n)[0]
    for rep in range(2):
        for si in (0, 1, 2):
            say(f"[gpu] replay {rep} of set {si}: k={len(handles[si])}")
            pv = si != 1
            totals, pvs = ctx.count_graphs(handles[si], per_vertex=pv, workspace=ws, replay=True)
            torch.cuda.synchronize()
            if si == 2:
                check(sets[2], totals[:-1], pvs[:-1])
                check(extra, totals[-1])
            else:
                check(sets[si], totals, pvs if pv else None)
            assert ctx.count(other.src, other.dst, other.n)[0] == other_tot
            torch.cuda.synchronize()


def test_replay_equals_eager_batch_workload(ctx, torch):
    """The small-graph batch recipe (first 192 graphs, at most 5000 vertices), each graph built
    on its own and all counted by one replayed launch sequence."""
    specs = W.batch_spec(192, seed=3, n_hi=5000)
    graphs = [W.batch_graph(sp) for sp in specs]
    hs = build_all(ctx, graphs)
    t_eager, _ = ctx.count_graphs(hs)
    ws = torch.empty(ctx.count_graphs_bytes(len(hs), sum(h.n for h in hs), max(h.m_in for h in hs)),
                     dtype=torch.uint8, device="cuda:0")
    for _ in range(3):
        t_rep, _ = ctx.count_graphs(hs, workspace=ws, replay=True)
        assert t_rep == t_eager
    check(graphs, t_eager)


def test_count_graphs_unaligned_workspace(ctx, torch):
    """The workspace is used from its first 64 KB boundary: buffers of exactly the queried size at
    any offset (filled with garbage first), eager and replayed, give the oracle's counts."""
    graphs = mixed(seed=3, count=3)
    hs = build_all(ctx, graphs)
    need = ctx.count_graphs_bytes(len(hs), sum(h.n for h in hs), max(max(h.m_in for h in hs), 1), per_vertex=True)
    for off in (256, 4096, 65536 - 256, 65536 + 512):
        buf = torch.full((need + off,), 0x5A, dtype=torch.uint8, device="cuda:0")
        ws = buf[off:off + need]
        for replay in (False, True):
            say(f"[gpu] tc_count_graphs workspace offset {off} replay={replay}")
            totals, pvs = ctx.count_graphs(hs, per_vertex=True, workspace=ws, replay=replay)
            check(graphs, totals, pvs)


def test_count_graphs_rejects(ctx, torch):
    from paper_2103_08053_amd import Context, Params, TCError
    g = gg.complete(10)
    h = ctx.build(g.src, g.dst, g.n)
    c2 = Context(0, Params(slots_per_bucket=2))
    h2 = c2.build(g.src, g.dst, g.n)
    with pytest.raises(TCError):  # built with other parameters
        ctx.count_graphs([h, h2])
    small = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(TCError):  # workspace too small
        ctx.count_graphs([h], workspace=small)
    no_pv = torch.empty(ctx.count_graphs_bytes(1, g.n, g.m_in, per_vertex=False), dtype=torch.uint8, device="cuda:0")
    assert ctx.count_graphs([h], workspace=no_pv)[0] == [120]
    with pytest.raises(TCError):  # no room for the per-vertex staging
        ctx.count_graphs([h], per_vertex=True, workspace=no_pv)
    c3 = Context(0, Params(flags=0x200))
    h3 = c3.build(g.src, g.dst, g.n)
    with pytest.raises(TCError):  # subwave modes are single-graph only
        c3.count_graphs([h3])
    assert ctx.count_graphs([h])[0] == [120]
