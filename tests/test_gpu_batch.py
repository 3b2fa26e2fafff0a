"""Batches of graphs in one build and one count launch, and HIP-graph replay.

Each graph's total (and per-vertex counts) must equal the oracle's on that
graph alone, bit for bit, whatever else shares the batch.
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
def ctx():
    import torch  # noqa: F401
    from paper_2103_08053_amd import Context
    return Context(0)


def mixed_graphs():
    gs = [gg.complete(30), gg.wheel(50), gg.EdgeList(0, np.zeros(0, np.uint32), np.zeros(0, np.uint32), "empty0"),
          gg.friendship(20), gg.EdgeList(7, np.zeros(0, np.uint32), np.zeros(0, np.uint32), "iso7"),
          gg.torus3d(6), gg.complete_tripartite(4, 5, 6), gg.dirty(gg.rmat(11, 16, seed=2), seed=3)]
    for s in range(12):
        rng = np.random.default_rng(100 + s)
        n = int(rng.integers(2, 2000))
        gs.append(gg.dirty(gg.erdos_renyi(n, int(rng.integers(1, 12 * n)), seed=s), seed=s))
        gs.append(gg.barabasi_albert(int(rng.integers(10, 3000)), int(rng.integers(2, 12)), seed=s))
    return gs


def check_batch(ctx, graphs, per_vertex=True, replay=False):
    from paper_2103_08053_amd import Batch
    say(f"[gpu] batch of {len(graphs)} graphs, params={ctx.params}, replay={replay}")
    b = Batch(ctx, [(g.n, g.src, g.dst) for g in graphs])
    totals, pv = b.count(per_vertex=per_vertex, replay=replay)
    totals = totals if isinstance(totals, list) else [totals]
    pvn = pv.cpu().numpy().astype(np.uint64) if per_vertex else None
    for i, g in enumerate(graphs):
        r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
        assert totals[i] == r.total, (i, g.name, totals[i], r.total)
        if per_vertex:
            assert (pvn[b.voff[i]:b.voff[i + 1]] == r.per_vertex).all(), (i, g.name)
    return b, totals


def test_mixed_batch(ctx):
    check_batch(ctx, mixed_graphs())


def test_single_graph_batch(ctx):
    g = gg.rmat(12, 16, seed=9)
    _, totals = check_batch(ctx, [g])
    assert totals[0] == ctx.count(g.src, g.dst, g.n)[0]


@pytest.mark.parametrize("kw", [dict(flags=2), dict(flags=4), dict(flags=32), dict(wg_lds_bytes=4096, wg_waves=2),
                                dict(slots_per_bucket=1, load_factor_pct=100), dict(hash_kind=1),
                                dict(flags=0x40), dict(flags=0x80), dict(flags=0x200), dict(flags=0x4000),
                                dict(flags=0x4000 | 4)],
                         ids=["wg", "hub", "big", "tinylds", "s1full", "hash1", "order_in", "order_collective",
                              "subwave16", "records", "records_hub"])
def test_batch_forced_paths(kw):
    from paper_2103_08053_amd import Context, Params
    check_batch(Context(0, Params(**kw)), mixed_graphs()[:14])


def test_batch_workload_sample(ctx):
    """The small-graph batch recipe (even index ER, odd index BA), first 256 graphs,
    sizes capped at 5000 vertices to keep the oracle quick."""
    specs = W.batch_spec(256, seed=1, n_hi=5000)
    graphs = [W.batch_graph(sp) for sp in specs]
    check_batch(ctx, graphs, per_vertex=False)


def test_batch_range_error(ctx):
    from paper_2103_08053_amd import Batch, RangeError
    good = gg.complete(5)
    bad = gg.EdgeList(4, np.array([0, 1, 4], np.uint32), np.array([1, 2, 0], np.uint32), "bad")  # 4 >= n_g
    with pytest.raises(RangeError):
        Batch(ctx, [(good.n, good.src, good.dst), (bad.n, bad.src, bad.dst)])


def test_replay_matches_eager_each_time(ctx):
    """Capture once, replay several times with other eager work and
    synchronisations in between; every replay equals the eager result."""
    import torch
    from paper_2103_08053_amd import Batch
    graphs = mixed_graphs()
    b = Batch(ctx, [(g.n, g.src, g.dst) for g in graphs])
    pv = torch.empty(b.n, dtype=torch.int64, device="cuda:0")
    b.count_async(pv)
    eager_tot = b.totals_dev.clone()
    eager_pv = pv.clone()
    other = gg.rmat(12, 16, seed=4)
    other_tot = ctx.count(other.src, other.dst, other.n)[0]
    for i in range(6):
        b.totals_dev.fill_(-1)
        pv.fill_(-1)
        b.count_async(pv, replay=True)
        torch.cuda.synchronize()
        assert torch.equal(b.totals_dev, eager_tot), i
        assert torch.equal(pv, eager_pv), i
        # eager work between replays
        assert ctx.count(other.src, other.dst, other.n)[0] == other_tot
        torch.cuda.synchronize()


def test_replay_single_graph(ctx):
    import torch
    g = W.small_rmat()
    graph = ctx.build(g.src, g.dst, g.n)
    t0, _ = graph.count()
    for _ in range(4):
        graph.totals_dev.zero_()
        graph.count_async(replay=True)
        torch.cuda.synchronize()
        assert int(graph.totals_dev[0]) == t0
