"""Parity of the HIP path against the CPU oracle (bit-exact integer counts).

Every test calls the C-ABI library through its binding.  The expected side is
the oracle (run here, or stored in golden/expected_counts.json by
golden/make_expected.py, which calls only the oracle) or a closed form.
"""
import json
import os
import sys
from math import comb

import numpy as np
import pytest

import graphgen as gg
import graphgen.workloads as W
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "expected_counts.json")


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


def gpu_count(ctx, g, per_vertex=True):
    say(f"[gpu] {g.name} n={g.n} m_in={g.m_in} params={ctx.params}")
    tot, pv = ctx.count(g.src, g.dst, g.n, per_vertex=per_vertex)
    return tot, (pv.cpu().numpy().astype(np.uint64) if per_vertex else None)


def assert_parity(ctx, g, expect=None):
    tot, pv = gpu_count(ctx, g)
    r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
    assert tot == r.total, (g.name, tot, r.total)
    assert (pv == r.per_vertex).all(), g.name
    if expect is not None:
        assert tot == expect
    return tot, pv


# ----------------------------------------------------------------------------- closed forms

CLOSED = [
    (gg.complete(3), 1), (gg.complete(4), 4), (gg.complete(50), comb(50, 3)), (gg.complete(300), comb(300, 3)),
    (gg.complete_bipartite(20, 30), 0), (gg.wheel(5), 4), (gg.wheel(1000), 999),
    (gg.complete_tripartite(7, 9, 11), 7 * 9 * 11), (gg.complete_tripartite(1, 1, 600), 600),
    (gg.cocktail_party(40), comb(80, 3) - 40 * 78), (gg.friendship(500), 500),
    (gg.cycle(3), 1), (gg.cycle(1000), 0), (gg.star(5000), 0), (gg.random_tree(3000, seed=2), 0),
    (gg.torus3d(12), 0),
]


@pytest.mark.parametrize("g,expect", CLOSED, ids=[g.name for g, _ in CLOSED])
def test_closed_forms(ctx, g, expect):
    assert_parity(ctx, g, expect)


def test_disjoint_union(ctx):
    parts = [gg.complete(40), gg.wheel(77), gg.friendship(9), gg.torus3d(5), gg.complete_tripartite(3, 4, 5)]
    g = gg.disjoint_union(parts)
    assert_parity(ctx, g, comb(40, 3) + 76 + 9 + 0 + 60)


# ----------------------------------------------------------------------------- random and dirty inputs

@pytest.mark.parametrize("seed", range(24))
def test_random_dirty_graphs(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 3000))
    m = int(rng.integers(1, 20 * n))
    g = gg.dirty(gg.erdos_renyi(n, m, seed=seed), seed=seed)
    assert_parity(ctx, g)


@pytest.mark.parametrize("k", [4, 9, 16])
def test_barabasi_albert(ctx, k):
    assert_parity(ctx, gg.barabasi_albert(20000, k, seed=k))


def test_rmat_scale16_against_stored(ctx):
    exp = json.load(open(GOLDEN))["rmat16"]
    g = W.small_rmat()
    tot, pv = assert_parity(ctx, g, exp["total"])
    ids = np.array(exp["sample_ids"])
    assert (pv[ids] == np.array(exp["sample_counts"], dtype=np.uint64)).all()


# ----------------------------------------------------------------------------- every code path, same answer

FORCED = [
    dict(flags=2),                              # every vertex in the workgroup bin
    dict(flags=4),                              # every vertex in the global-memory table bin
    dict(flags=32),                             # every vertex in the large-LDS bin
    dict(flags=0x40), dict(flags=0x80),         # hash ids in in-degree / collective-degree order
    dict(flags=0x80 | 4, slots_per_bucket=1, load_factor_pct=100),
    dict(flags=0x100), dict(flags=0x200), dict(flags=0x400), dict(flags=0x800),   # subwave / per-wave lists
    dict(flags=0x100 | 4), dict(flags=0x200 | 32), dict(flags=0x400 | 2, slots_per_bucket=1, load_factor_pct=100),
    dict(wg_lds_bytes=4096, wg_waves=2),        # tiny LDS: most vertices spill to the global-table bin
    dict(wg_lds_bytes=4096, wg_waves=2, flags=0x2000),   # ... with every large-LDS vertex in the full launch
    dict(slots_per_bucket=1), dict(slots_per_bucket=4),
    dict(load_factor_pct=100), dict(load_factor_pct=10),
    dict(slots_per_bucket=1, load_factor_pct=100, flags=2),   # long probe chains in LDS
    dict(slots_per_bucket=1, load_factor_pct=100, flags=4),   # long probe chains in global memory
    dict(hash_kind=1), dict(light_chunk=1), dict(light_chunk=7), dict(flags=1), dict(flags=8),
    dict(wg_waves=1), dict(wg_waves=4), dict(wg_waves=16, wg_lds_bytes=131072),
    dict(grid_wgs=3), dict(grid_wgs=1, flags=4), dict(grid_wgs=2, flags=32), dict(wave_max_dplus=8),
    dict(flags=16), dict(flags=16 | 2, slots_per_bucket=1, load_factor_pct=100),   # 64-bit list addressing
    # the record layout, through every bin and probe variant
    dict(flags=0x4000), dict(flags=0x4000 | 2), dict(flags=0x4000 | 4), dict(flags=0x4000 | 32),
    dict(flags=0x4000, wg_lds_bytes=4096, wg_waves=2), dict(flags=0x4000 | 0x1000), dict(flags=0x4000 | 0x100),
    dict(flags=0x4000 | 0x800), dict(flags=0x4000 | 16), dict(flags=0x4000, hash_kind=1),
    dict(flags=0x4000 | 1, slots_per_bucket=1, load_factor_pct=100), dict(flags=0x4000 | 0x40),
]


@pytest.fixture(scope="module")
def forced_graphs():
    return [gg.dirty(gg.rmat(13, 16, seed=3), seed=1), gg.barabasi_albert(5000, 12, seed=5),
            gg.complete(200)]


@pytest.mark.parametrize("kw", FORCED, ids=[str(k) for k in FORCED])
def test_forced_paths_agree(torch, forced_graphs, kw):
    from paper_2103_08053_amd import Context, Params
    c = Context(0, Params(**kw))
    for g in forced_graphs:
        assert_parity(c, g)


def test_bins_are_exercised(torch):
    """A low wavefront cap routes a skewed graph through both LDS bins; the
    tiny-LDS parameters route its largest vertices to the large-LDS bin (the
    global-table bin is reached through TC_F_FORCE_HUB in the forced-path
    cases: no graph the oracle counts quickly has an out-degree beyond the
    large-LDS limit)."""
    from paper_2103_08053_amd import Context, Params
    g = gg.rmat(14, 16, seed=1)
    info = Context(0, Params(wave_max_dplus=32)).build(g.src, g.dst, g.n).info()
    assert info.n_wg > 0 and info.n_wave > 0 and info.n_hub == 0 and info.n_big == 0
    assert info.big_cap > info.wg_cap
    c = Context(0, Params(wg_lds_bytes=4096, wg_waves=2))
    small = c.build(g.src, g.dst, g.n).info()
    assert small.n_big > 0 and small.n_hub == 0
    assert 0 < small.n_mid <= small.n_big and small.wg_cap < small.mid_cap < small.big_cap
    assert_parity(c, g)


@pytest.mark.parametrize("flags", [0, 4], ids=["default", "global_tables"])
def test_scratch_at_unaligned_offsets(torch, flags):
    """The library uses a caller's count scratch from its first 64 KB boundary: scratch buffers of
    exactly the queried size starting at any offset (filled with garbage first) give the oracle's
    counts, through the LDS bins and through the global-memory tables that live in the scratch."""
    from paper_2103_08053_amd import Context, Params
    g = gg.dirty(gg.rmat(13, 16, seed=5), seed=4)
    r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
    c = Context(0, Params(flags=flags))
    graph = c.build(g.src, g.dst, g.n)
    need = c.scratch_bytes(g.n, graph.m_in)
    for off in (0, 256, 4096, 65536 - 256, 65536 + 512, 3 * 65536 + 768):
        buf = torch.full((need + off,), 0xA5, dtype=torch.uint8, device="cuda:0")
        graph.scratch = buf[off:off + need]
        say(f"[gpu] scratch offset {off} flags {flags:#x}")
        tot, pv = graph.count(per_vertex=True)
        assert tot == r.total, off
        assert (pv.cpu().numpy().astype(np.uint64) == r.per_vertex).all(), off


def test_record_layout_flag(torch):
    """TC_F_RECORDS gives the graph its records unless a relabelling or the counting-sort build is asked
    for; the counts agree either way (the element-wise oracle checks are the forced-path cases)."""
    from paper_2103_08053_amd import Context, Params
    g = gg.dirty(gg.rmat(12, 16, seed=8), seed=2)
    res = {}
    for flags, want in ((0, 0), (0x4000, 1), (0x4000 | 0x40, 0), (0x4000 | 0x8, 0)):
        graph = Context(0, Params(flags=flags)).build(g.src, g.dst, g.n)
        assert graph.info().records == want, flags
        tot, pv = graph.count(per_vertex=True)
        res[flags] = (tot, pv.cpu().numpy())
    for flags in res:
        assert res[flags][0] == res[0][0] and (res[flags][1] == res[0][1]).all(), flags
    # sizes: the records take at most R = 2 m_in + n + 32 (ceil(n / 64) + 1) words (line-aligned
    # placement) and their placement 8 (n + 1) bytes of storage, each rounded up to the alignment;
    # the build's placement temporaries 16 (ceil(n / 64) + 1) bytes; the per-vertex staging grows from
    # n to R 8-byte words; where the flag is ignored it changes nothing
    n, m_in = g.n, g.m_in
    chunks = (n + 63) // 64
    words = 2 * m_in + n + 32 * (chunks + 1)
    base = Context(0, Params())
    rec = Context(0, Params(flags=0x4000))
    (s0, t0), (s1, t1) = base.footprint(n, m_in), rec.footprint(n, m_in)
    assert 4 * words + 8 * (n + 1) <= s1 - s0 < 4 * words + 8 * (n + 1) + 1024
    assert 16 * (chunks + 1) <= t1 - t0 < 16 * (chunks + 1) + 512
    for other in (0x40, 0x8):
        a, b = Context(0, Params(flags=other)), Context(0, Params(flags=other | 0x4000))
        assert a.footprint(n, m_in) == b.footprint(n, m_in), other
        assert a.scratch_bytes(n, m_in) == b.scratch_bytes(n, m_in), other
    c0, c1 = base.scratch_bytes(n, m_in), rec.scratch_bytes(n, m_in)
    assert abs((c1 - c0) - 8 * (words - n)) < 512


def test_record_placement_near_line_size(torch):
    """Record layout where records are about a 128-byte line long (mean out-degree near 32, so many
    records of up to 32 words would straddle a line and are moved to the next one, and the longer
    ones are not), with vertex counts that leave a partial chunk of 64 ranks, and a near-complete
    graph whose records take every length from 1 to 65 words: every count equals the oracle's."""
    from paper_2103_08053_amd import Context, Params
    c = Context(0, Params(flags=0x4000))
    graphs = [gg.erdos_renyi(n, n * deg // 2, seed=seed) for n, deg, seed in ((64 * 37 + 7, 64, 1), (1000, 70, 2))]
    for g in graphs + [gg.complete(65)]:
        graph = c.build(g.src, g.dst, g.n)
        assert graph.info().records == 1
        assert_parity(c, g)


def test_half_lds_launch(torch):
    """Large-LDS-bin vertices in both launches: K_2500 has out-degrees 0..2499 in rank order, so
    those above the half-LDS limit (about 2000) take the full-LDS launch and those between the
    workgroup limit and it the half-LDS one; every count is the closed form, with and without the
    split, and the split changes no count."""
    from paper_2103_08053_amd import Context, Params
    n = 2500
    g = gg.complete(n)
    res = {}
    for flags in (0, 0x2000):
        c = Context(0, Params(flags=flags))
        graph = c.build(g.src, g.dst, g.n)
        info = graph.info()
        say(f"[gpu] K_{n} flags={flags:#x} n_big={info.n_big} n_mid={info.n_mid} mid_cap={info.mid_cap}")
        tot, pv = graph.count(per_vertex=True)
        pv = pv.cpu().numpy().astype(np.uint64)
        assert tot == comb(n, 3)
        assert (pv == comb(n - 1, 2)).all()
        res[flags] = info
    on, off = res[0], res[0x2000]
    assert on.wg_cap < on.mid_cap < on.big_cap and off.mid_cap == 0 and off.n_mid == 0
    assert on.n_big == off.n_big and 0 < on.n_mid < on.n_big
    assert on.n_big - on.n_mid == sum(1 for d in range(n) if d > on.mid_cap)


# ----------------------------------------------------------------------------- edge cases

def test_empty_inputs(ctx, torch):
    e = np.zeros(0, np.uint32)
    assert ctx.count(e, e, 0)[0] == 0
    tot, pv = ctx.count(e, e, 10, per_vertex=True)
    assert tot == 0 and int(pv.abs().sum()) == 0
    loops = np.arange(100, dtype=np.uint32)
    tot, pv = ctx.count(loops, loops, 100, per_vertex=True)
    assert tot == 0 and int(pv.abs().sum()) == 0
    tot, pv = ctx.count(np.array([0], np.uint32), np.array([1], np.uint32), 2, per_vertex=True)
    assert tot == 0


def test_large_id_space(ctx):
    """Ids near the top of a 2^27 + 5 id space (28-bit ids, 56-bit sort keys)."""
    n = 2**27 + 5
    a = np.array([n - 1, n - 2, n - 3, 0, n - 1], np.uint32)
    b = np.array([n - 2, n - 3, n - 1, n - 1, 0], np.uint32)
    tot, pv = ctx.count(a, b, n, per_vertex=True)
    assert tot == 1
    pv = pv.cpu().numpy()
    assert pv[n - 1] == 1 and pv[n - 2] == 1 and pv[n - 3] == 1 and pv[0] == 0 and int(pv.sum()) == 3


def test_out_of_range_ids_rejected(ctx):
    from paper_2103_08053_amd import RangeError
    with pytest.raises(RangeError):
        ctx.count(np.array([0, 1, 5], np.uint32), np.array([1, 2, 0], np.uint32), 5)
    # the context stays usable
    assert ctx.count(np.array([0, 1, 2], np.uint32), np.array([1, 2, 0], np.uint32), 3)[0] == 1


def test_unsupported_size(ctx):
    from paper_2103_08053_amd import TCError
    with pytest.raises(TCError):
        ctx.workspace_bytes(100, 2**31)


def test_deterministic_repeats(ctx):
    g = W.small_rmat()
    graph = ctx.build(g.src, g.dst, g.n)
    t0, p0 = graph.count(per_vertex=True)
    for _ in range(20):
        t, p = graph.count(per_vertex=True)
        assert t == t0
        assert bool((p == p0).all())
    assert graph.count(per_vertex=False)[0] == t0


def test_graph_info_matches_oracle(ctx):
    g = gg.dirty(gg.rmat(14, 16, seed=4), seed=2)
    info = ctx.build(g.src, g.dst, g.n).info()
    r = oracle.count(g.n, g.src, g.dst)
    assert (info.m, info.wedges_plus, info.max_dplus) == (r.m, r.wedges_plus, r.max_dplus)


# ----------------------------------------------------------------------------- full-size workload

def check_full_size(ctx, name, gen, one_shot=True, live=False):
    """Total, a checksum of the whole per-vertex array and sampled per-vertex
    counts against values stored by the oracle, plus sum t(x) = 3T.  With
    `live` the oracle also runs here and the whole per-vertex array is
    compared element by element."""
    data = json.load(open(GOLDEN))
    if name not in data:
        pytest.skip(f"no stored oracle values for {name} (tests/golden/make_expected.py)")
    exp = data[name]
    g = gen()
    say(f"[gpu] {name} n={g.n} m_in={g.m_in}")
    assert (g.n, g.m_in) == (exp["n"], exp["m_in"])
    graph = ctx.build(g.src, g.dst, g.n)
    info = graph.info()
    assert (info.m, info.wedges_plus, info.max_dplus) == (exp["m"], exp["wedges_plus"], exp["max_dplus"])
    tot, pv = graph.count(per_vertex=True)
    assert tot == exp["total"]
    pvn = pv.cpu().numpy().astype(np.uint64)
    x = np.arange(g.n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        chk = int(np.sum(pvn * (x * np.uint64(0x9E3779B97F4A7C15) + np.uint64(1)), dtype=np.uint64))
    assert chk == exp["per_vertex_checksum"]
    ids = np.array(exp["sample_ids"])
    assert (pvn[ids] == np.array(exp["sample_counts"], dtype=np.uint64)).all()
    assert int(pvn.sum()) == 3 * tot
    if live:
        say(f"[gpu] {name}: oracle per-vertex run")
        r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
        say(f"[gpu] {name}: oracle took {r.t_clean_s + r.t_count_s:.1f} s on {r.threads} threads")
        assert r.total == tot
        bad = np.flatnonzero(pvn != r.per_vertex)
        assert bad.size == 0, (bad[:10], pvn[bad[:10]], r.per_vertex[bad[:10]])
    graph.release()
    del graph, pv
    if one_shot:  # the one-shot entry point the benchmark times agrees
        assert ctx.count(g.src, g.dst, g.n)[0] == exp["total"]


def test_rmat_scale22_full_size(ctx, torch):
    """The throughput workload (R-MAT scale 22), in the launch configuration the benchmark times;
    every vertex's count against a live oracle run."""
    check_full_size(ctx, "rmat22", W.large_rmat, live=True)


def test_er_2pow25_full_size(ctx, torch):
    """Erdos-Renyi, 2^25 vertices, mean degree 32: every vertex in the wavefront bin."""
    check_full_size(ctx, "er25", W.uniform_er)


def test_rmat_scale26_full_size(ctx, torch):
    """R-MAT scale 26 (about 1.05e9 edges): col past 4 GiB, so the count takes
    the 64-bit addressing variant; skewed hubs."""
    check_full_size(ctx, "rmat26", W.huge_rmat, one_shot=False)


# ----------------------------------------------------------------------------- workload partitioning

def owned_counts(g):
    """Triangles per table owner u (the (degree, id)-lowest vertex of the triangle), from the oracle's
    oriented lists: sum over v in N+(u) of |N+(u) & N+(v)|; and each vertex's rank in (degree, id) order."""
    deg, dplus, nbr = oracle.oriented(g.n, g.src, g.dst)
    off = np.concatenate([[0], np.cumsum(dplus.astype(np.int64))])
    lists = [set(nbr[off[u]:off[u + 1]].tolist()) for u in range(g.n)]
    own = np.array([sum(len(lists[u] & lists[v]) for v in lists[u]) for u in range(g.n)], np.int64)
    order = np.lexsort((np.arange(g.n), deg))  # by degree, then id
    rank = np.empty(g.n, np.int64)
    rank[order] = np.arange(g.n)
    return own, rank


@pytest.mark.parametrize("shards", [2, 3, 8])
def test_shards_sum_to_whole(ctx, torch, shards):
    """Workload partitions (table owner's rank mod shards) add up to the whole count, total and per
    vertex, and each shard's total is the number of triangles whose lowest-rank vertex is in it."""
    g = gg.dirty(gg.rmat(12, 16, seed=5), seed=6)
    r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
    own, rank = owned_counts(g)
    assert own.sum() == r.total
    graph = ctx.build(g.src, g.dst, g.n)
    tot, pv = 0, np.zeros(g.n, np.uint64)
    parts = []
    for s in range(shards):
        t, p = graph.count(per_vertex=True, shard=(s, shards))
        assert t == int(own[rank % shards == s].sum()), s
        parts.append(t)
        tot += t
        pv += p.cpu().numpy().astype(np.uint64)
    assert tot == r.total
    assert (pv == r.per_vertex).all()
    if shards == 8:
        # rank order spreads the work: no shard holds more than twice its even share
        assert max(parts) <= 2 * r.total / shards


def test_shards_batch_and_forced_paths(torch):
    from paper_2103_08053_amd import Batch, Context, Params
    gs = [gg.complete(40), gg.wheel(60), gg.dirty(gg.rmat(11, 16, seed=2), seed=3), gg.friendship(30)]
    for kw in (dict(), dict(flags=4), dict(flags=32), dict(wg_lds_bytes=4096, wg_waves=2)):
        c = Context(0, Params(**kw))
        b = Batch(c, [(g.n, g.src, g.dst) for g in gs])
        whole = b.count()[0]
        acc = [0] * len(gs)
        for s in range(4):
            part = b.count(shard=(s, 4))[0]
            acc = [x + y for x, y in zip(acc, part)]
        assert acc == whole == [oracle.count(g.n, g.src, g.dst).total for g in gs], kw


def test_shard_arguments_checked(ctx, torch):
    from paper_2103_08053_amd import TCError
    g = gg.complete(10)
    graph = ctx.build(g.src, g.dst, g.n)
    for bad in ((0, 0), (3, 3), (5, 2)):
        with pytest.raises(TCError):
            graph.count(shard=bad)


# ----------------------------------------------------------------------------- collision statistics

def test_collision_stats_complete_graph(ctx, torch):
    """K_100: N+(u) is a run of d+ consecutive ranks.  With default knobs and no packed bin every
    table (d+ < 100) is a wavefront table with a filter, which keeps the load-factor bucket count:
    B = the power of two >= d+/2, so B < d+ <= 2B and d+ consecutive ids under the low-bits hash put
    exactly two out-neighbours in some home bucket and never three: max collision 2 everywhere and
    phi (Equation 2) = 2 W+."""
    from paper_2103_08053_amd import Context, Params
    g = gg.complete(100)
    for flags, mc in ((0x1000, 2),):
        graph = Context(0, Params(flags=flags)).build(g.src, g.dst, g.n)
        info = graph.info()
        assert info.n_wave == g.n - 2
        for pv in (True, False):
            st = graph.collisions(per_vertex=pv)
            assert st["tables"] == g.n - 2 == info.n_wave + info.n_wg + info.n_big + info.n_hub + info.n_packed
            assert st["max_collision"] == mc and st["sum_max_collision"] == mc * st["tables"], (flags, pv, st)
            assert st["phi"] == mc * info.wedges_plus


def test_collision_stats_bounds(torch):
    """On a skewed graph: 1 <= max collision(u), so phi >= W+ of the tabled vertices and the sum of
    maxima >= tables; a full one-slot table at 100% load cannot collide less than a 10% one."""
    from paper_2103_08053_amd import Context, Params
    g = gg.dirty(gg.rmat(13, 16, seed=7), seed=8)
    lo = Context(0, Params(load_factor_pct=10, slots_per_bucket=1, wave_max_dplus=0)).build(g.src, g.dst, g.n)
    hi = Context(0, Params(load_factor_pct=100, slots_per_bucket=1)).build(g.src, g.dst, g.n)
    a, b = lo.collisions(), hi.collisions()
    for st, gr in ((a, lo), (b, hi)):
        info = gr.info()
        assert st["tables"] == info.n_wave + info.n_wg + info.n_big + info.n_hub + info.n_packed
        assert st["sum_max_collision"] >= st["tables"] and st["max_collision"] >= 1
        assert st["phi"] >= st["sum_max_collision"]
    assert b["sum_max_collision"] >= a["sum_max_collision"]
    for order in (0x40, 0x80):  # other vertex orders: same tables, same counts
        c = Context(0, Params(flags=order))
        gr = c.build(g.src, g.dst, g.n)
        assert gr.collisions()["tables"] == a["tables"]
        assert gr.count()[0] == oracle.count(g.n, g.src, g.dst).total


# ----------------------------------------------------------------------------- Section 3.3 designs

SIMPLE_CASES = [gg.complete(60), gg.wheel(300), gg.complete_tripartite(5, 6, 7), gg.friendship(40),
                gg.torus3d(6), gg.dirty(gg.rmat(12, 16, seed=11), seed=12), gg.barabasi_albert(3000, 8, seed=4)]


@pytest.mark.parametrize("g", SIMPLE_CASES, ids=[g.name for g in SIMPLE_CASES])
def test_plain_vertex_and_edge_centric_designs(ctx, torch, g):
    """Algorithm 1 without the optimisations and Algorithm 2 (one table per edge) count exactly;
    table construction alone counts nothing."""
    graph = ctx.build(g.src, g.dst, g.n)
    want = oracle.count(g.n, g.src, g.dst).total
    assert graph.count_simple(edge_centric=False) == want
    assert graph.count_simple(edge_centric=True) == want
    assert graph.count_simple(edge_centric=True, build_only=True) == 0
    assert graph.count_simple(edge_centric=False, build_only=True) == 0


def test_plain_designs_reject_what_they_cannot_hold(torch):
    from paper_2103_08053_amd import Batch, Context, Params, TCError
    c = Context(0, Params(wg_lds_bytes=4096, wg_waves=2))
    g = gg.complete(9000)  # d+ up to 8999: beyond any LDS table
    graph = c.build(g.src, g.dst, g.n)
    with pytest.raises(TCError):
        graph.count_simple()
    b = Batch(c, [(5, gg.complete(5).src, gg.complete(5).dst)] * 2)
    with pytest.raises(TCError):
        b.count_simple()


# ----------------------------------------------------------------------------- packed light vertices

def test_packed_light_vertices_match_unpacked(torch):
    """Runs of light vertices share a wavefront (4 x 16 or 2 x 32 lanes); the counts equal the
    one-vertex-per-wavefront path and the oracle, per vertex too, also in batches and shards."""
    from paper_2103_08053_amd import Batch, Context, Params
    gs = [gg.dirty(gg.erdos_renyi(5000, 40000, seed=3), seed=4), gg.erdos_renyi(20000, 320000, seed=5),
          gg.barabasi_albert(4000, 6, seed=6), gg.complete(20), gg.cycle(50), gg.torus3d(7)]
    for kw in (dict(), dict(flags=0x1000), dict(load_factor_pct=10), dict(slots_per_bucket=1, load_factor_pct=100),
               dict(wg_lds_bytes=8192, wg_waves=4), dict(hash_kind=1), dict(flags=0x40)):
        c = Context(0, Params(**kw))
        if not kw:
            info = c.build(gs[1].src, gs[1].dst, gs[1].n).info()
            assert info.n_packed > 0
        for g in gs:
            assert_parity(c, g)
        b = Batch(c, [(g.n, g.src, g.dst) for g in gs])
        assert b.count()[0] == [oracle.count(g.n, g.src, g.dst).total for g in gs], kw
    g = gs[1]
    graph = Context(0).build(g.src, g.dst, g.n)
    assert sum(graph.count(shard=(s, 3))[0] for s in range(3)) == oracle.count(g.n, g.src, g.dst).total


def test_bin_work_sums_to_wedges(ctx, torch):
    """Work per bin adds up to W+ (the oracle's 2-hop probe count), with work in every used bin."""
    from paper_2103_08053_amd import Context, Params
    g = gg.dirty(gg.rmat(14, 16, seed=9), seed=10)
    r = oracle.count(g.n, g.src, g.dst)
    for kw in (dict(), dict(wave_max_dplus=32), dict(wg_lds_bytes=4096, wg_waves=2), dict(flags=4)):
        graph = Context(0, Params(**kw)).build(g.src, g.dst, g.n)
        info, work = graph.info(), graph.bin_work()
        assert sum(work) == r.wedges_plus == info.wedges_plus, kw
        counts = [info.n_hub, info.n_big, info.n_wg, info.n_wave, info.n_packed]
        for b in range(5):
            assert (work[b] > 0) == (counts[b] > 0), (kw, b, work, counts)
