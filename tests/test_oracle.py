"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: closed forms of
graph families, a dense matrix brute force, two independent library
routines, the paper's own 3-D grid row, and invariances that any correct
triangle count has.  Each family is chosen so that a plausible slip in the
oracle (a dropped per-vertex term, a missing dedup or self-loop filter, an
orientation that keeps both directions, a swapped operand in the merge) breaks
at least one test.
"""
from math import comb

import numpy as np
import pytest

import graphgen as gg
import oracle


def run(g, pv=True):
    return oracle.count(g.n, g.src, g.dst, per_vertex=pv)


# ----------------------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 8, 17, 40])
def test_complete(n):
    g = gg.complete(n) if n >= 2 else gg.EdgeList(n, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    r = run(g)
    assert r.total == comb(n, 3)
    assert (r.per_vertex == (comb(n - 1, 2) if n else 0)).all()
    assert r.m == comb(n, 2)


@pytest.mark.parametrize("a,b", [(1, 1), (3, 4), (10, 25)])
def test_complete_bipartite(a, b):
    r = run(gg.complete_bipartite(a, b))
    assert r.total == 0 and not r.per_vertex.any()


@pytest.mark.parametrize("n", [5, 6, 9, 50])
def test_wheel(n):
    r = run(gg.wheel(n))
    assert r.total == n - 1
    assert r.per_vertex[0] == n - 1
    assert (r.per_vertex[1:] == 2).all()


def test_wheel4_is_k4():
    assert run(gg.wheel(4)).total == 4


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 3, 4), (5, 1, 7)])
def test_complete_tripartite(a, b, c):
    r = run(gg.complete_tripartite(a, b, c))
    assert r.total == a * b * c
    pv = r.per_vertex
    assert (pv[:a] == b * c).all() and (pv[a:a + b] == a * c).all() and (pv[a + b:] == a * b).all()


@pytest.mark.parametrize("k", [2, 3, 6])
def test_cocktail_party(k):
    r = run(gg.cocktail_party(k))
    assert r.total == comb(2 * k, 3) - k * (2 * k - 2)
    assert (r.per_vertex == comb(2 * k - 2, 2) - (k - 1)).all()


@pytest.mark.parametrize("k", [1, 4, 30])
def test_friendship(k):
    r = run(gg.friendship(k))
    assert r.total == k
    assert r.per_vertex[0] == k and (r.per_vertex[1:] == 1).all()


@pytest.mark.parametrize("n,t", [(3, 1), (4, 0), (11, 0)])
def test_cycle(n, t):
    assert run(gg.cycle(n)).total == t


def test_trees_and_stars():
    assert run(gg.star(100)).total == 0
    assert run(gg.random_tree(500, seed=3)).total == 0


def test_paper_3d_grid_row():
    """Table 2's 3-D grid: |V| = 464^3, |E| = 3|V|, 0 triangles.  The same
    torus structure at small sides gives the same edge ratio and count."""
    rows = {}
    for line in open(__file__.replace("test_oracle.py", "golden/paper_table2_3dgrid.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            rows[k] = int(v)
    assert rows["V"] == 464 ** 3 and rows["E"] == 3 * rows["V"] and rows["triangles"] == 0
    for side in (4, 5, 9):
        r = run(gg.torus3d(side))
        assert r.m == 3 * side ** 3
        assert r.total == rows["triangles"]


def test_disjoint_union_adds():
    parts = [gg.complete(7), gg.wheel(8), gg.friendship(3), gg.complete_tripartite(2, 2, 3)]
    r = run(gg.disjoint_union(parts))
    rs = [run(p) for p in parts]
    assert r.total == sum(x.total for x in rs)
    assert (r.per_vertex == np.concatenate([x.per_vertex for x in rs])).all()


# ----------------------------------------------------------------------------- brute force

def _random_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    p = float(rng.random()) ** 2
    i, j = np.triu_indices(n, 1)
    keep = rng.random(i.shape[0]) < p
    g = gg.EdgeList(n, i[keep].astype(np.uint32), j[keep].astype(np.uint32), f"tiny{seed}")
    return gg.dirty(g, seed=seed, dup_frac=0.5, loops=3) if n > 0 else g


@pytest.mark.parametrize("seed", range(240))
def test_brute_force_dense(seed):
    g = _random_tiny(seed)
    T, diag = oracle.brute_force(g.n, g.src, g.dst)
    r = run(g)
    assert r.total == T
    assert (r.per_vertex == diag).all()
    assert int(r.per_vertex.sum()) == 3 * r.total


def test_vertex_counts_definition_matches_brute_force():
    for seed in range(30):
        g = _random_tiny(1000 + seed)
        if g.n == 0:
            continue
        _, diag = oracle.brute_force(g.n, g.src, g.dst)
        q = np.arange(g.n, dtype=np.uint32)
        assert (oracle.vertex_counts(g.n, g.src, g.dst, q) == diag).all()


# ----------------------------------------------------------------------------- library routines

def test_networkx_triangles_rmat12():
    nx = pytest.importorskip("networkx")
    g = gg.rmat(12, 16, seed=5)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(g.src, g.dst) if a != b)
    tri = nx.triangles(G)
    r = run(g)
    assert r.total == sum(tri.values()) // 3
    assert all(int(r.per_vertex[x]) == c for x, c in tri.items())


def test_scipy_sparse_rmat16():
    sp = pytest.importorskip("scipy.sparse")
    g = gg.rmat(16, 16, seed=1)
    s = g.src.astype(np.int64)
    d = g.dst.astype(np.int64)
    keep = s != d
    A = sp.coo_matrix((np.ones(keep.sum() * 2), (np.r_[s[keep], d[keep]], np.r_[d[keep], s[keep]])),
                      shape=(g.n, g.n)).tocsr()
    A.data[:] = 1.0  # duplicates summed by tocsr -> back to 0/1
    A.sum_duplicates()
    A.data[:] = 1.0
    A = A.astype(np.int64)
    B = (A @ A).multiply(A)
    per = np.asarray(B.sum(axis=1)).ravel() // 2
    r = run(g)
    assert r.total == int(B.sum()) // 6
    assert (r.per_vertex == per).all()


# ----------------------------------------------------------------------------- invariants

def test_relabel_shuffle_dirty_isolated():
    g = gg.rmat(13, 16, seed=2)
    base = run(g)
    h, p = gg.relabel(g, seed=9)
    r = run(h)
    assert r.total == base.total and r.m == base.m
    assert (r.per_vertex[p] == base.per_vertex).all()
    assert run(gg.shuffled(g, seed=4)).total == base.total
    rd = run(gg.dirty(g, seed=5))
    assert rd.total == base.total and (rd.per_vertex == base.per_vertex).all() and rd.m == base.m
    ri = run(gg.with_isolated(g, 1000))
    assert ri.total == base.total and not ri.per_vertex[g.n:].any()
    assert int(base.per_vertex.sum()) == 3 * base.total


def test_orientation_and_wedges_by_hand():
    """The oriented lists follow (degree, id) order, and W+ (the number of
    2-hop probes, the collective degree summed over all u) equals the number
    of oriented 2-paths x -> y -> z, counted here by explicit enumeration."""
    for seed in range(20):
        g = _random_tiny(500 + seed)
        if g.n == 0:
            continue
        deg, dplus, nbr = oracle.oriented(g.n, g.src, g.dst)
        edges = {(min(a, b), max(a, b)) for a, b in zip(g.src.tolist(), g.dst.tolist()) if a != b}
        d = np.zeros(g.n, np.int64)
        for a, b in edges:
            d[a] += 1; d[b] += 1
        assert (deg == d).all()
        out = {x: [] for x in range(g.n)}
        for a, b in edges:
            if (d[a], a) < (d[b], b):
                out[a].append(b)
            else:
                out[b].append(a)
        assert (dplus == np.array([len(out[x]) for x in range(g.n)])).all()
        assert nbr.tolist() == [y for x in range(g.n) for y in sorted(out[x])]
        paths = sum(1 for x in out for y in out[x] for _ in out[y])
        r = run(g, pv=False)
        assert r.wedges_plus == paths
        assert r.max_dplus == max([len(v) for v in out.values()] + [0])
        assert r.max_dplus ** 2 <= 2 * max(r.m, 0) + 1


def test_out_of_range_rejected():
    with pytest.raises(oracle.OracleRangeError):
        oracle.count(5, np.array([0, 5], np.uint32), np.array([1, 2], np.uint32))
    with pytest.raises(oracle.OracleRangeError):
        oracle.vertex_counts(5, np.array([0], np.uint32), np.array([1], np.uint32), np.array([7], np.uint32))


def test_stride_sample_counts_exactly_the_sampled_owners():
    """stride s counts only the vertices x with x % s == 0: its total is the number of triangles
    whose (degree, id)-first vertex x is such a vertex, enumerated here in Python from the oriented
    lists (sum over sampled x and y in N+(x) of |N+(x) & N+(y)|), and its work figures are those
    vertices' edges and 2-hop lengths.  An inverted or shifted filter fails this."""
    g = gg.dirty(gg.rmat(11, 16, seed=8), seed=9)
    deg, dplus, nbr = oracle.oriented(g.n, g.src, g.dst)
    off = np.concatenate([[0], np.cumsum(dplus.astype(np.int64))])
    lists = [set(nbr[off[x]:off[x + 1]].tolist()) for x in range(g.n)]
    owned = np.array([sum(len(lists[x] & lists[y]) for y in lists[x]) for x in range(g.n)], np.int64)
    full = run(g, pv=False)
    assert owned.sum() == full.total
    for s in (1, 2, 3, 7):
        sel = np.arange(g.n) % s == 0
        r = oracle.count(g.n, g.src, g.dst, stride=s)
        assert r.total == int(owned[sel].sum()), s
        assert r.counted_vertices == int(sel.sum())
        assert r.counted_edges == int(dplus[sel].sum())
        assert r.counted_wedges == sum(int(dplus[y]) for x in np.flatnonzero(sel) for y in lists[x])
        assert r.wedges_plus == full.wedges_plus  # W+ is always over the whole graph
    # the residues other than 0 are not counted: with s = 2 the odd owners' triangles are missing
    odd = int(owned[np.arange(g.n) % 2 == 1].sum())
    assert odd > 0 and oracle.count(g.n, g.src, g.dst, stride=2).total == full.total - odd


def test_erdos_renyi_expected_triangles():
    """Statistical sanity (not exact): G(n, M) with mean degree c has about
    c^3 / 6 triangles, independent of n.  c = 32 gives 5461 +- 74."""
    n = 1 << 16
    g = gg.erdos_renyi(n, 16 * n, seed=1)
    r = run(g, pv=False)
    c = 2 * r.m / n
    assert abs(r.total - c ** 3 / 6) < 5 * np.sqrt(c ** 3 / 6)
