"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle against a result the paper's definitions or
plain mathematics fix: brute-force enumeration on tiny graphs, the matrix
form of the common-neighbour counts (an independent library computation),
closed forms on complete bipartite graphs, a clamp-exercising closed form,
invariants (sums, level soundness, monotone peel order) and the wedge
count that bottom-up peeling must walk.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import synth


def C2(x):
    return x * (x - 1) // 2


def _tiny_graphs(count, seed0, max_u=8, max_v=8):
    out = []
    for s in range(count):
        rng = np.random.default_rng(1000 + seed0 + s)
        n_u = int(rng.integers(1, max_u + 1))
        n_v = int(rng.integers(1, max_v + 1))
        p = float(rng.choice([0.3, 0.5, 0.7, 0.9]))
        out.append(synth.random_small(n_u, n_v, p, seed=seed0 + s))
    return out


def _adj(g):
    a = np.zeros((g.n_u, g.n_v), dtype=np.int64)
    u, v = g.edges()
    a[u, v] = 1
    return a


# ---------------------------------------------------------------- counting


def test_count_vs_bruteforce_tiny():
    for g in _tiny_graphs(150, 0):
        bu, bv = oracle.count_vertex(g)
        ru, rv = brute.count_vertex(g)
        assert np.array_equal(bu, ru), g.name
        assert np.array_equal(bv, rv), g.name
        assert np.array_equal(oracle.count_edge(g), brute.count_edge(g)), g.name


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_count_vs_matrix_identity(seed):
    # support(u)   = sum_{u' != u} C((A A^T)_{uu'}, 2)
    # support(u,v) = (A A^T A)_{uv} - d_u - d_v + 1   (walks u-v'-u'-v minus the degenerate ones)
    g = synth.er(300, 200, 6000, seed=seed) if seed != 3 else synth.chung_lu(400, 150, 5000, 2.1, 150, seed=seed)
    a = _adj(g)
    uu = a @ a.T
    np.fill_diagonal(uu, 0)
    exp_u = (uu * (uu - 1) // 2).sum(axis=1)
    vv = a.T @ a
    np.fill_diagonal(vv, 0)
    exp_v = (vv * (vv - 1) // 2).sum(axis=1)
    bu, bv = oracle.count_vertex(g)
    assert np.array_equal(bu.astype(np.int64), exp_u)
    assert np.array_equal(bv.astype(np.int64), exp_v)
    aata = a @ a.T @ a
    u, v = g.edges()
    du = a.sum(axis=1)
    dv = a.sum(axis=0)
    exp_e = aata[u, v] - du[u] - dv[v] + 1
    assert np.array_equal(oracle.count_edge(g).astype(np.int64), exp_e)
    # sums: each butterfly has two U vertices, two V vertices, four edges
    total = int(bu.sum()) // 2
    assert int(bu.sum()) == 2 * total == int(bv.sum())
    assert int(oracle.count_edge(g).sum()) == 4 * total


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 2), (3, 4), (5, 3), (7, 9)])
def test_count_complete_bipartite(a, b):
    g = synth.complete(a, b)
    bu, bv = oracle.count_vertex(g)
    assert (bu == (a - 1) * C2(b)).all()
    assert (bv == (b - 1) * C2(a)).all()
    assert (oracle.count_edge(g) == (a - 1) * (b - 1)).all()


def test_count_forest_and_star_zero():
    star = synth.complete(1, 12)
    forest = synth.from_edges(6, 6, [(0, 0), (0, 1), (1, 2), (2, 2), (3, 3), (4, 4), (4, 5)])
    for g in (star, forest):
        bu, bv = oracle.count_vertex(g)
        assert not bu.any() and not bv.any()
        assert not oracle.count_edge(g).any()
        assert not oracle.tip(g, 0).any() and not oracle.tip(g, 1).any()
        assert not oracle.wing(g).any()


def test_empty_graphs():
    g = synth.from_edges(3, 4, [])
    assert oracle.count_vertex(g)[0].tolist() == [0, 0, 0]
    assert oracle.tip(g, 0).tolist() == [0, 0, 0]
    assert oracle.tip(g, 1).tolist() == [0, 0, 0, 0]
    assert oracle.wing(g).size == 0
    g0 = synth.from_edges(0, 0, [])
    assert oracle.tip(g0, 0).size == 0


def test_validate_rejects_malformed():
    g = synth.er(10, 10, 30, seed=5)
    bad = synth.Graph(g.n_u, g.n_v, g.row_ptr.copy(), g.col_idx.copy())
    r = int(np.flatnonzero(np.diff(g.row_ptr) >= 2)[0])
    j = int(g.row_ptr[r])
    bad.col_idx[j + 1] = bad.col_idx[j]        # duplicate inside a row
    assert oracle.validate(bad) == -2
    bad2 = synth.Graph(g.n_u, g.n_v, g.row_ptr.copy(), g.col_idx.copy())
    bad2.col_idx[0] = g.n_v                     # out of range
    assert oracle.validate(bad2) == -2
    with pytest.raises(oracle.OracleError):
        oracle.tip(bad, 0)


# ---------------------------------------------------------------- tip numbers


def test_tip_vs_bruteforce_tiny():
    for g in _tiny_graphs(120, 500, max_u=9, max_v=7):
        assert np.array_equal(oracle.tip(g, 0), brute.tip(g, 0)), g.name
        if g.n_v <= 12:
            assert np.array_equal(oracle.tip(g, 1), brute.tip(g, 1)), g.name


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (6, 4), (10, 10)])
def test_tip_complete_bipartite(a, b):
    g = synth.complete(a, b)
    assert (oracle.tip(g, 0) == (a - 1) * C2(b)).all()
    assert (oracle.tip(g, 1) == (b - 1) * C2(a)).all()


@pytest.mark.parametrize("a,b,t", [(2, 5, 4), (3, 6, 2), (4, 7, 5), (5, 9, 8)])
def test_tip_clamp_closed_form(a, b, t):
    # K_{a,b} plus one U-vertex x adjacent to t of the b V-vertices:
    # x has a*C(t,2) butterflies and is the unique minimum; after it is peeled
    # the others keep max(a*C(t,2), (a-1)*C(b,2)).  Without the clamp of
    # Algorithm 2 the others would drop to (a-1)*C(b,2).
    edges = [(u, v) for u in range(a) for v in range(b)] + [(a, v) for v in range(t)]
    g = synth.from_edges(a + 1, b, edges)
    th = oracle.tip(g, 0)
    assert th[a] == a * C2(t)
    assert (th[:a] == max(a * C2(t), (a - 1) * C2(b))).all()
    if (a, b, t) == (2, 5, 4):
        assert th.tolist() == [12, 12, 12]


# ---------------------------------------------------------------- wing numbers


def test_wing_vs_bruteforce_tiny():
    n = 0
    for g in _tiny_graphs(400, 900, max_u=6, max_v=6):
        if g.m > 14:
            continue
        assert np.array_equal(oracle.wing(g), brute.wing(g)), g.name
        n += 1
    assert n >= 100


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (6, 4), (9, 11)])
def test_wing_complete_bipartite(a, b):
    g = synth.complete(a, b)
    assert (oracle.wing(g) == (a - 1) * (b - 1)).all()


def test_wing_k22_plus_pendant():
    # K_{2,2}: every edge in the single butterfly; a pendant edge stays at 0
    g = synth.from_edges(3, 3, [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)])
    assert oracle.wing(g).tolist() == [1, 1, 1, 1, 0]


# ---------------------------------------------------------------- structure


def test_disjoint_union_and_pendant():
    g1 = synth.chung_lu(60, 30, 400, 2.2, 25, seed=7)
    g2 = synth.er(40, 25, 300, seed=8)
    gu = synth.disjoint_union([g1, g2])
    assert np.array_equal(oracle.tip(gu, 0), np.concatenate([oracle.tip(g1, 0), oracle.tip(g2, 0)]))
    assert np.array_equal(oracle.tip(gu, 1), np.concatenate([oracle.tip(g1, 1), oracle.tip(g2, 1)]))
    assert np.array_equal(oracle.wing(gu), np.concatenate([oracle.wing(g1), oracle.wing(g2)]))
    # a pendant U-vertex hanging off V-vertex 0 is in no butterfly and changes nothing
    u, v = g1.edges()
    edges = list(zip(u.tolist(), v.tolist())) + [(g1.n_u, 0)]
    gp = synth.from_edges(g1.n_u + 1, g1.n_v, edges)
    tp = oracle.tip(gp, 0)
    assert tp[-1] == 0 and np.array_equal(tp[:-1], oracle.tip(g1, 0))
    wp = oracle.wing(gp)
    # the pendant edge is the last edge id (largest u)
    assert wp[-1] == 0 and np.array_equal(wp[:-1], oracle.wing(g1))


def _level_sound_tip(g, theta, side):
    a = _adj(g) if side == 0 else _adj(g).T
    for k in sorted(set(theta.tolist()))[:: max(1, len(set(theta.tolist())) // 12)]:
        if k == 0:
            continue
        keep = theta >= k
        sub = a[keep]
        cc = sub @ sub.T
        np.fill_diagonal(cc, 0)
        sup = (cc * (cc - 1) // 2).sum(axis=1)
        assert (sup >= k).all(), k


@pytest.mark.parametrize("seed", [11, 12])
def test_tip_invariants(seed):
    g = synth.chung_lu(300, 120, 2500, 2.2, 100, seed=seed)
    bu, bv = oracle.count_vertex(g)
    for side, sup in ((0, bu), (1, bv)):
        theta, st, order = oracle.tip(g, side, return_stats=True, return_order=True)
        assert (theta <= sup).all()
        seq = theta[order]
        assert (np.diff(seq.astype(np.int64)) >= 0).all()      # non-decreasing along the peel order
        assert st["peeled"] == theta.size
        # wedges walked without dynamic graph updates: sum_u sum_{v in N_u} (d_v - 1)
        a = _adj(g) if side == 0 else _adj(g).T
        dv = a.sum(axis=0)
        assert st["wedges"] == int((a * (dv - 1)).sum())
        _level_sound_tip(g, theta, side)


@pytest.mark.parametrize("seed", [21, 22])
def test_wing_invariants(seed):
    g = synth.chung_lu(150, 80, 1200, 2.2, 60, seed=seed)
    be = oracle.count_edge(g)
    theta, st, order = oracle.wing(g, return_stats=True, return_order=True)
    assert (theta <= be).all()
    assert (np.diff(theta[order].astype(np.int64)) >= 0).all()
    # level soundness: inside {theta >= k} every edge there has >= k butterflies
    u, v = g.edges()
    for k in sorted(set(theta.tolist()))[::3]:
        if k == 0:
            continue
        keep = theta >= k
        a = np.zeros((g.n_u, g.n_v), np.int64)
        a[u[keep], v[keep]] = 1
        aata = a @ a.T @ a
        du = a.sum(axis=1)
        dv = a.sum(axis=0)
        sup = aata[u[keep], v[keep]] - du[u[keep]] - dv[v[keep]] + 1
        assert (sup >= k).all(), k


def test_single_level_ranges_give_their_level():
    """A range holding one support value (the GPU path's single-level
    partitions): with k the smallest support among the alive vertices of one
    side, removing every vertex whose support over the remaining graph is
    at most k, until none is left, must give each removed vertex tip number
    k.  Supports are recomputed from common-neighbour counts, independently
    of the oracle."""
    graphs = _tiny_graphs(40, 700) + [synth.complete(3, 4), synth.complete(4, 6)]
    for g in graphs:
        a = _adj(g)
        for side in (0, 1):
            m = a if side == 0 else a.T
            cn = m @ m.T
            n = m.shape[0]
            alive = np.ones(n, dtype=bool)
            theta = np.zeros(n, dtype=np.uint64)

            def supports():
                c = cn * alive[None, :] * alive[:, None]
                np.fill_diagonal(c, 0)
                return (c * (c - 1) // 2).sum(axis=1)

            while alive.any():
                s = supports()
                k = int(s[alive].min())
                while True:
                    low = alive & (s <= k)
                    if not low.any():
                        break
                    theta[low] = k
                    alive &= ~low
                    s = supports()
            assert np.array_equal(theta, oracle.tip(g, side)), (g.name, side)


# ---------------------------------------------------------------- k-tips / k-wings

def test_components_match_definitions_on_tiny_graphs():
    """The oracle's k-tips and k-wings (components of the entities at level
    >= k) equal the maximal sets of Definitions 1-2 found by exhaustive
    search, at every level k of every tiny graph."""
    for s in range(24):
        rng = np.random.default_rng(900 + s)
        g = synth.random_small(int(rng.integers(2, 8)), int(rng.integers(2, 7)), float(rng.choice([0.5, 0.8])),
                               seed=900 + s)
        for side in (0, 1):
            th = oracle.tip(g, side)
            for k in sorted(set([0] + th.tolist() + [int(th.max()) + 1])):
                assert np.array_equal(oracle.tip_components(g, side, th, k), brute.tip_components(g, side, k)), \
                    (g.name, side, k)
        if g.m <= 13:
            th = oracle.wing(g)
            for k in sorted(set([0] + th.tolist() + [int(th.max()) + 1])):
                assert np.array_equal(oracle.wing_components(g, th, k), brute.wing_components(g, k)), (g.name, k)


def test_components_two_squares_sharing_a_vertex():
    """Squares u0,u1 x v0,v1 and u1,u2 x v2,v3: every entity number is 1.
    The three U vertices form one 1-tip (u1 shares two neighbours with each
    of the others), but the edges form two 1-wings: no butterfly holds edges
    of both squares, although they share the vertex u1."""
    g = synth.from_edges(3, 4, [(0, 0), (0, 1), (1, 0), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3)])
    tu = oracle.tip(g, 0)
    assert tu.tolist() == [1, 1, 1]
    assert oracle.tip_components(g, 0, tu, 1).tolist() == [0, 0, 0]
    assert oracle.tip_components(g, 0, tu, 2).tolist() == [-1, -1, -1]
    tw = oracle.wing(g)
    assert tw.tolist() == [1] * 8
    assert oracle.wing_components(g, tw, 1).tolist() == [0, 0, 0, 0, 4, 4, 4, 4]
    assert oracle.wing_components(g, tw, 2).tolist() == [-1] * 8
    tv = oracle.tip(g, 1)
    # V side: v0, v1 share u0, u1; v2, v3 share u1, u2; no V pair spans both
    assert oracle.tip_components(g, 1, tv, 1).tolist() == [0, 0, 2, 2]


def test_components_nest_across_levels():
    """Every (k+1)-tip lies inside one k-tip, and likewise for wings (the
    hierarchy of Section 2.2); a complete bipartite graph is one component
    at every level up to its entity number."""
    g = synth.chung_lu(400, 120, 2500, 2.1, 100, seed=21)
    for side in (0, 1):
        th = oracle.tip(g, side)
        levels = sorted(set(th.tolist()))[::7]
        prev = None
        for k in levels:
            cur = oracle.tip_components(g, side, th, k)
            if prev is not None:
                for c in np.unique(cur[cur >= 0]):
                    assert len(np.unique(prev[cur == c])) == 1
            prev = cur
    tw = oracle.wing(g)
    prev = None
    for k in sorted(set(tw.tolist()))[::5]:
        cur = oracle.wing_components(g, tw, k)
        if prev is not None:
            for c in np.unique(cur[cur >= 0]):
                assert len(np.unique(prev[cur == c])) == 1
        prev = cur
    kab = synth.complete(4, 5)
    th = oracle.tip(kab, 0)
    assert oracle.tip_components(kab, 0, th, int(th[0])).tolist() == [0] * 4
    tw = oracle.wing(kab)
    assert oracle.wing_components(kab, tw, int(tw[0])).tolist() == [0] * 20
