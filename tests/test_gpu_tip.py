"""Parity of tip decomposition on the GPU with the CPU oracle (bit-exact),
plus invariance of the result under every schedule knob."""
import numpy as np
import pytest

import oracle
import paper_2110_12511_amd as pb
import synth
from gpu_util import u64, golden, check_golden

pytestmark = pytest.mark.gpu


def C2(x):
    return x * (x - 1) // 2


def gpu_tip(ctx, g, side, **kw):
    dg = pb.DeviceGraph.from_graph(g)
    return u64(pb.tip(ctx, dg, side, pb.make_opts(**kw) if kw else None))


def test_tip_tiny_random(ctx):
    for s in range(50):
        rng = np.random.default_rng(100 + s)
        g = synth.random_small(int(rng.integers(1, 14)), int(rng.integers(1, 10)), float(rng.choice([0.3, 0.6, 0.9])), seed=s)
        for side in (0, 1):
            exp = oracle.tip(g, side)
            for P in (1, 2, 5):
                assert np.array_equal(gpu_tip(ctx, g, side, P=P), exp), (g.name, side, P)


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (12, 9)])
def test_tip_complete(ctx, a, b):
    g = synth.complete(a, b)
    assert (gpu_tip(ctx, g, 0) == (a - 1) * C2(b)).all()
    assert (gpu_tip(ctx, g, 1) == (b - 1) * C2(a)).all()


@pytest.mark.parametrize("a,b,t", [(2, 5, 4), (4, 7, 5)])
def test_tip_clamp_closed_form(ctx, a, b, t):
    edges = [(u, v) for u in range(a) for v in range(b)] + [(a, v) for v in range(t)]
    g = synth.from_edges(a + 1, b, edges)
    for P in (1, 2, 3):
        th = gpu_tip(ctx, g, 0, P=P)
        assert th[a] == a * C2(t)
        assert (th[:a] == max(a * C2(t), (a - 1) * C2(b))).all()


def test_tip_empty_and_isolated(ctx):
    g = synth.from_edges(4, 3, [(0, 0), (3, 2)])
    assert gpu_tip(ctx, g, 0).tolist() == [0, 0, 0, 0]
    assert gpu_tip(ctx, g, 1).tolist() == [0, 0, 0]


@pytest.mark.parametrize("side", [0, 1])
def test_tip_er_small_config(ctx, side):
    g = synth.config_graph("er_2k_1k_20k")
    rec = golden("er_2k_1k_20k", "tip_u" if side == 0 else "tip_v")
    res = gpu_tip(ctx, g, side, P=8)
    check_golden(rec, res, g.digest())
    assert np.array_equal(res, oracle.tip(g, side))


@pytest.fixture(scope="module")
def cl_mid():
    g = synth.chung_lu(30000, 6000, 300000, 2.1, 4000, seed=5)
    return g, oracle.tip(g, 0), oracle.tip(g, 1)


@pytest.mark.parametrize("P", [0, 1, 7, 150, 1000])
def test_tip_power_law_partitions(ctx, cl_mid, P):
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=P), eu)
    assert np.array_equal(gpu_tip(ctx, g, 1, P=P), ev)


ALL_ALIVE = (1 << 31) - 1  # level_alive: single levels from the start


@pytest.mark.parametrize("P,max_alive", [(1, ALL_ALIVE), (40, 5000), (150, 800)])
def test_tip_single_level_partitions(ctx, cl_mid, P, max_alive):
    """A range holding one support value k gives every vertex tip number k
    with no fine-grained peeling; ranges first, then single levels once at
    most `max_alive` vertices are left whatever their work (from the start
    with P = 1), must reproduce the oracle."""
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=P, level_alive=max_alive), eu)
    if P == 1:
        # every partition is one level: one partition per distinct tip number
        assert ctx.stats()["partitions"] == len(np.unique(eu))
    assert np.array_equal(gpu_tip(ctx, g, 1, P=P, level_alive=max_alive), ev)


def test_tip_single_level_small_graphs(ctx):
    for s in range(20):
        rng = np.random.default_rng(300 + s)
        g = synth.random_small(int(rng.integers(1, 14)), int(rng.integers(1, 10)), float(rng.choice([0.4, 0.8])), seed=s)
        for side in (0, 1):
            for P in (1, 2):
                res = gpu_tip(ctx, g, side, P=P, level_alive=ALL_ALIVE)
                assert np.array_equal(res, oracle.tip(g, side)), (g.name, side, P)
    for a, b in ((3, 5), (12, 9)):
        g = synth.complete(a, b)
        assert np.array_equal(gpu_tip(ctx, g, 0, P=1, level_alive=ALL_ALIVE), oracle.tip(g, 0))


@pytest.mark.parametrize("b,t", [(65535, 65000), (70000, 66000)])
@pytest.mark.parametrize("P", [1, 2, 0])
def test_tip_degree_at_least_2_16(ctx, b, t, P):
    """K_{2,b} plus a vertex x on t of the b columns: x is peeled alone with
    c(x, u) = t common neighbours, and every tip number is 2 C(t, 2) (the
    clamp closed form a C(t, 2) >= (a - 1) C(b, 2) with a = 2).  At
    b = 65535 every count fits 16 bits (the largest packed counter value);
    at b = 70000 the degrees and counts pass 2^16, which the key-tile and
    fine-grained counters must hold without carrying or wrapping."""
    edges = [(u, v) for u in range(2) for v in range(b)] + [(2, v) for v in range(t)]
    g = synth.from_edges(3, b, edges)
    exp = 2 * C2(t)
    assert exp > C2(b)
    res = gpu_tip(ctx, g, 0, P=P)
    assert res.tolist() == [exp, exp, exp]
    assert np.array_equal(res, oracle.tip(g, 0))
    assert np.array_equal(gpu_tip(ctx, g, 1, P=P), oracle.tip(g, 1))


@pytest.mark.parametrize("P", [2, 7, 40])
def test_tip_recount_rounds(ctx, cl_mid, P):
    """Section 5.1: a round whose active set has more live wedges than the
    recount bound recounts the remaining graph instead of peeling.  With the
    bound forced down to 1 every such round recounts (P = 1 has no rounds:
    its one partition takes every vertex at once); results are the
    oracle's."""
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=P, recount_w=1), eu)
    assert ctx.stats()["recounts"] > 0
    assert np.array_equal(gpu_tip(ctx, g, 1, P=P, recount_w=1), ev)
    assert ctx.stats()["recounts"] > 0
    for s in range(10):
        gs = synth.random_small(12, 9, 0.6, seed=700 + s)
        assert np.array_equal(gpu_tip(ctx, gs, 0, P=3, recount_w=1), oracle.tip(gs, 0))


@pytest.mark.parametrize("P", [1, 7, 150])
def test_tip_host_rounds_match_captured(ctx, cl_mid, P):
    """Coarse-grained rounds replayed from a captured HIP graph and rounds
    driven from the host give the oracle's numbers in the same number of
    rounds."""
    g, eu, ev = cl_mid
    for side, exp in ((0, eu), (1, ev)):
        a = gpu_tip(ctx, g, side, P=P)
        ra = ctx.stats()["rho"]
        b = gpu_tip(ctx, g, side, P=P, flags=pb.F_HOST_ROUNDS)
        rb = ctx.stats()["rho"]
        assert np.array_equal(a, exp) and np.array_equal(b, exp)
        assert ra == rb, (side, ra, rb)


def test_tip_recount_rounds_host_driven(ctx, cl_mid):
    g, eu, _ = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=7, recount_w=1, flags=pb.F_HOST_ROUNDS), eu)
    assert ctx.stats()["recounts"] > 0


def test_tip_paper_rule(ctx, cl_mid):
    """The paper's bound rule alone (no vertex-count target, no single
    levels) gives the same numbers."""
    g, eu, ev = cl_mid
    for P in (7, 150):
        assert np.array_equal(gpu_tip(ctx, g, 0, P=P, bound_rule=pb.BOUND_PAPER), eu)
        assert ctx.stats()["bound_rule_used"] == pb.BOUND_PAPER
        assert np.array_equal(gpu_tip(ctx, g, 1, P=P, bound_rule=pb.BOUND_PAPER), ev)


def _check_schedule(ctx, g, side, exp, **kw):
    """Theorem 1 and the initialisation vector: every vertex of partition i
    has theta(i) <= tip < theta(i+1); bounds increase; a vertex's support at
    its partition's start equals its butterflies among the vertices of its
    own and later partitions (the oracle's count on that subgraph)."""
    dg = pb.DeviceGraph.from_graph(g)
    th, part, init, bounds, npart = pb.tip_schedule(ctx, dg, side, pb.make_opts(**kw))
    th, init, bounds = u64(th), u64(init), u64(bounds)
    part = part.cpu().numpy()
    assert np.array_equal(th, exp)
    assert npart == bounds.size and npart >= 1
    assert (part >= 0).all() and (part < npart).all()
    assert (np.diff(bounds.astype(object)) > 0).all()
    lo = np.concatenate([[0], bounds[:-1]]).astype(np.uint64)
    assert (lo[part] <= th).all() and (th < bounds[part]).all()
    # initialisation vector against the oracle, partition by partition
    gx = g if side == 0 else synth.from_edges(g.n_v, g.n_u, list(zip(*reversed(g.edges()))))
    u, v = gx.edges()
    for i in np.unique(part):
        keep = part[u] >= i
        sub = synth.from_edges(gx.n_u, gx.n_v, list(zip(u[keep], v[keep])))
        sup = oracle.count_vertex(sub)[0]
        sel = part == i
        assert np.array_equal(init[sel], sup[sel]), (side, int(i))
    return npart


@pytest.mark.parametrize("rule", [pb.BOUND_PLAIN, pb.BOUND_PAPER, pb.BOUND_RANDOM])
def test_tip_schedule_theorem1(ctx, rule):
    g = synth.config_graph("er_2k_1k_20k")
    for side in (0, 1):
        exp = oracle.tip(g, side)
        npart = _check_schedule(ctx, g, side, exp, P=8, bound_rule=rule, seed=3)
        # (a random bound may take every vertex into its first partition)
        assert npart > 1 or rule == pb.BOUND_RANDOM
    gm = synth.chung_lu(6000, 1500, 40000, 2.1, 800, seed=9)
    for side in (0, 1):
        _check_schedule(ctx, gm, side, oracle.tip(gm, side), P=12, bound_rule=rule, seed=5)


def test_tip_schedule_levels_and_recounts(ctx):
    gm = synth.chung_lu(6000, 1500, 40000, 2.1, 800, seed=9)
    exp = oracle.tip(gm, 0)
    _check_schedule(ctx, gm, 0, exp, P=6, level_alive=400)
    _check_schedule(ctx, gm, 0, exp, P=6, recount_w=1)


@pytest.mark.parametrize("flags", [pb.F_NO_DYNAMIC, pb.F_NO_BATCH, pb.F_NO_DYNAMIC | pb.F_NO_BATCH])
def test_tip_ablation_flags(ctx, cl_mid, flags):
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=40, flags=flags), eu)
    assert np.array_equal(gpu_tip(ctx, g, 1, P=40, flags=flags), ev)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tip_random_bounds(ctx, cl_mid, seed):
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=60, bound_rule=pb.BOUND_RANDOM, seed=seed), eu)


def test_tip_stats_and_host_buffers(ctx, cl_mid):
    g, eu, _ = cl_mid
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    ci = np.ascontiguousarray(g.col_idx, np.int32)
    out = np.zeros(g.n_u, np.uint64)
    ctx.tip_raw(pb.host_csr(g.n_u, g.n_v, rp, ci), pb.SIDE_U, out.ctypes.data, pb.make_opts(P=150))
    assert np.array_equal(out, eu)
    st = ctx.stats()
    assert st["partitions"] >= 1 and st["rho"] >= st["partitions"] - 1
    assert st["wedges"] == st["wedges_count"] + st["wedges_cd"] + st["wedges_fd"]


@pytest.mark.parametrize("wl,q", [("cl_500k_100k_5m", "tip_u"), ("cl_500k_100k_5m", "tip_v"),
                                  ("cl_1m_200k_20m", "tip_u"), ("cl_1m_200k_20m", "tip_v")])
def test_tip_full_size_golden(ctx, wl, q):
    rec = golden(wl, q)
    if rec is None:
        pytest.skip("no stored oracle result")
    g = synth.config_graph(wl)
    res = gpu_tip(ctx, g, 0 if q == "tip_u" else 1, P=150)
    check_golden(rec, res, g.digest())


@pytest.fixture(scope="module")
def graph_100m():
    return synth.config_graph("cl_5m_1m_100m")


@pytest.mark.parametrize("rule", [pb.BOUND_PAPER, pb.BOUND_PLAIN])
def test_tip_100m_edges_golden(ctx, graph_100m, rule):
    """Side U of the 100M-edge Chung-Lu graph (5M x 1M, exponent 2.0, degree
    cap 50k) at P = 150, in the benchmark's launch configuration (captured
    rounds), against the oracle's full result, under the paper's range-bound
    rule and the library's plain rule."""
    rec = golden("cl_5m_1m_100m", "tip_u")
    if rec is None:
        pytest.skip("no stored oracle result")
    dg = pb.DeviceGraph.from_graph(graph_100m)
    res = u64(pb.tip(ctx, dg, 0, pb.make_opts(P=150, bound_rule=rule)))
    check_golden(rec, res, graph_100m.digest())


@pytest.mark.parametrize("cut", [-1, 16, 256])
def test_tip_dense_tile_cutovers(ctx, cl_mid, cut):
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=150, dense_cut=cut), eu)
    assert np.array_equal(gpu_tip(ctx, g, 1, P=150, dense_cut=cut), ev)


@pytest.mark.parametrize("tile_w", [-1, 1, 5000, 100000])
def test_tip_heavy_paths(ctx, cl_mid, tile_w):
    """Key tiles vs LDS hash ranges for the heavy active vertices: same result."""
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=150, tile_w=tile_w), eu)
    assert np.array_equal(gpu_tip(ctx, g, 1, P=150, tile_w=tile_w), ev)


def clustered_graph(seed=7):
    """Three hubs over overlapping blocks of ~17k consecutive U ids plus sparse
    extras: the 2-hop keys of a block vertex crowd one key range, more than an
    LDS hash range holds, so keys spill to the HBM counters."""
    rng = np.random.default_rng(seed)
    n_u, n_v = 200000, 64
    edges = set()
    for v, (a, b) in enumerate([(0, 17000), (500, 17500), (1000, 18000)]):
        for u in range(a, b):
            edges.add((u, v))
    for u in range(0, 20000):
        for v in rng.choice(np.arange(3, n_v), size=int(rng.integers(0, 4)), replace=False):
            edges.add((u, int(v)))
    for u in rng.integers(20000, n_u, 3000):
        edges.add((int(u), int(rng.integers(3, n_v))))
    return synth.from_edges(n_u, n_v, sorted(edges))


@pytest.fixture(scope="module")
def clustered():
    g = clustered_graph()
    return g, oracle.tip(g, 0)


@pytest.mark.parametrize("P,tile_w", [(1, 0), (8, 0), (40, 0), (40, -1), (40, 5000)])
def test_tip_clustered_keys_overflow(ctx, clustered, P, tile_w):
    g, eu = clustered
    assert np.array_equal(gpu_tip(ctx, g, 0, P=P, tile_w=tile_w), eu)


@pytest.mark.parametrize("tile_w", [-1, 0])
def test_tip_short_probe_overflow_pass(ctx, cl_mid, clustered, tile_w):
    """With a one-slot LDS probe limit most items of the key-range kernel
    overflow and are counted again in the HBM counters that all workgroups
    share under a lock: the result is unchanged."""
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=150, tile_w=tile_w, flags=pb.F_SHORT_PROBE), eu)
    # kernel-class counters (filled under kernel timing): the path ran
    t = gpu_tip(ctx, g, 0, P=150, tile_w=tile_w, flags=pb.F_SHORT_PROBE | pb.binding.F_KERNEL_TIMING)
    assert np.array_equal(t, eu)
    assert ctx.stats()["kstat"]["tip_hrange"]["wedges"] > 0
    assert np.array_equal(gpu_tip(ctx, g, 1, P=150, tile_w=tile_w, flags=pb.F_SHORT_PROBE), ev)
    gc, ec = clustered
    assert np.array_equal(gpu_tip(ctx, gc, 0, P=8, tile_w=tile_w, flags=pb.F_SHORT_PROBE), ec)


def test_autotune_tip_and_cache(ctx, cl_mid):
    g, eu, ev = cl_mid
    dg = pb.DeviceGraph.from_graph(g)
    best, ms = ctx.autotune(dg, 0, pb.make_opts(P=40))
    assert ms > 0 and best.P in (20, 40, 80)
    assert best.bound_rule in (pb.BOUND_PLAIN, pb.BOUND_PAPER) and best.recount_w in (0, -1)
    assert np.array_equal(u64(pb.tip(ctx, dg, 0, best)), eu)
    best2, ms2 = ctx.autotune(dg, 0, pb.make_opts(P=40))
    assert (best2.P, best2.dense_cut, best2.tile_w, best2.bound_rule, best2.recount_w, ms2) == \
        (best.P, best.dense_cut, best.tile_w, best.bound_rule, best.recount_w, ms)
    # a caller's learned rule is kept
    best3, _ = ctx.autotune(dg, 1, pb.make_opts(P=40, bound_rule=pb.BOUND_LEARNED))
    assert best3.bound_rule == pb.BOUND_LEARNED
    bv, _ = ctx.autotune(dg, 1)
    assert np.array_equal(u64(pb.tip(ctx, dg, 1, bv)), ev)
