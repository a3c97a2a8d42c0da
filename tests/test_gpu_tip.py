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


@pytest.fixture
def force_levels(monkeypatch):
    """Single-level partitions as soon as at most `max_alive` vertices are
    left, whatever their work (the default needs a small, heavy core)."""
    def setup(max_alive=1 << 40):
        monkeypatch.setenv("PBNG_LEVEL_MAX_ALIVE", str(max_alive))
        monkeypatch.setenv("PBNG_LEVEL_MIN_WORK", "0")
        monkeypatch.setenv("PBNG_LEVEL_MIN_AVG", "0")
    return setup


@pytest.mark.parametrize("P,max_alive", [(1, 1 << 40), (40, 5000), (150, 800)])
def test_tip_single_level_partitions(ctx, cl_mid, force_levels, P, max_alive):
    """A range holding one support value k gives every vertex tip number k
    with no fine-grained peeling; ranges first, then single levels once few
    vertices are left (from the start with P = 1), must reproduce the
    oracle."""
    force_levels(max_alive)
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=P), eu)
    if P == 1:
        # every partition is one level: one partition per distinct tip number
        assert ctx.stats()["partitions"] == len(np.unique(eu))
    assert np.array_equal(gpu_tip(ctx, g, 1, P=P), ev)


def test_tip_single_level_small_graphs(ctx, force_levels):
    force_levels()
    for s in range(20):
        rng = np.random.default_rng(300 + s)
        g = synth.random_small(int(rng.integers(1, 14)), int(rng.integers(1, 10)), float(rng.choice([0.4, 0.8])), seed=s)
        for side in (0, 1):
            for P in (1, 2):
                assert np.array_equal(gpu_tip(ctx, g, side, P=P), oracle.tip(g, side)), (g.name, side, P)
    for a, b in ((3, 5), (12, 9)):
        g = synth.complete(a, b)
        assert np.array_equal(gpu_tip(ctx, g, 0, P=1), oracle.tip(g, 0))


@pytest.mark.parametrize("min_f", [0, 200])
def test_tip_receiving_side_rounds(ctx, cl_mid, monkeypatch, min_f):
    """Rounds peeled from the receiving side (off by default; on for every
    round at min_f = 0, for active sets of 200 or more at min_f = 200) give
    the oracle's numbers."""
    monkeypatch.setenv("PBNG_PULL_MIN_F", str(min_f))
    g, eu, ev = cl_mid
    assert np.array_equal(gpu_tip(ctx, g, 0, P=40), eu)
    assert np.array_equal(gpu_tip(ctx, g, 1, P=40), ev)


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


def test_autotune_tip_and_cache(ctx, cl_mid):
    g, eu, ev = cl_mid
    dg = pb.DeviceGraph.from_graph(g)
    best, ms = ctx.autotune(dg, 0, pb.make_opts(P=40))
    assert ms > 0 and best.P in (20, 40, 80)
    assert np.array_equal(u64(pb.tip(ctx, dg, 0, best)), eu)
    best2, ms2 = ctx.autotune(dg, 0, pb.make_opts(P=40))
    assert (best2.P, best2.dense_cut, best2.tile_w, ms2) == (best.P, best.dense_cut, best.tile_w, ms)
    bv, _ = ctx.autotune(dg, 1)
    assert np.array_equal(u64(pb.tip(ctx, dg, 1, bv)), ev)
