"""Parity of butterfly counting on the GPU with the CPU oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
import paper_2110_12511_amd as pb
import synth
from gpu_util import u64, golden, check_golden

pytestmark = pytest.mark.gpu


def _gpu_counts(ctx, g, host=False):
    if host:
        rp = np.ascontiguousarray(g.row_ptr, np.int64)
        ci = np.ascontiguousarray(g.col_idx, np.int32)
        csr = pb.host_csr(g.n_u, g.n_v, rp, ci)
        outs = []
        for kind, n in ((pb.COUNT_VERTEX_U, g.n_u), (pb.COUNT_VERTEX_V, g.n_v), (pb.COUNT_EDGE, g.m)):
            o = np.zeros(max(n, 1), np.uint64)
            ctx.count_raw(csr, kind, o.ctypes.data)
            outs.append(o[:n])
        return outs
    dg = pb.DeviceGraph.from_graph(g)
    return [u64(pb.count(ctx, dg, k)) for k in (pb.COUNT_VERTEX_U, pb.COUNT_VERTEX_V, pb.COUNT_EDGE)]


def _check(ctx, g, host=False):
    bu, bv, be = _gpu_counts(ctx, g, host)
    ou, ov = oracle.count_vertex(g)
    oe = oracle.count_edge(g)
    assert np.array_equal(bu, ou), g.name
    assert np.array_equal(bv, ov), g.name
    assert np.array_equal(be, oe), g.name


def test_count_tiny_random(ctx):
    for s in range(60):
        rng = np.random.default_rng(s)
        g = synth.random_small(int(rng.integers(1, 12)), int(rng.integers(1, 12)), float(rng.choice([0.2, 0.5, 0.9])), seed=s)
        _check(ctx, g)


def test_count_host_buffers(ctx):
    _check(ctx, synth.er(200, 150, 3000, seed=3), host=True)


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (3, 7), (40, 33)])
def test_count_complete(ctx, a, b):
    _check(ctx, synth.complete(a, b))


def test_count_empty_and_isolated(ctx):
    _check(ctx, synth.from_edges(5, 7, []))
    _check(ctx, synth.from_edges(5, 7, [(0, 0), (4, 6)]))


def test_count_er_small_config(ctx):
    _check(ctx, synth.config_graph("er_2k_1k_20k"))


@pytest.mark.parametrize("seed", [5, 6])
def test_count_power_law_all_bins(ctx, seed):
    # hubs of a few thousand: starts land in the small, medium and dense bins
    g = synth.chung_lu(30000, 6000, 300000, 2.1, 4000, seed=seed)
    _check(ctx, g)


def test_count_malformed_rejected(ctx):
    g = synth.er(20, 20, 60, seed=9)
    col = g.col_idx.copy()
    r = int(np.flatnonzero(np.diff(g.row_ptr) >= 2)[0])
    col[g.row_ptr[r] + 1] = col[g.row_ptr[r]]
    dg = pb.DeviceGraph(g.n_u, g.n_v, g.row_ptr, col)
    with pytest.raises(pb.PbngError) as ei:
        pb.count(ctx, dg, pb.COUNT_VERTEX_U)
    assert ei.value.code == -2


@pytest.mark.parametrize("quantity", ["count_u", "count_e"])
def test_count_full_size_golden(ctx, quantity):
    wl = "cl_500k_100k_5m"
    rec = golden(wl, quantity)
    if rec is None:
        pytest.skip("no stored oracle result")
    g = synth.config_graph(wl)
    dg = pb.DeviceGraph.from_graph(g)
    kind = pb.COUNT_VERTEX_U if quantity == "count_u" else pb.COUNT_EDGE
    res = u64(pb.count(ctx, dg, kind))
    check_golden(rec, res, g.digest())


# ---- hub blocks on matrix cores: identical counts for every cut-over degree


def _side_counts(ctx, g, cut):
    dg = pb.DeviceGraph.from_graph(g)
    o = pb.make_opts(dense_cut=cut)
    return (u64(pb.count(ctx, dg, pb.COUNT_VERTEX_U, o)), u64(pb.count(ctx, dg, pb.COUNT_VERTEX_V, o)))


@pytest.mark.parametrize("cut", [-1, 1, 2, 5, 40])
def test_count_dense_tile_cutovers_tiny(ctx, cut):
    for s in range(25):
        rng = np.random.default_rng(700 + s)
        g = synth.random_small(int(rng.integers(2, 40)), int(rng.integers(2, 40)), float(rng.choice([0.2, 0.5, 0.9])), seed=s)
        ou, ov = oracle.count_vertex(g)
        bu, bv = _side_counts(ctx, g, cut)
        assert np.array_equal(bu, ou), (g.name, cut)
        assert np.array_equal(bv, ov), (g.name, cut)


@pytest.mark.parametrize("cut", [-1, 8, 64, 1024])
def test_count_dense_tile_power_law(ctx, cut):
    g = synth.chung_lu(30000, 6000, 300000, 2.1, 4000, seed=5)
    ou, ov = oracle.count_vertex(g)
    bu, bv = _side_counts(ctx, g, cut)
    assert np.array_equal(bu, ou) and np.array_equal(bv, ov)
    st = ctx.stats()
    if cut > 0:
        assert st["dense_pairs"] > 0


def test_count_dense_tile_complete(ctx):
    # K_{70,90}: every vertex is a hub at cut 10; all butterflies come from the Gram tile
    g = synth.complete(70, 90)
    bu, bv = _side_counts(ctx, g, 10)
    assert (bu == 69 * (90 * 89 // 2)).all() and (bv == 89 * (70 * 69 // 2)).all()
