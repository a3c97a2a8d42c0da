"""pbng_count_noalloc: the counting entry point that allocates nothing
(its work memory is the library's static per-device scratch array) gives
exactly pbng_count's results, call after call on the same array (the second
call on a smaller graph), and rejects a graph too large for the array."""
import ctypes

import numpy as np
import pytest

import paper_2110_12511_amd as pb
import synth
from gpu_util import u64

pytestmark = pytest.mark.gpu


def _noalloc(ctx, dg, kind, opts=None):
    import torch

    n = dg.n_u if kind == pb.COUNT_VERTEX_U else (dg.n_v if kind == pb.COUNT_VERTEX_V else dg.m)
    out = torch.full((max(n, 1),), 7, dtype=torch.uint64, device="cuda")
    rc = ctx.lib.pbng_count_noalloc(ctx.h, ctypes.byref(dg.csr()), kind, ctypes.byref(opts) if opts else None,
                                    ctypes.c_void_p(out.data_ptr()))
    return rc, out[:n]


def test_noalloc_matches_count_twice(ctx):
    big = synth.chung_lu(40000, 8000, 200000, 2.1, 3000, seed=11)
    small = synth.er(2000, 1000, 20000, seed=1)
    for g in (big, small):  # the second call reuses the array with a smaller graph
        dg = pb.DeviceGraph.from_graph(g)
        for kind in (pb.COUNT_VERTEX_U, pb.COUNT_VERTEX_V, pb.COUNT_EDGE):
            rc, res = _noalloc(ctx, dg, kind)
            assert rc == 0, ctx.lib.pbng_last_error(ctx.h).decode()
            exp = u64(pb.count(ctx, dg, kind))
            assert np.array_equal(u64(res), exp), (g.name, kind)


def test_noalloc_scalar_hub_path_and_empty(ctx):
    g = synth.chung_lu(20000, 4000, 100000, 2.0, 3000, seed=12)
    dg = pb.DeviceGraph.from_graph(g)
    for opts in (pb.make_opts(dense_cut=-1), pb.make_opts(dense_cut=256)):
        rc, res = _noalloc(ctx, dg, pb.COUNT_VERTEX_U, opts)
        assert rc == 0, ctx.lib.pbng_last_error(ctx.h).decode()
        assert np.array_equal(u64(res), u64(pb.count(ctx, dg, pb.COUNT_VERTEX_U, opts)))
    empty = pb.DeviceGraph.from_graph(synth.from_edges(3, 2, []))
    rc, res = _noalloc(ctx, empty, pb.COUNT_VERTEX_U)
    assert rc == 0 and u64(res).tolist() == [0, 0, 0]


def test_noalloc_rejects_large_and_host_graphs(ctx):
    # 40 bytes per edge beyond the 64 MiB array: rejected before any work
    m = (64 << 20) // 40 + 1
    rp = np.array([0, m], np.int64)
    ci = np.arange(m, dtype=np.int32)
    dg = pb.DeviceGraph(1, m, rp, ci)
    rc, _ = _noalloc(ctx, dg, pb.COUNT_VERTEX_U)
    assert rc == -5
    g = synth.complete(3, 4)
    hc = pb.host_csr(g.n_u, g.n_v, np.ascontiguousarray(g.row_ptr), np.ascontiguousarray(g.col_idx))
    out = np.zeros(3, np.uint64)
    assert ctx.lib.pbng_count_noalloc(ctx.h, ctypes.byref(hc), 0, None, out.ctypes.data) == -1
