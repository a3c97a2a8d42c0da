"""k-tips and k-wings (hierarchy retrieval, Section 2.2) on the GPU against
the oracle's components (bit-exact component labels: the smallest id of
each component), at several levels of tiny, closed-form and power-law
graphs, for device and host buffers."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2110_12511_amd as pb
import synth
from gpu_util import u64

pytestmark = pytest.mark.gpu


def _levels(th, n=6):
    if th.size == 0:
        return [0, 1]
    vals = np.unique(th)
    pick = set([0, int(vals.max()) + 1])
    pick |= set(int(v) for v in vals[np.linspace(0, vals.size - 1, min(n, vals.size)).astype(int)])
    return sorted(pick)


def _check(ctx, g, levels_tip=6, levels_wing=6, wing=True):
    dg = pb.DeviceGraph.from_graph(g)
    for side in (0, 1):
        th = pb.tip(ctx, dg, side)
        thn = u64(th)
        for k in _levels(thn, levels_tip):
            got = pb.tip_components(ctx, dg, side, th, k).cpu().numpy()
            exp = oracle.tip_components(g, side, thn, k)
            assert np.array_equal(got.astype(np.int64), exp), (g.name, side, k)
    if wing:
        tw = pb.wing(ctx, dg)
        twn = u64(tw)
        for k in _levels(twn, levels_wing):
            got = pb.wing_components(ctx, dg, tw, k).cpu().numpy()
            exp = oracle.wing_components(g, twn, k)
            assert np.array_equal(got.astype(np.int64), exp), (g.name, k)


def test_components_tiny_and_closed_forms(ctx):
    for s in range(20):
        rng = np.random.default_rng(1200 + s)
        g = synth.random_small(int(rng.integers(1, 12)), int(rng.integers(1, 9)), float(rng.choice([0.4, 0.7])),
                               seed=1200 + s)
        _check(ctx, g, 20, 20)
    g = synth.from_edges(3, 4, [(0, 0), (0, 1), (1, 0), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3)])
    dg = pb.DeviceGraph.from_graph(g)
    tw = pb.wing(ctx, dg)
    assert pb.wing_components(ctx, dg, tw, 1).cpu().tolist() == [0, 0, 0, 0, 4, 4, 4, 4]
    tu = pb.tip(ctx, dg, 0)
    assert pb.tip_components(ctx, dg, 0, tu, 1).cpu().tolist() == [0, 0, 0]
    _check(ctx, synth.disjoint_union([synth.complete(3, 4), synth.complete(2, 5), synth.from_edges(2, 2, [(0, 0)])]))


@pytest.mark.parametrize("seed", [31, 32])
def test_components_power_law(ctx, seed):
    g = synth.chung_lu(6000, 1500, 40000, 2.1, 800, seed=seed)
    _check(ctx, g, 6, 5)


def test_components_host_buffers(ctx):
    g = synth.chung_lu(800, 300, 5000, 2.2, 200, seed=33)
    th = oracle.tip(g, 0)
    k = int(np.median(th[th > 0]))
    rp, ci = np.ascontiguousarray(g.row_ptr), np.ascontiguousarray(g.col_idx)
    hc = pb.host_csr(g.n_u, g.n_v, rp, ci)
    out = np.zeros(g.n_u, np.int32)
    assert ctx.lib.pbng_tip_components(ctx.h, ctypes.byref(hc), 0, th.ctypes.data, ctypes.c_uint64(k), out.ctypes.data) == 0
    assert np.array_equal(out.astype(np.int64), oracle.tip_components(g, 0, th, k))
    tw = oracle.wing(g)
    kw = int(np.median(tw[tw > 0]))
    outw = np.zeros(g.m, np.int32)
    assert ctx.lib.pbng_wing_components(ctx.h, ctypes.byref(hc), tw.ctypes.data, ctypes.c_uint64(kw),
                                        outw.ctypes.data) == 0
    assert np.array_equal(outw.astype(np.int64), oracle.wing_components(g, tw, kw))
