"""CPU oracle for butterfly counting and tip / wing decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it, and
it shares no code with that path; both take their inputs from ``synth``.

``oracle.c`` holds the plain sequential routines (definitions of Section 2.1
and the bottom-up peeling of Section 2.2 / Algorithm 2); ``brute.py`` holds
exhaustive enumerations for tiny graphs.  This module compiles ``oracle.c``
with gcc on first use and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.rc = rc


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, i32 = ctypes.c_int64, ctypes.c_int
    lib.orc_validate.argtypes = [i64, i64, _i64p, _i32p]
    lib.orc_count_vertex.argtypes = [i64, i64, _i64p, _i32p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_count_edge.argtypes = [i64, i64, _i64p, _i32p, _u64p]
    lib.orc_tip.argtypes = [i64, i64, _i64p, _i32p, i32, _u64p, _u64p, ctypes.c_uint64, ctypes.c_void_p]
    lib.orc_wing.argtypes = [i64, i64, _i64p, _i32p, _u64p, _u64p, ctypes.c_uint64, ctypes.c_void_p]
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_tip_components.argtypes = [i64, i64, _i64p, _i32p, i32, _u64p, ctypes.c_uint64, _i64p]
    lib.orc_wing_components.argtypes = [i64, i64, _i64p, _i32p, _u64p, ctypes.c_uint64, _i64p]
    lib.orc_tip_components.restype = i32
    lib.orc_wing_components.restype = i32
    for f in (lib.orc_validate, lib.orc_count_vertex, lib.orc_count_edge, lib.orc_tip, lib.orc_wing, lib.orc_set_threads):
        f.restype = i32
    _lib = lib
    return lib


def _csr(g):
    return (int(g.n_u), int(g.n_v), np.ascontiguousarray(g.row_ptr, dtype=np.int64),
            np.ascontiguousarray(g.col_idx, dtype=np.int32))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> int:
    """Host threads for counting (start vertices split among them; results
    do not depend on it).  Peeling stays sequential.  Default 1."""
    return _load().orc_set_threads(int(n))


def validate(g) -> int:
    return _load().orc_validate(*_csr(g))


def count_vertex(g):
    """(support_u uint64[n_u], support_v uint64[n_v]) in the input graph."""
    n_u, n_v, rp, ci = _csr(g)
    bu = np.zeros(n_u, np.uint64)
    bv = np.zeros(n_v, np.uint64)
    rc = _load().orc_count_vertex(n_u, n_v, rp, ci, _ptr(bu), _ptr(bv))
    if rc:
        raise OracleError(rc, "count_vertex")
    return bu, bv


def count_edge(g):
    """Per-edge butterfly counts, uint64[m] in edge-id order."""
    n_u, n_v, rp, ci = _csr(g)
    be = np.zeros(g.m, np.uint64)
    rc = _load().orc_count_edge(n_u, n_v, rp, ci, be)
    if rc:
        raise OracleError(rc, "count_edge")
    return be


def tip(g, side: int = 0, return_stats: bool = False, wedge_budget: int = 0, return_order: bool = False):
    """Tip numbers of side U (side=0) or V (side=1) by bottom-up peeling."""
    n_u, n_v, rp, ci = _csr(g)
    n = n_u if side == 0 else n_v
    theta = np.zeros(n, np.uint64)
    stats = np.zeros(2, np.uint64)
    order = np.full(n, -1, np.int64) if return_order else None
    t0 = time.perf_counter()
    rc = _load().orc_tip(n_u, n_v, rp, ci, int(side), theta, stats, int(wedge_budget), _ptr(order))
    dt = time.perf_counter() - t0
    if rc and not (rc == -9 and wedge_budget):
        raise OracleError(rc, "tip")
    out = [theta]
    if return_stats:
        out.append(dict(wedges=int(stats[0]), peeled=int(stats[1]), seconds=dt, complete=(rc == 0)))
    if return_order:
        out.append(order)
    return out[0] if len(out) == 1 else tuple(out)


def wing(g, return_stats: bool = False, wedge_budget: int = 0, return_order: bool = False):
    """Wing numbers of every edge (edge-id order) by bottom-up peeling."""
    n_u, n_v, rp, ci = _csr(g)
    theta = np.zeros(g.m, np.uint64)
    stats = np.zeros(2, np.uint64)
    order = np.full(g.m, -1, np.int64) if return_order else None
    t0 = time.perf_counter()
    rc = _load().orc_wing(n_u, n_v, rp, ci, theta, stats, int(wedge_budget), _ptr(order))
    dt = time.perf_counter() - t0
    if rc and not (rc == -9 and wedge_budget):
        raise OracleError(rc, "wing")
    out = [theta]
    if return_stats:
        out.append(dict(wedges=int(stats[0]), updates=int(stats[1]), seconds=dt, complete=(rc == 0)))
    if return_order:
        out.append(order)
    return out[0] if len(out) == 1 else tuple(out)


def tip_components(g, side: int, theta, k: int):
    """k-tips of one side (Definition 2): for every vertex with tip number >= k
    the smallest vertex id of its butterfly-connected component, -1 below k."""
    n_u, n_v, rp, ci = _csr(g)
    th = np.ascontiguousarray(theta, dtype=np.uint64)
    out = np.zeros(max(n_u if side == 0 else n_v, 1), dtype=np.int64)
    rc = _load().orc_tip_components(n_u, n_v, rp, ci, int(side), th, int(k), out)
    if rc:
        raise OracleError(rc, "tip_components")
    return out[: (n_u if side == 0 else n_v)]


def wing_components(g, theta, k: int):
    """k-wings (Definition 1): for every edge with wing number >= k the
    smallest edge id of its butterfly-connected component, -1 below k."""
    n_u, n_v, rp, ci = _csr(g)
    th = np.ascontiguousarray(theta, dtype=np.uint64)
    out = np.zeros(max(g.m, 1), dtype=np.int64)
    rc = _load().orc_wing_components(n_u, n_v, rp, ci, th, int(k), out)
    if rc:
        raise OracleError(rc, "wing_components")
    return out[: g.m]
