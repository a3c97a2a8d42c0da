"""Thin ctypes binding of libpbng.so (argument marshalling only).

Every computation runs in the HIP library; this module only moves pointers
and sizes across the C ABI declared in include/pbng.h.  It raises when the
built library is missing: there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbng.so")

COUNT_VERTEX_U, COUNT_VERTEX_V, COUNT_EDGE = 0, 1, 2
SIDE_U, SIDE_V = 0, 1
BOUND_PLAIN, BOUND_LEARNED, BOUND_RANDOM, BOUND_PAPER = 0, 1, 2, 3
F_NO_DYNAMIC, F_NO_BATCH, F_NO_DENSE_TILE = 0x1, 0x2, 0x4

ERRORS = {
    -1: "PBNG_E_ARG",
    -2: "PBNG_E_GRAPH",
    -3: "PBNG_E_NOMEM",
    -4: "PBNG_E_DEVICE",
    -5: "PBNG_E_OVERFLOW",
    -6: "PBNG_E_TIMEOUT",
    -7: "PBNG_E_UNSUPPORTED",
}


class PbngError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [
        ("n_u", ctypes.c_int64),
        ("n_v", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("on_device", ctypes.c_int32),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("P", ctypes.c_int32),
        ("bound_rule", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("seed", ctypes.c_int32),
        ("dense_cut", ctypes.c_int32),
        ("tile_w", ctypes.c_int32),
        ("batch_edges", ctypes.c_int32),
        ("wide_work", ctypes.c_int32),
        ("level_alive", ctypes.c_int32),
        ("recount_w", ctypes.c_int32),
    ]


K_COUNT, K_TIP_PEEL, K_FD, K_WING_CD, K_DENSE, K_TIP_HRANGE, K_TIP_TILED, K_NCLASS = 0, 1, 2, 3, 4, 5, 6, 7
K_NAMES = ["count", "tip_peel", "fd", "wing_cd", "dense", "tip_hrange", "tip_tiled"]
F_KERNEL_TIMING = 0x8
F_HOST_ROUNDS = 0x10
F_SHORT_PROBE = 0x20


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double),
        ("launches", ctypes.c_uint64),
        ("bytes", ctypes.c_uint64),
        ("wedges", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("ms_total", ctypes.c_double),
        ("ms_prep", ctypes.c_double),
        ("ms_count", ctypes.c_double),
        ("ms_cd", ctypes.c_double),
        ("ms_fd_prep", ctypes.c_double),
        ("ms_fd", ctypes.c_double),
        ("wedges", ctypes.c_uint64),
        ("wedges_count", ctypes.c_uint64),
        ("wedges_cd", ctypes.c_uint64),
        ("wedges_fd", ctypes.c_uint64),
        ("updates", ctypes.c_uint64),
        ("links", ctypes.c_uint64),
        ("blooms", ctypes.c_uint64),
        ("bloom_pairs", ctypes.c_uint64),
        ("rho", ctypes.c_uint64),
        ("recounts", ctypes.c_uint64),
        ("partitions", ctypes.c_int32),
        ("P_used", ctypes.c_int32),
        ("bound_rule_used", ctypes.c_int32),
        ("fd_wide", ctypes.c_int32),
        ("fd_work_max", ctypes.c_uint64),
        ("fd_work_sum", ctypes.c_uint64),
        ("dense_pairs", ctypes.c_uint64),
        ("kstat", KernelStat * K_NCLASS),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "kstat"}
        d["kstat"] = {
            K_NAMES[i]: dict(ms=self.kstat[i].ms, launches=self.kstat[i].launches, bytes=self.kstat[i].bytes,
                             wedges=self.kstat[i].wedges)
            for i in range(K_NCLASS)
        }
        return d


EXPORTS = ["pbng_create", "pbng_destroy", "pbng_last_error", "pbng_last_stats", "pbng_count", "pbng_tip", "pbng_wing",
           "pbng_tip_features", "pbng_mlp_init", "pbng_mlp_set", "pbng_mlp_get", "pbng_mlp_forward",
           "pbng_mlp_loss_grad", "pbng_mlp_train", "pbng_tip_batch", "pbng_wing_batch", "pbng_autotune",
           "pbng_tip_schedule", "pbng_predictor_load", "pbng_count_noalloc", "pbng_tip_hinted",
           "pbng_tip_components", "pbng_wing_components"]
MLP_NPARAM = 8961

_lib = None


def load():
    """Load libpbng.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or python -m paper_2110_12511_amd.build")
    # PyTorch ships its own HIP runtime.  Importing it first makes the dynamic
    # loader bind this library to that same runtime, so device pointers and
    # streams from torch are valid here (one HIP runtime per process).
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.pbng_create.argtypes = [ctypes.POINTER(vp), vp]
    lib.pbng_create.restype = ctypes.c_int
    lib.pbng_destroy.argtypes = [vp]
    lib.pbng_destroy.restype = None
    lib.pbng_last_error.argtypes = [vp]
    lib.pbng_last_error.restype = ctypes.c_char_p
    lib.pbng_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.pbng_last_stats.restype = ctypes.c_int
    lib.pbng_count.argtypes = [vp, ctypes.POINTER(Csr), ctypes.c_int, ctypes.POINTER(Opts), vp]
    lib.pbng_count.restype = ctypes.c_int
    lib.pbng_count_noalloc.argtypes = [vp, ctypes.POINTER(Csr), ctypes.c_int, ctypes.POINTER(Opts), vp]
    lib.pbng_count_noalloc.restype = ctypes.c_int
    lib.pbng_tip.argtypes = [vp, ctypes.POINTER(Csr), ctypes.c_int, ctypes.POINTER(Opts), vp]
    lib.pbng_tip.restype = ctypes.c_int
    lib.pbng_wing.argtypes = [vp, ctypes.POINTER(Csr), ctypes.POINTER(Opts), vp]
    lib.pbng_wing.restype = ctypes.c_int
    i64, f32 = ctypes.c_int64, ctypes.c_float
    sigs = {
        "pbng_tip_features": [vp, ctypes.POINTER(Csr), ctypes.c_int, vp],
        "pbng_mlp_init": [vp, ctypes.c_uint64],
        "pbng_mlp_set": [vp, vp],
        "pbng_mlp_get": [vp, vp],
        "pbng_mlp_forward": [vp, vp, i64, vp],
        "pbng_mlp_loss_grad": [vp, vp, vp, vp, i64, vp, vp],
        "pbng_mlp_train": [vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_int32, f32, vp],
        "pbng_tip_batch": [vp, vp, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(Opts), vp],
        "pbng_wing_batch": [vp, vp, ctypes.c_int32, ctypes.POINTER(Opts), vp],
        "pbng_autotune": [vp, ctypes.POINTER(Csr), ctypes.c_int32, ctypes.POINTER(Opts), ctypes.POINTER(Opts),
                          ctypes.POINTER(ctypes.c_double)],
        "pbng_tip_schedule": [vp, ctypes.POINTER(Csr), ctypes.c_int, ctypes.POINTER(Opts), vp, vp, vp, vp,
                              ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
        "pbng_predictor_load": [vp, ctypes.c_char_p],
        "pbng_tip_hinted": [vp, ctypes.POINTER(Csr), ctypes.c_int, ctypes.POINTER(Opts), vp, vp],
        "pbng_tip_components": [vp, ctypes.POINTER(Csr), ctypes.c_int, vp, ctypes.c_uint64, vp],
        "pbng_wing_components": [vp, ctypes.POINTER(Csr), vp, ctypes.c_uint64, vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def make_opts(P=0, bound_rule=BOUND_PLAIN, flags=0, seed=0, dense_cut=0, tile_w=0, batch_edges=0,
              wide_work=0, level_alive=0, recount_w=0) -> Opts:
    o = Opts()
    o.P, o.bound_rule, o.flags, o.seed, o.dense_cut = int(P), int(bound_rule), int(flags), int(seed), int(dense_cut)
    o.tile_w, o.batch_edges, o.wide_work = int(tile_w), int(batch_edges), int(wide_work)
    o.level_alive, o.recount_w = int(level_alive), int(recount_w)
    return o


class Context:
    """One library context on the current HIP device and a stream (or NULL)."""

    def __init__(self, stream_ptr: int | None = None):
        self.lib = load()
        self.h = ctypes.c_void_p()
        rc = self.lib.pbng_create(ctypes.byref(self.h), ctypes.c_void_p(stream_ptr) if stream_ptr else None)
        if rc:
            raise PbngError(rc, "pbng_create failed")

    def close(self):
        if self.h:
            self.lib.pbng_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise PbngError(rc, self.lib.pbng_last_error(self.h).decode())

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.pbng_last_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    # raw pointer calls -------------------------------------------------
    def count_raw(self, csr: Csr, kind: int, out_ptr: int, opts: Opts | None = None):
        self._check(self.lib.pbng_count(self.h, ctypes.byref(csr), kind, ctypes.byref(opts) if opts else None,
                                        ctypes.c_void_p(out_ptr)))

    def tip_raw(self, csr: Csr, side: int, out_ptr: int, opts: Opts | None = None):
        self._check(self.lib.pbng_tip(self.h, ctypes.byref(csr), side, ctypes.byref(opts) if opts else None,
                                      ctypes.c_void_p(out_ptr)))

    def wing_raw(self, csr: Csr, out_ptr: int, opts: Opts | None = None):
        self._check(self.lib.pbng_wing(self.h, ctypes.byref(csr), ctypes.byref(opts) if opts else None,
                                       ctypes.c_void_p(out_ptr)))

    # autotuner ---------------------------------------------------------------
    def autotune(self, dg, kind: int, base: Opts | None = None):
        """(best Opts, its time in ms) for kind 0 (tip U), 1 (tip V), 2 (wing)."""
        best = Opts()
        ms = ctypes.c_double()
        self._check(self.lib.pbng_autotune(self.h, ctypes.byref(dg.csr()), int(kind),
                                           ctypes.byref(base) if base else None, ctypes.byref(best), ctypes.byref(ms)))
        return best, float(ms.value)

    # learned range-bound predictor ----------------------------------------
    def predictor_load(self, path: str):
        """Load predictor parameters from a .npy file of MLP_NPARAM float32."""
        self._check(self.lib.pbng_predictor_load(self.h, os.fsencode(path)))

    def mlp_init(self, seed: int = 0):
        self._check(self.lib.pbng_mlp_init(self.h, ctypes.c_uint64(int(seed))))

    def mlp_set(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAM,):
            raise ValueError(f"expected {MLP_NPARAM} parameters, got {p.shape}")
        self._check(self.lib.pbng_mlp_set(self.h, p.ctypes.data))

    def mlp_get(self) -> np.ndarray:
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(self.lib.pbng_mlp_get(self.h, p.ctypes.data))
        return p

    def mlp_forward(self, x):
        """r_hat for the rows of a float32 cuda tensor [n, 8]."""
        import torch

        x = x.contiguous()
        y = torch.empty(max(x.shape[0], 1), dtype=torch.float32, device=x.device)
        self._check(self.lib.pbng_mlp_forward(self.h, x.data_ptr(), x.shape[0], y.data_ptr()))
        return y[: x.shape[0]]

    def mlp_loss_grad(self, x, r, wt):
        import torch

        x, r, wt = x.contiguous(), r.contiguous(), wt.contiguous()
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        self._check(self.lib.pbng_mlp_loss_grad(self.h, x.data_ptr(), r.data_ptr(), wt.data_ptr(), x.shape[0],
                                                g.data_ptr(), ctypes.byref(loss)))
        return float(loss.value), g

    def mlp_train(self, x, r, wt, batch=4096, epochs=1, lr=1e-3):
        x, r, wt = x.contiguous(), r.contiguous(), wt.contiguous()
        out = np.zeros(max(int(epochs), 1), dtype=np.float32)
        self._check(self.lib.pbng_mlp_train(self.h, x.data_ptr(), r.data_ptr(), wt.data_ptr(), x.shape[0], int(batch),
                                            int(epochs), ctypes.c_float(lr), out.ctypes.data))
        return out[: int(epochs)]


# ---------------------------------------------------------------- graphs

class DeviceGraph:
    """A U-side CSR resident in device memory (torch tensors as storage)."""

    def __init__(self, n_u, n_v, row_ptr, col_idx):
        import torch

        self.n_u, self.n_v = int(n_u), int(n_v)
        self.row_ptr = torch.as_tensor(np.ascontiguousarray(row_ptr, dtype=np.int64)).to("cuda")
        self.col_idx = torch.as_tensor(np.ascontiguousarray(col_idx, dtype=np.int32)).to("cuda")
        self.m = int(self.col_idx.numel())

    @classmethod
    def from_graph(cls, g):
        return cls(g.n_u, g.n_v, g.row_ptr, g.col_idx)

    def csr(self) -> Csr:
        c = Csr()
        c.n_u, c.n_v, c.m = self.n_u, self.n_v, self.m
        c.row_ptr = self.row_ptr.data_ptr()
        c.col_idx = self.col_idx.data_ptr() if self.m else 0
        c.on_device = 1
        return c


def host_csr(n_u, n_v, row_ptr: np.ndarray, col_idx: np.ndarray) -> Csr:
    c = Csr()
    c.n_u, c.n_v, c.m = int(n_u), int(n_v), int(col_idx.shape[0])
    c.row_ptr = row_ptr.ctypes.data
    c.col_idx = col_idx.ctypes.data if col_idx.shape[0] else 0
    c.on_device = 0
    return c


def _out_tensor(n):
    import torch

    return torch.zeros(max(int(n), 1), dtype=torch.uint64, device="cuda")


def count(ctx: Context, dg: DeviceGraph, kind: int, opts: Opts | None = None):
    n = dg.n_u if kind == COUNT_VERTEX_U else (dg.n_v if kind == COUNT_VERTEX_V else dg.m)
    out = _out_tensor(n)
    ctx.count_raw(dg.csr(), kind, out.data_ptr(), opts)
    return out[:n]


def tip(ctx: Context, dg: DeviceGraph, side: int, opts: Opts | None = None):
    n = dg.n_u if side == SIDE_U else dg.n_v
    out = _out_tensor(n)
    ctx.tip_raw(dg.csr(), side, out.data_ptr(), opts)
    return out[:n]


def tip_components(ctx: Context, dg: DeviceGraph, side: int, theta, k: int):
    """k-tips of one side from its tip numbers (uint64 device tensor): int32
    device tensor, smallest vertex id of each vertex's k-tip or -1."""
    import torch

    n = dg.n_u if side == SIDE_U else dg.n_v
    out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    ctx._check(ctx.lib.pbng_tip_components(ctx.h, ctypes.byref(dg.csr()), side, ctypes.c_void_p(theta.data_ptr()),
                                           ctypes.c_uint64(int(k)), ctypes.c_void_p(out.data_ptr())))
    return out[:n]


def wing_components(ctx: Context, dg: DeviceGraph, theta, k: int):
    """k-wings from the wing numbers (uint64 device tensor): int32 device
    tensor, smallest edge id of each edge's k-wing or -1."""
    import torch

    out = torch.empty(max(dg.m, 1), dtype=torch.int32, device="cuda")
    ctx._check(ctx.lib.pbng_wing_components(ctx.h, ctypes.byref(dg.csr()), ctypes.c_void_p(theta.data_ptr()),
                                            ctypes.c_uint64(int(k)), ctypes.c_void_p(out.data_ptr())))
    return out[: dg.m]


def tip_hinted(ctx: Context, dg: DeviceGraph, side: int, hint, opts: Opts | None = None):
    """Tip numbers of one side with learned bounds from predicted tip numbers
    `hint` (uint64 device tensor of the side's size)."""
    n = dg.n_u if side == SIDE_U else dg.n_v
    out = _out_tensor(n)
    ctx._check(ctx.lib.pbng_tip_hinted(ctx.h, ctypes.byref(dg.csr()), side, ctypes.byref(opts) if opts else None,
                                       ctypes.c_void_p(hint.data_ptr()), ctypes.c_void_p(out.data_ptr())))
    return out[:n]


def tip_schedule(ctx: Context, dg: DeviceGraph, side: int, opts: Opts | None = None, bounds_cap: int = 1 << 16):
    """(tip numbers, partition ids, supports at partition start, partition
    upper bounds) of one side, as uint64 / int32 device tensors."""
    import torch

    n = dg.n_u if side == SIDE_U else dg.n_v
    tip_t = _out_tensor(n)
    part = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    init = _out_tensor(n)
    bounds = _out_tensor(bounds_cap)
    np_out = ctypes.c_int32()
    ctx._check(ctx.lib.pbng_tip_schedule(ctx.h, ctypes.byref(dg.csr()), side, ctypes.byref(opts) if opts else None,
                                         ctypes.c_void_p(tip_t.data_ptr()), ctypes.c_void_p(part.data_ptr()),
                                         ctypes.c_void_p(init.data_ptr()), ctypes.c_void_p(bounds.data_ptr()),
                                         int(bounds_cap), ctypes.byref(np_out)))
    k = min(int(np_out.value), int(bounds_cap))
    return tip_t[:n], part[:n], init[:n], bounds[:k], int(np_out.value)


def _batch(ctx: Context, graphs, kind: int, side: int, opts: Opts | None):
    ng = len(graphs)
    descs = (Csr * max(ng, 1))()
    outs = []
    for k, dg in enumerate(graphs):
        descs[k] = dg.csr()
        n = dg.m if kind == 1 else (dg.n_u if side == SIDE_U else dg.n_v)
        outs.append(_out_tensor(n))
    ptrs = (ctypes.c_void_p * max(ng, 1))(*[t.data_ptr() for t in outs])
    o = ctypes.byref(opts) if opts else None
    if kind == 1:
        rc = ctx.lib.pbng_wing_batch(ctx.h, ctypes.cast(descs, ctypes.c_void_p), ng, o, ctypes.cast(ptrs, ctypes.c_void_p))
    else:
        rc = ctx.lib.pbng_tip_batch(ctx.h, ctypes.cast(descs, ctypes.c_void_p), ng, side, o,
                                    ctypes.cast(ptrs, ctypes.c_void_p))
    ctx._check(rc)
    return [t[: (dg.m if kind == 1 else (dg.n_u if side == SIDE_U else dg.n_v))] for t, dg in zip(outs, graphs)]


def tip_batch(ctx: Context, graphs, side: int, opts: Opts | None = None):
    """Tip numbers of one side of every DeviceGraph in `graphs` (one call)."""
    return _batch(ctx, graphs, 0, side, opts)


def wing_batch(ctx: Context, graphs, opts: Opts | None = None):
    """Wing numbers of every edge of every DeviceGraph in `graphs` (one call)."""
    return _batch(ctx, graphs, 1, 0, opts)


def tip_features(ctx: Context, dg: DeviceGraph, side: int):
    """The predictor's 8 features of every vertex of one side (float32 [n, 8])."""
    import torch

    n = dg.n_u if side == SIDE_U else dg.n_v
    out = torch.zeros((max(n, 1), 8), dtype=torch.float32, device="cuda")
    ctx._check(ctx.lib.pbng_tip_features(ctx.h, ctypes.byref(dg.csr()), side, ctypes.c_void_p(out.data_ptr())))
    return out[:n]


def wing(ctx: Context, dg: DeviceGraph, opts: Opts | None = None):
    out = _out_tensor(dg.m)
    ctx.wing_raw(dg.csr(), out.data_ptr(), opts)
    return out[: dg.m]


def to_numpy_u64(t) -> np.ndarray:
    """uint64 device tensor -> numpy (via int64 view: torch lacks uint64 copies on some builds)."""
    import torch

    return t.view(torch.int64).cpu().numpy().view(np.uint64)
