"""Training of the learned range-bound predictor on the GPU.

Rows are vertices of seeded synthetic training graphs: the predictor's eight
features (``tip_features``) and the target r = theta / support, where theta
comes from the library's exact tip decomposition and the support from its
counting (vertices without butterflies are left out: their tip number is 0
whatever the prediction).  Training runs the library's own forward, backward
and Adam kernels (``Context.mlp_train``).

Training graphs: Chung-Lu bipartite graphs with m log-uniform in [1e4, 2e5],
exponent uniform in [1.8, 2.8] on both sides, |U| = m / 20, |V| = m / 100,
degree cap 50000 clipped per side to the other side's size, seeds 40000 + i.

    python -m paper_2110_12511_amd.predictor --graphs 2000 --epochs 8 --out predictor_tip.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import binding as B

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_tip.npy")


def training_graph(i: int, seed0: int = 40000):
    """Seeded training graph number i (see the module docstring)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth

    rng = np.random.default_rng(seed0 + i)
    m = int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e5)))))
    gamma = float(rng.uniform(1.8, 2.8))
    n_u, n_v = max(m // 20, 2), max(m // 100, 2)
    return synth.chung_lu(n_u, n_v, m, gamma, 50000, seed=seed0 + i)


def rows_for_graph(ctx: B.Context, g, side: int = B.SIDE_U, P: int = 0):
    """(features [k, 8], r [k]) on the device for the vertices of one side
    that lie in at least one butterfly."""
    import torch

    dg = B.DeviceGraph.from_graph(g)
    F = B.tip_features(ctx, dg, side)
    S = B.count(ctx, dg, B.COUNT_VERTEX_U if side == B.SIDE_U else B.COUNT_VERTEX_V)
    th = B.tip(ctx, dg, side, B.make_opts(P=P))
    S64 = S.view(torch.int64).to(torch.float64)
    T64 = th.view(torch.int64).to(torch.float64)
    keep = S64 > 0
    r = (T64[keep] / S64[keep]).to(torch.float32)
    return F[keep].contiguous(), r.contiguous()


def build_dataset(ctx: B.Context, graphs, seed: int = 0, log=None):
    """Rows of all graphs, shuffled with a seeded permutation."""
    import torch

    xs, rs = [], []
    t0 = time.time()
    for k, g in enumerate(graphs):
        x, r = rows_for_graph(ctx, g)
        xs.append(x)
        rs.append(r)
        if log and (k + 1) % 100 == 0:
            log(f"[predictor] labelled {k + 1} graphs, {sum(t.shape[0] for t in rs)} rows, {time.time() - t0:.1f} s")
    X = torch.cat(xs) if xs else torch.zeros((0, 8), dtype=torch.float32, device="cuda")
    R = torch.cat(rs) if rs else torch.zeros(0, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=gen).to(X.device)
    X, R = X[perm].contiguous(), R[perm].contiguous()
    W = torch.ones_like(R)
    return X, R, W


def train(ctx: B.Context, X, R, W, epochs=8, batch=4096, lr=2e-3, seed=0, log=None):
    """Fresh network trained by minibatch Adam; returns (params, epoch losses)."""
    ctx.mlp_init(seed)
    losses = []
    for e in range(epochs):
        # step size halves over the last epochs
        lr_e = lr if e < epochs // 2 else lr * 0.5 ** (e - epochs // 2 + 1)
        losses.append(float(ctx.mlp_train(X, R, W, batch=batch, epochs=1, lr=lr_e)[0]))
        if log:
            log(f"[predictor] epoch {e + 1}/{epochs}: loss {losses[-1]:.5f}")
    return ctx.mlp_get(), losses


def save(params, path: str = DEFAULT_PATH):
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)


def load_params(path: str = DEFAULT_PATH) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.shape != (B.MLP_NPARAM,) or p.dtype != np.float32:
        raise ValueError(f"{path}: expected float32[{B.MLP_NPARAM}]")
    return p


def install(ctx: B.Context, path: str = DEFAULT_PATH) -> bool:
    """Load stored parameters into the context; False when none are stored."""
    if not os.path.exists(path):
        return False
    ctx.mlp_set(load_params(path))
    return True


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--graphs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_PATH)
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    ctx = B.Context()
    t0 = time.time()
    graphs = (training_graph(i) for i in range(args.graphs))
    X, R, W = build_dataset(ctx, graphs, log=log)
    log(f"[predictor] {X.shape[0]} rows from {args.graphs} graphs in {time.time() - t0:.1f} s")
    t1 = time.time()
    params, losses = train(ctx, X, R, W, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    log(f"[predictor] trained in {time.time() - t1:.2f} s; losses {[round(v, 5) for v in losses]}")
    save(params, args.out)
    log(f"[predictor] wrote {args.out}")


if __name__ == "__main__":
    main()
