"""Oracle of the learned coarse-grained bound predictor, in numpy float64.

Test infrastructure: only tests, the smoke entry point and the benchmark's
CPU baseline use it; the library never does.

The predictor replaces the work-estimate proxy of the range determination
(Section 3.1.3: the partition bounds are picked from the current supports,
which overshoot; the scaling factor corrects that after the fact) by an
estimate of each vertex's final tip number, theta_hat = r_hat * support,
where r_hat in [0, 1] comes from a small multilayer perceptron on per-vertex
features.  The bounds only change the schedule: every tip number stays exact
(Lemmas 3-4 hold for any increasing bounds).

Network: 8 inputs -> 64 -> 64 -> 64 (ReLU) -> 1 (sigmoid); 8961 parameters
in one flat float32 vector laid out as
    W1[64][8], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4
(row-major, output index first).  Loss: weighted mean squared error
    L = sum_s wt_s (y_hat_s - y_s)^2 / sum_s wt_s.
Optimiser: Adam (Kingma and Ba, 2015) with bias correction.

Features of vertex x on side X (d = degree, w = sum of its neighbours'
degrees, dmax/dmin = largest/smallest neighbour degree, S = butterfly support
of x, Smax/Wmax = maxima of S and w over side X, m = edges, L = log1p):
    f0 = L(d)/8, f1 = L(S)/32, f2 = L(w)/16, f3 = L(dmax)/12, f4 = L(dmin)/12,
    f5 = L(S)/L(Smax), f6 = L(w)/L(Wmax), f7 = L(m)/24
(0 where a quotient's divisor is 0; a vertex of degree 0 has f0..f6 = 0).
Label: r = theta / S (0 when S = 0).
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 64
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("w4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
assert NPARAM == 8961


def unpack(p):
    """Views of the flat parameter vector by name."""
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = p[o:o + k].reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            d[name] = np.zeros(shp)
        else:
            fan_in = shp[1] if len(shp) == 2 else shp[0]
            lim = np.sqrt(6.0 / fan_in)
            d[name] = rng.uniform(-lim, lim, size=shp)
    return pack(d)


def forward(p, X):
    """r_hat for every row of X [n, 8]; also the activations."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ q["W3"].T + q["b3"]
    h3 = np.maximum(z3, 0.0)
    z4 = h3 @ q["w4"] + q["b4"][0]
    y = 1.0 / (1.0 + np.exp(-z4))
    return y, (X, z1, h1, z2, h2, z3, h3, z4, y)


def loss(p, X, Y, Wt):
    y, _ = forward(p, X)
    Wt = np.asarray(Wt, dtype=np.float64)
    return float(np.sum(Wt * (y - Y) ** 2) / np.sum(Wt))


def loss_grad(p, X, Y, Wt):
    """Loss and its gradient by reverse-mode differentiation (chain rule)."""
    q = unpack(p)
    y, (X, z1, h1, z2, h2, z3, h3, z4, _) = forward(p, X)
    Y = np.asarray(Y, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    ws = np.sum(Wt)
    L = float(np.sum(Wt * (y - Y) ** 2) / ws)
    dz4 = 2.0 * Wt * (y - Y) / ws * y * (1.0 - y)
    g = {"w4": h3.T @ dz4, "b4": np.array([dz4.sum()])}
    dz3 = np.outer(dz4, q["w4"]) * (z3 > 0)
    g["W3"], g["b3"] = dz3.T @ h2, dz3.sum(0)
    dz2 = (dz3 @ q["W3"]) * (z2 > 0)
    g["W2"], g["b2"] = dz2.T @ h1, dz2.sum(0)
    dz1 = (dz2 @ q["W2"]) * (z1 > 0)
    g["W1"], g["b1"] = dz1.T @ X, dz1.sum(0)
    return L, pack(g)


def adam_step(p, m, v, t, g, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(g, side, support):
    """The 8 features of every vertex of one side (module docstring)."""
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    ci = np.asarray(g.col_idx, dtype=np.int64)
    du = np.diff(rp)
    dv = np.bincount(ci, minlength=g.n_v).astype(np.int64)
    if side == 0:
        nx, xdeg, ydeg = g.n_u, du, dv
        rows = np.repeat(np.arange(g.n_u), du)
        nb = ci
    else:
        nx, xdeg, ydeg = g.n_v, dv, du
        rows = ci
        nb = np.repeat(np.arange(g.n_u), du)
    S = np.asarray(support, dtype=np.float64)
    w = np.zeros(nx)
    np.add.at(w, rows, ydeg[nb].astype(np.float64))
    dmax = np.zeros(nx)
    np.maximum.at(dmax, rows, ydeg[nb].astype(np.float64))
    dmin = np.full(nx, np.inf)
    np.minimum.at(dmin, rows, ydeg[nb].astype(np.float64))
    dmin[xdeg == 0] = 0.0
    L = np.log1p
    Smax = S.max() if nx else 0.0
    Wmax = w.max() if nx else 0.0
    F = np.zeros((nx, IN))
    F[:, 0] = L(xdeg) / 8
    F[:, 1] = L(S) / 32
    F[:, 2] = L(w) / 16
    F[:, 3] = L(dmax) / 12
    F[:, 4] = L(dmin) / 12
    F[:, 5] = L(S) / L(Smax) if Smax > 0 else 0.0
    F[:, 6] = L(w) / L(Wmax) if Wmax > 0 else 0.0
    F[:, 7] = L(float(g.m)) / 24
    F[xdeg == 0, :7] = 0.0
    return F


def labels(theta, support):
    theta = np.asarray(theta, dtype=np.float64)
    S = np.asarray(support, dtype=np.float64)
    return np.where(S > 0, theta / np.where(S > 0, S, 1.0), 0.0)
