"""Pins of the predictor oracle (oracle/mlp.py) to facts outside itself:
finite differences for the gradient, hand-built networks with known outputs
and a hand-computed loss,
Adam's bias-corrected steps under a constant gradient, and closed-form
features of complete bipartite graphs."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
import synth


def rand_data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.5, 1.5, size=(n, mlp.IN))
    Y = rng.uniform(0, 1, size=n)
    Wt = rng.uniform(0.5, 2.0, size=n)
    return X, Y, Wt


def test_param_count():
    assert mlp.NPARAM == 8 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1 == 8961


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    p = mlp.init(seed)
    p[mlp.NPARAM - 1] = 0.3  # b4 away from 0 so the sigmoid slope varies
    X, Y, Wt = rand_data(37, seed + 10)
    _, g = mlp.loss_grad(p, X, Y, Wt)
    rng = np.random.default_rng(seed)
    # indices in every block of the layout
    offs, o = [], 0
    for _, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        offs += list(o + rng.choice(k, size=min(k, 12), replace=False))
        o += k
    eps = 1e-6
    for i in offs:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (mlp.loss(pp, X, Y, Wt) - mlp.loss(pm, X, Y, Wt)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_constant_network():
    p = np.zeros(mlp.NPARAM)
    p[-1] = 0.7
    X, _, _ = rand_data(5, 3)
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, 1 / (1 + math.exp(-0.7)))


@pytest.mark.parametrize("b4,expected", [(0.0, 1.0 / 15.0), (math.log(3.0), 2.1875 / 15.0)])
def test_loss_of_constant_network(b4, expected):
    """A network whose only nonzero parameter is the output bias predicts
    sigmoid(b4) for every row: 0.5 at b4 = 0 and 0.75 at b4 = ln 3.  With
    labels (0, 1, 1/4, 1/2) and row weights (1, 2, 4, 8) the weighted mean
    squared error is, by hand, (1/4 + 2/4 + 4/16 + 0) / 15 = 1/15 and
    (9/16 + 2/16 + 4/4 + 8/16) / 15 = 2.1875/15.  An unweighted mean (1/4),
    an absolute error (2.5/15) or a sum without the division would differ."""
    p = np.zeros(mlp.NPARAM)
    p[-1] = b4
    X = np.random.default_rng(4).uniform(-1, 2, size=(4, mlp.IN))
    Y = np.array([0.0, 1.0, 0.25, 0.5])
    Wt = np.array([1.0, 2.0, 4.0, 8.0])
    assert mlp.loss(p, X, Y, Wt) == pytest.approx(expected, rel=1e-12)
    assert mlp.loss_grad(p, X, Y, Wt)[0] == pytest.approx(expected, rel=1e-12)
    # the loss is a weighted mean: scaling every weight leaves it unchanged
    assert mlp.loss(p, X, Y, 3.0 * Wt) == pytest.approx(expected, rel=1e-12)


def test_forward_hand_built_path():
    """Unit 5 of layer 1 reads input 2; unit 7 of layer 2 reads it x2; unit 1
    of layer 3 reads that x3; the output reads unit 1: y = sigmoid(6 relu(x2))."""
    d = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    d["W1"][5, 2] = 1.0
    d["W2"][7, 5] = 2.0
    d["W3"][1, 7] = 3.0
    d["w4"][1] = 1.0
    p = mlp.pack(d)
    X = np.zeros((4, mlp.IN))
    X[:, 2] = [-1.0, 0.0, 0.25, 1.0]
    X[:, 5] = 9.0  # an input no path reads
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, 1 / (1 + np.exp(-6 * np.maximum(X[:, 2], 0))))


def test_adam_constant_gradient_steps():
    """With a constant gradient, bias correction makes every step lr * g / (|g| + eps)."""
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    lr = 0.01
    for t in range(1, 6):
        p2, m, v = mlp.adam_step(p, m, v, t, g, lr)
        assert np.allclose(p2 - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-12)
        p = p2


@pytest.mark.parametrize("a,b", [(2, 3), (5, 4), (7, 9)])
def test_features_complete_bipartite(a, b):
    g = synth.complete(a, b)
    S = oracle.count_vertex(g)[0]
    F = mlp.features(g, 0, S)
    L = math.log1p
    Sx = (a - 1) * b * (b - 1) // 2
    exp = [L(b) / 8, L(Sx) / 32, L(a * b) / 16, L(a) / 12, L(a) / 12, 1.0 if Sx else 0.0, 1.0, L(a * b) / 24]
    assert np.allclose(F, np.array(exp)[None, :])
    Fv = mlp.features(g, 1, oracle.count_vertex(g)[1])
    Sy = (b - 1) * a * (a - 1) // 2
    expv = [L(a) / 8, L(Sy) / 32, L(a * b) / 16, L(b) / 12, L(b) / 12, 1.0 if Sy else 0.0, 1.0, L(a * b) / 24]
    assert np.allclose(Fv, np.array(expv)[None, :])


def test_features_isolated_and_star():
    # U0 -- V0..V2 (a star), U1 isolated, U2 -- V0
    g = synth.from_edges(3, 3, [(0, 0), (0, 1), (0, 2), (2, 0)])
    S = oracle.count_vertex(g)[0]
    F = mlp.features(g, 0, S)
    L = math.log1p
    assert np.allclose(F[1], [0] * 7 + [L(4) / 24])
    # U0: d=3, neighbour degrees 2,1,1 -> w=4, dmax=2, dmin=1, no butterflies
    assert np.allclose(F[0], [L(3) / 8, 0, L(4) / 16, L(2) / 12, L(1) / 12, 0, 1.0, L(4) / 24])
    assert np.allclose(F[2], [L(1) / 8, 0, L(2) / 16, L(2) / 12, L(2) / 12, 0, L(2) / L(4), L(4) / 24])


def test_labels_complete_and_bounds():
    g = synth.complete(4, 6)
    S = oracle.count_vertex(g)[0]
    assert np.allclose(mlp.labels(oracle.tip(g, 0), S), 1.0)
    g = synth.chung_lu(3000, 800, 20000, 2.2, 400, seed=9)
    S = oracle.count_vertex(g)[0]
    r = mlp.labels(oracle.tip(g, 0), S)
    assert (r >= 0).all() and (r <= 1).all()
    assert (r[S == 0] == 0).all()
