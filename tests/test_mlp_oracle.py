"""Pins for the CPU reference of the task cost model (oracle/mlp.py):
gradients against central finite differences, closed-form forward passes, the
first Adam step, and hand-computed features of a tiny graph."""
import numpy as np

from oracle import mlp


def rand_w(seed, scale=0.5):
    return np.random.default_rng(seed).normal(0, scale, size=mlp.NP)


def test_parameter_count():
    assert mlp.NP == 1313


def test_forward_closed_forms():
    X = np.random.default_rng(0).normal(size=(5, mlp.NI))
    P = mlp.unpack(np.zeros(mlp.NP))
    P["b3"] = 7.5
    assert np.allclose(mlp.forward(mlp.pack(P), X), 7.5)
    # one path: h1_0 = relu(x_0), h2_0 = relu(h1_0), y = 2 h2_0 + 1
    P = mlp.unpack(np.zeros(mlp.NP))
    W1 = np.zeros((32, 6)); W1[0, 0] = 1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1.0
    W3 = np.zeros(32); W3[0] = 2.0
    P.update(W1=W1, W2=W2, W3=W3, b3=1.0)
    x = np.array([[3.0, 9, 9, 9, 9, 9], [-2.0, 1, 1, 1, 1, 1]])
    assert np.allclose(mlp.forward(mlp.pack(P), x), [7.0, 1.0])


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = rand_w(2)
    X = rng.normal(1.0, 1.0, size=(40, mlp.NI))
    t = rng.normal(size=40)
    loss, g = mlp.loss_grad(w, X, t)
    assert np.isclose(loss, np.mean((mlp.forward(w, X) - t) ** 2))
    h = 1e-6
    idx = rng.choice(mlp.NP, size=60, replace=False)
    idx = np.concatenate([idx, [mlp.NP - 1, 0, 192, 224, 1248]])  # b3, W1, b1, W2, b2/W3 boundaries
    for q in idx:
        e = np.zeros(mlp.NP); e[q] = h
        num = (mlp.loss_grad(w + e, X, t)[0] - mlp.loss_grad(w - e, X, t)[0]) / (2 * h)
        assert abs(num - g[q]) <= 1e-6 + 1e-5 * abs(num), (q, num, g[q])


def test_first_adam_step():
    # from zero moments the bias-corrected step is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w, m1, m2 = mlp.adam_step(np.ones(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(w, 1.0 - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_task_features_by_hand():
    # path 0-1-2 plus edge 0-2 (a triangle) and a pendant 3 on 0:
    # rows: 0:[1,2,3] 1:[0,2] 2:[0,1] 3:[0]
    off = [0, 3, 5, 7, 8]
    nb = [1, 2, 3, 0, 2, 0, 1, 0]
    F = mlp.task_features(off, nb)
    # tasks in CSR order: (0,1), (0,2), (0,3), (1,2). Of N(u) the merge walks
    # the ids above u (row 0: 1,2,3; row 1: 2), of N(v) the ids from u on
    # (N(1) from 0: 0,2; N(2) from 0: 0,1; N(3) from 0: 0; N(2) from 1: 1)
    raw = np.array([[3, 2, 5, 2, 3, 2], [3, 2, 5, 2, 3, 1], [3, 1, 4, 1, 3, 0], [1, 1, 2, 1, 1, 0]], float)
    assert np.allclose(F, np.log2(1 + raw))


def test_gradient_magnitude_bounds_the_gradient():
    """The rounding bound's magnitudes dominate the gradient element by element
    and are positive wherever a parameter takes part."""
    rng = np.random.default_rng(4)
    w = rand_w(5)
    X = rng.normal(1.0, 2.0, size=(64, mlp.NI))
    t = rng.normal(size=64)
    _, g = mlp.loss_grad(w, X, t)
    s = mlp.grad_magnitude(w, X, t)
    assert s.shape == g.shape
    assert np.all(s >= np.abs(g) * (1 - 1e-12))
    assert s[-1] > 0  # b3 takes part in every sample

