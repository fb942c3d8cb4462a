"""CPU reference of the task cost model (float64 numpy). TEST INFRASTRUCTURE ONLY.

Model: multilayer perceptron 6 -> 32 -> 32 -> 1 with ReLU hidden layers,
parameters packed as W1[32][6] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3
(1313 values):

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 . h2 + b3

Loss: mean squared error L = (1/m) sum_s (y_s - t_s)^2; gradients by the
chain rule, written out layer by layer (no autodiff library).
Optimiser: Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization",
ICLR 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
Features of a task (u, v), each log2(1 + x), from the lengths of the two
lists its merge walks (the sweep of Fig. 5 needs, of N(u), only the ids above
u, and of N(v) only the ids from u on, Sec. 6): a = |{w in N(u): w > u}|,
b = |{w in N(v): w >= u}|, a + b, min(a, b), max(a, b), and the number of
entries of N(u) above v.

These are not census arithmetic: the census counts never depend on the model.
Parity of the GPU kernels with this reference is to a floating-point
tolerance (float32 sums in a different order).
"""
from __future__ import annotations

import numpy as np

NI, NH = 6, 32
SHAPES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", ())]
NP = NH * NI + NH + NH * NH + NH + NH + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == NP
    out, p = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp)) if shp else 1
        out[name] = w[p:p + k].reshape(shp) if shp else w[p]
        p += k
    return out


def pack(parts):
    return np.concatenate([np.atleast_1d(np.asarray(parts[n], dtype=np.float64)).ravel() for n, _ in SHAPES])


def forward(w, X):
    P = unpack(w)
    X = np.asarray(X, dtype=np.float64).reshape(-1, NI)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    return h2 @ P["W3"] + P["b3"]


def loss_grad(w, X, t):
    """Mean squared error and its gradient with respect to the packed parameters."""
    P = unpack(w)
    X = np.asarray(X, dtype=np.float64).reshape(-1, NI)
    t = np.asarray(t, dtype=np.float64).ravel()
    m = X.shape[0]
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ P["W3"] + P["b3"]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / m                       # dL/dy_s
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dh2 = np.outer(dy, P["W3"]) * (a2 > 0)  # through relu
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0)
    gW1 = dh1.T @ X
    gb1 = dh1.sum(axis=0)
    return loss, pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3})


def grad_magnitude(w, X, t):
    """Per parameter, a bound on the size of every quantity that enters its
    gradient: loss_grad's chain rule with each factor replaced by its magnitude,
    the forward values by the sums of the magnitudes of their terms, and the
    residual y - t by |y - t| + |y|'s term magnitudes + |t| (the residual of a
    rounded y is off by a fraction of those, not of |y - t|). A float32
    evaluation sums the same products in some order, so its rounding error is
    at most (depth * 2^-24) times this, depth being the longest chain of
    roundings (the dot products of the forward and backward passes, the sum
    over samples, the activations)."""
    P = unpack(w)
    X = np.asarray(X, dtype=np.float64).reshape(-1, NI)
    t = np.asarray(t, dtype=np.float64).ravel()
    m = X.shape[0]
    a1 = X @ P["W1"].T + P["b1"]
    a2 = np.maximum(a1, 0.0) @ P["W2"].T + P["b2"]
    y = np.maximum(a2, 0.0) @ P["W3"] + P["b3"]
    aX, aW1, aW2, aW3 = np.abs(X), np.abs(P["W1"]), np.abs(P["W2"]), np.abs(P["W3"])
    h1m = (aX @ aW1.T + np.abs(P["b1"])) * (a1 > 0)
    h2m = (h1m @ aW2.T + np.abs(P["b2"])) * (a2 > 0)
    ym = h2m @ aW3 + abs(P["b3"])
    dy = 2.0 * (np.abs(y - t) + ym + np.abs(t)) / m
    gW3 = h2m.T @ dy
    gb3 = dy.sum()
    dh2 = np.outer(dy, aW3) * (a2 > 0)
    gW2 = dh2.T @ h1m
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ aW2) * (a1 > 0)
    gW1 = dh1.T @ aX
    gb1 = dh1.sum(axis=0)
    return pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3})


def adam_step(w, m1, m2, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mhat = m1 / (1 - b1 ** t)
    vhat = m2 / (1 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def task_features(offsets, nbrs):
    """Features of every task (u, v), u < v, in CSR order."""
    off = np.asarray(offsets, dtype=np.int64)
    nb = np.asarray(nbrs, dtype=np.int64)
    n = off.size - 1
    d = np.diff(off)
    rows = np.repeat(np.arange(n, dtype=np.int64), d)
    j = np.flatnonzero(nb > rows)
    u, v = rows[j], nb[j]
    # (row, id) pairs in CSR order are sorted, so a count of the ids of a row
    # above (or from) a value is a difference of two sorted-search positions
    key = rows * n + nb
    a = off[u + 1] - np.searchsorted(key, u * n + u, side="right")  # ids of N(u) above u
    b = off[v + 1] - np.searchsorted(key, v * n + u, side="left")   # ids of N(v) from u on
    above = off[u + 1] - j - 1
    F = np.stack([a, b, a + b, np.minimum(a, b), np.maximum(a, b), above], axis=1).astype(np.float64)
    return np.log2(1.0 + F)
