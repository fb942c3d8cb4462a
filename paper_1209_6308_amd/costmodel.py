"""Learned task-cost model for scheduling the census (argument marshalling only).

The model (an FP32 MLP 6 -> 32 -> 32 -> 1, see include/triad.h) is trained on
the GPU by the library's own kernels (triad_mlp_train) on per-task cycle counts
that the census kernel records (triad_opts.task_cycles), and then used by the
census to bin and order the tasks (schedule="learned"). Ordering by the
merge length d+(u) + d(v) - s(u, v) (schedule="heuristic": d+(u) the ids of
N(u) above u, s the ids of N(v) below u) is its fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import graphs, triad

_CACHE = {}


def init_weights(seed: int = 1, b3: float = 12.0) -> np.ndarray:
    """He-normal hidden weights, zero biases, output bias b3 (log2 cycles)."""
    rng = np.random.default_rng(seed)
    H, I = triad.MLP_HIDDEN, triad.MLP_IN
    w1 = rng.normal(0.0, np.sqrt(2.0 / I), size=(H, I))
    w2 = rng.normal(0.0, np.sqrt(2.0 / H), size=(H, H))
    w3 = rng.normal(0.0, np.sqrt(1.0 / H), size=H)
    return np.concatenate([w1.ravel(), np.zeros(H), w2.ravel(), np.zeros(H), w3, [b3]]).astype(np.float32)


def features(g, device="cuda", stream=None):
    """Device float32 [tasks, 6] features of every task in CSR order."""
    import torch
    d_off, d_nbr, _ = triad.to_device(g, device)
    nt = ctypes.c_int64(0)
    triad._check(triad.lib().triad_task_features(g.n, g.nnz, triad._tp(d_off), triad._tp(d_nbr),
                                                 triad._stream(stream), None, ctypes.byref(nt)))
    feat = torch.empty((max(nt.value, 1), triad.MLP_IN), dtype=torch.float32, device=device)
    triad._check(triad.lib().triad_task_features(g.n, g.nnz, triad._tp(d_off), triad._tp(d_nbr),
                                                 triad._stream(stream), triad._tp(feat), ctypes.byref(nt)))
    return feat[: nt.value]


def record_cycles(g, device="cuda", stream=None, **kw):
    """Per-task wavefront cycle counts (CSR task order) from one census;
    0 for tasks split into chunks (not timed)."""
    import torch
    d = triad.to_device(g, device)
    cyc = torch.zeros(max(g.nnz // 2, 1), dtype=torch.int32, device=device)  # uint32 counts < 2^31
    triad.triad_census_device(g.n, g.nnz, *d, stream=stream, task_cycles=cyc, **kw)
    return cyc[: g.nnz // 2]


def forward(w, X, stream=None):
    import torch
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    triad._check(triad.lib().triad_mlp_forward(triad._tp(w), triad._tp(X), X.shape[0], triad._tp(y),
                                               triad._stream(stream)))
    return y


def loss_grad(w, X, t, stream=None):
    import torch
    g = torch.empty(triad.MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    triad._check(triad.lib().triad_mlp_loss_grad(triad._tp(w), triad._tp(X), triad._tp(t), X.shape[0],
                                                 triad._tp(g), triad._tp(loss), triad._stream(stream)))
    return float(loss.item()), g


def adam(w, m1, m2, g, step, lr, stream=None):
    triad._check(triad.lib().triad_mlp_adam(triad._tp(w), triad._tp(m1), triad._tp(m2), triad._tp(g), step,
                                            ctypes.c_float(lr), triad._stream(stream)))


def train(X, t, w0=None, epochs=30, batch=8192, lr=3e-3, seed=1, stream=None):
    """Minibatch Adam on the GPU; returns (weights tensor, per-epoch mean loss)."""
    import torch
    if w0 is None:
        w0 = init_weights(seed, b3=float(t.float().mean().item()))
    w = torch.as_tensor(w0, dtype=torch.float32).to(X.device).clone()
    hist = torch.zeros(epochs, dtype=torch.float32, device=X.device)
    triad._check(triad.lib().triad_mlp_train(triad._tp(w), triad._tp(X), triad._tp(t), X.shape[0], epochs, batch,
                                             ctypes.c_float(lr), seed, triad._stream(stream), triad._tp(hist)))
    return w, hist.cpu().numpy()


def training_set(names=("rmat10", "rmat20"), max_samples=1 << 21, seed=3, device="cuda", stream=None):
    """(features, log2 cycles) of the timed tasks of the given workloads."""
    import torch
    Xs, ts = [], []
    for name in names:
        g = graphs.workload(name)
        cyc = record_cycles(g, device, stream)
        X = features(g, device, stream)
        keep = cyc > 0
        Xs.append(X[keep])
        ts.append(torch.log2(cyc[keep].double()).float())
    X = torch.cat(Xs)
    t = torch.cat(ts)
    if X.shape[0] > max_samples:
        gen = torch.Generator(device="cpu").manual_seed(seed)
        idx = torch.randperm(X.shape[0], generator=gen)[:max_samples].to(device)
        X, t = X[idx], t[idx]
    return X.contiguous(), t.contiguous()


def affine_fit(X, t):
    """Least-squares coefficients (slope, intercept) of the best affine
    predictor of log2 cycles from log2(1 + merge length), the heuristic's key
    (feature 2)."""
    x = X[:, 2].double().cpu().numpy()
    y = t.double().cpu().numpy()
    A = np.stack([x, np.ones_like(x)], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    return coef


def affine_mse(coef, X, t):
    x = X[:, 2].double().cpu().numpy()
    r = coef[0] * x + coef[1] - t.double().cpu().numpy()
    return float(np.mean(r * r))


def affine_baseline_mse(X, t):
    """Mean squared error of the best affine predictor of log2 cycles from
    log2(1 + merge length) (the heuristic's key), fitted on the same samples."""
    return affine_mse(affine_fit(X, t), X, t)


def model_mse(w, X, t, stream=None):
    """Mean squared error of the network's predicted log2 cycles."""
    return float(((forward(w, X, stream) - t) ** 2).double().mean().item())


def held_out_report(w, g, stream=None):
    """The trained network and the affine fit of the training samples, both
    evaluated on the per-task cycles of another graph g (not trained on)."""
    import torch
    e = next((v for (dev, ep), v in _CACHE.items()), None)
    cyc = record_cycles(g, stream=stream)
    X = features(g, stream=stream)
    keep = cyc > 0
    X, t = X[keep].contiguous(), torch.log2(cyc[keep].double()).float().contiguous()
    out = {"graph": g.name, "tasks": int(X.shape[0]), "network_mse": model_mse(w, X, t, stream)}
    if e is not None and len(e) > 3:
        out["affine_len_mse"] = affine_mse(e[3], X, t)
    return out


def load_or_train(stream=None, device="cuda", epochs=30):
    """Weights trained on R-MAT scale 10 and scale 20 cycle counts (cached per
    process)."""
    key = (device, epochs)
    if key not in _CACHE:
        X, t = training_set(device=device, stream=stream)
        w, hist = train(X, t, epochs=epochs, stream=stream)
        coef = affine_fit(X, t)
        _CACHE[key] = (w, hist, affine_mse(coef, X, t), coef)
    return _CACHE[key][0]


def last_training_report(device="cuda", epochs=30):
    e = _CACHE.get((device, epochs))
    if e is None:
        return None
    return {"final_mse": float(e[1][-1]), "affine_len_mse": e[2], "epochs": epochs}
