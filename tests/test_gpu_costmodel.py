"""GPU cost-model kernels against the CPU reference (oracle/mlp.py), and the
heuristic / learned schedules against the census oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1209_6308_amd import costmodel, graphs, triad

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


def test_forward_matches_reference(torch):
    rng = np.random.default_rng(0)
    w = rng.normal(0, 0.3, mlp.NP)
    X = rng.uniform(0, 20, size=(3000, mlp.NI))
    y = costmodel.forward(torch.tensor(w, dtype=torch.float32, device="cuda"),
                          torch.tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy()
    ref = mlp.forward(w.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.allclose(y, ref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("m", [1, 127, 128, 1000, 4099])
def test_gradient_matches_reference(torch, m):
    rng = np.random.default_rng(m)
    w = rng.normal(0, 0.3, mlp.NP).astype(np.float32)
    X = rng.uniform(0, 16, size=(m, mlp.NI)).astype(np.float32)
    t = rng.normal(10, 3, size=m).astype(np.float32)
    loss, g = costmodel.loss_grad(torch.tensor(w, device="cuda"), torch.tensor(X, device="cuda"),
                                  torch.tensor(t, device="cuda"))
    rl, rg = mlp.loss_grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    g = g.cpu().numpy()
    assert abs(loss - rl) <= 1e-4 * abs(rl) + 1e-6
    # per element: 1e-4 relative, plus the float32 rounding bound of that
    # element's sum of products (depth: forward dot products of 6 and 32 terms,
    # the backward one of 32, the sum over m samples, and the activations)
    depth = 6 + 32 + 32 + int(np.ceil(np.log2(max(m, 2)))) + 8
    atol = depth * 2.0 ** -24 * mlp.grad_magnitude(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    err = np.abs(g - rg)
    bound = 1e-4 * np.abs(rg) + atol
    assert np.all(err <= bound), (int(np.argmax(err / bound)), float(np.max(err / bound)))


def test_adam_matches_reference(torch):
    rng = np.random.default_rng(3)
    w = rng.normal(size=mlp.NP).astype(np.float32)
    g = rng.normal(size=mlp.NP).astype(np.float32)
    m1 = rng.normal(size=mlp.NP).astype(np.float32) * 0.1
    m2 = np.abs(rng.normal(size=mlp.NP)).astype(np.float32) * 0.1
    tw, tm1, tm2 = (torch.tensor(a, device="cuda") for a in (w, m1, m2))
    costmodel.adam(tw, tm1, tm2, torch.tensor(g, device="cuda"), 5, 0.01)
    rw, rm1, rm2 = mlp.adam_step(w.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64),
                                 g.astype(np.float64), 5, 0.01)
    assert np.allclose(tw.cpu().numpy(), rw, rtol=1e-5, atol=1e-6)
    assert np.allclose(tm1.cpu().numpy(), rm1, rtol=1e-5, atol=1e-7)
    assert np.allclose(tm2.cpu().numpy(), rm2, rtol=1e-5, atol=1e-7)


def test_features_match_reference(torch):
    g = graphs.rmat(12, 8, seed=4)
    F = costmodel.features(g).cpu().numpy()
    ref = mlp.task_features(g.offsets, g.nbrs)
    assert F.shape == ref.shape
    assert np.allclose(F, ref, atol=2e-6 * 32)


def test_cycle_recording(torch):
    g = graphs.rmat(12, 8, seed=4)
    cyc = costmodel.record_cycles(g, hub_threshold=-1).cpu().numpy().astype(np.int64)
    assert cyc.size == g.nnz // 2
    assert np.all(cyc > 0)
    # longer merges take longer on average
    F = mlp.task_features(g.offsets, g.nbrs)
    r = np.corrcoef(F[:, 2], np.log2(cyc))[0, 1]
    assert r > 0.3, r


def test_cycle_recording_under_a_schedule(torch):
    """With a schedule the queue is reordered, but the cycles still come back
    indexed by CSR task: they correlate with the task's own features."""
    g = graphs.rmat(12, 8, seed=4)
    cyc = costmodel.record_cycles(g, hub_threshold=-1, schedule="heuristic", tail_share=-1).cpu().numpy().astype(np.int64)
    assert cyc.size == g.nnz // 2
    assert np.all(cyc > 0)
    F = mlp.task_features(g.offsets, g.nbrs)
    r = np.corrcoef(F[:, 2], np.log2(cyc))[0, 1]
    assert r > 0.3, r


@pytest.mark.parametrize("schedule", ["heuristic", "learned"])
def test_schedules_exact(torch, schedule):
    g = graphs.rmat(13, 8, seed=6, recip_p=0.2)
    want = oracle.census(g)
    d = triad.to_device(g)
    kw = {}
    if schedule == "learned":
        w = torch.tensor(costmodel.init_weights(2), device="cuda")
        kw["model"] = w
    # hub 0: the default threshold; 64: a long-task list of most tasks, many
    # of them split; -1: no hub split (the learned schedule still lists the
    # tasks above its own threshold)
    # tail_share -1: the last batches are always reordered; 0: only when the
    # keys predict a costly batch at the end
    for hub in (0, 64, -1):
        for share in (-1, 0):
            got, st, tm = triad.triad_census_device(g.n, g.nnz, *d, schedule=schedule, hub_threshold=hub, chunk=256,
                                                    tail_share=share, **kw)
            assert got == want, (hub, share)


def test_wave_spans(torch):
    g = graphs.rmat(12, 8, seed=4)
    d = triad.to_device(g)
    span = torch.zeros((4096, 2), dtype=torch.int64, device="cuda")
    got, st, tm = triad.triad_census_device(g.n, g.nnz, *d, grid_groups=64, waves_per_group=1, wave_span=span)
    assert tm["waves"] == 64
    s = span[:64].cpu().numpy()
    assert np.all(s[:, 1] >= s[:, 0]) and np.all(s[:, 0] > 0)


def test_training_beats_degree_heuristic(torch):
    """What the trained network gains: a lower prediction error of per-task
    log2 cycles than the best affine fit of log2(merge length), the heuristic's key."""
    Xs, ts = [], []
    for g in (graphs.workload("rmat10"), graphs.rmat(15, 16, seed=2, recip_p=0.1)):
        cyc = costmodel.record_cycles(g)
        X = costmodel.features(g)
        keep = cyc > 0
        Xs.append(X[keep]); ts.append(torch.log2(cyc[keep].double()).float())
    X, t = torch.cat(Xs).contiguous(), torch.cat(ts).contiguous()
    w, hist = costmodel.train(X, t, epochs=25, batch=4096, lr=3e-3)
    assert hist[-1] < hist[0]
    mse = float(((costmodel.forward(w, X) - t) ** 2).mean().item())
    base = costmodel.affine_baseline_mse(X, t)
    assert mse < base, (mse, base)


def test_trained_network_on_held_out_graphs(torch):
    """Trained on the cycles of two R-MAT graphs, the network predicts the
    per-task cycles of graphs it never saw (another R-MAT seed, a Chung-Lu
    graph) better than the affine fit of log2(merge length) made on the same
    training samples."""
    Xs, ts = [], []
    for g in (graphs.workload("rmat10"), graphs.rmat(15, 16, seed=2, recip_p=0.1)):
        cyc = costmodel.record_cycles(g)
        X = costmodel.features(g)
        keep = cyc > 0
        Xs.append(X[keep]); ts.append(torch.log2(cyc[keep].double()).float())
    X, t = torch.cat(Xs).contiguous(), torch.cat(ts).contiguous()
    w, hist = costmodel.train(X, t, epochs=25, batch=4096, lr=3e-3)
    coef = costmodel.affine_fit(X, t)
    for h in (graphs.rmat(14, 16, seed=9), graphs.chung_lu(1 << 14, 2.1, 16.0, 2048.0, seed=4)):
        cyc = costmodel.record_cycles(h)
        Xh = costmodel.features(h)
        keep = cyc > 0
        Xh, th = Xh[keep].contiguous(), torch.log2(cyc[keep].double()).float().contiguous()
        net = costmodel.model_mse(w, Xh, th)
        aff = costmodel.affine_mse(coef, Xh, th)
        assert net < aff, (h.n, net, aff)

