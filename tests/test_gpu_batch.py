"""Batched census (one captured hipGraph over many graphs) against the oracle,
graph by graph, bit-exact."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1209_6308_amd import graphs, triad

from _helpers import GOLDEN, random_digraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


def concat(members):
    """BatchCSR from a list of graphs.CSR (graph-local ids)."""
    vb = [0]
    offs, nbs, fls = [np.zeros(1, np.int64)], [], []
    e0 = 0
    for g in members:
        vb.append(vb[-1] + g.n)
        offs.append(g.offsets[1:] + e0)
        nbs.append(g.nbrs)
        fls.append(g.flag_array())
        e0 += g.nnz
    f = np.concatenate(fls) if fls else np.zeros(0, np.uint8)
    j = np.arange(f.size)
    packed = np.zeros((f.size + 3) // 4, np.uint8)
    np.bitwise_or.at(packed, j >> 2, (f << (2 * (j & 3))).astype(np.uint8))
    return graphs.BatchCSR(len(members), np.array(vb, np.int64), np.concatenate(offs).astype(np.int64),
                           np.concatenate(nbs).astype(np.int32) if nbs else np.zeros(0, np.int32), packed,
                           np.zeros((len(members), 6)))


@pytest.mark.parametrize("short_tasks", [0, -1])
def test_small_ensemble(torch, short_tasks):
    B = graphs.null_ensemble(G=48, seed=5, nmin=64, nmax=700, dmin=4, dmax=20)
    d = triad.batch_to_device(B)
    got = triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d, short_tasks=short_tasks)
    for g in range(B.G):
        assert got[g] == oracle.census(B.graph(g)), g


def test_grouped_rounds_across_graphs(torch):
    """Many tiny members: grouped rounds of short tasks span graph boundaries
    (each lane's counts go to its own task's graph), next to members whose
    tasks fill every bin and the item path (a star with a 300-leaf hub)."""
    members = []
    rng = np.random.default_rng(12)
    for k in range(300):
        n = int(rng.integers(3, 9))
        s, t = random_digraph(n, 0.6, 0.3, 1000 + k)
        members.append(graphs.build_csr(n, s, t))
    star = [(0, j) for j in range(1, 301)] + [(j, j + 1) for j in range(1, 300, 3)]
    members.append(graphs.from_arcs(302, star))
    for n, dens in ((120, 0.5), (260, 0.9), (40, 0.2)):
        s, t = random_digraph(n, dens, 0.2, n)
        members.append(graphs.build_csr(n, s, t))
    B = concat(members)
    d = triad.batch_to_device(B)
    got = triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d)
    for g, m in enumerate(members):
        assert got[g] == oracle.census(m), g


def test_degenerate_members(torch):
    rng_graphs = [graphs.build_csr(0, np.zeros(0, np.int32), np.zeros(0, np.int32)),
                  graphs.build_csr(1, np.zeros(0, np.int32), np.zeros(0, np.int32)),
                  graphs.from_arcs(2, [(0, 1), (1, 0)]),
                  graphs.build_csr(9, np.zeros(0, np.int32), np.zeros(0, np.int32)),
                  graphs.from_arcs(3, [(0, 1), (1, 2), (2, 0)])]
    for k, (n, dens, rec) in enumerate([(40, 0.3, 0.3), (65, 0.1, 1.0), (130, 0.05, 0.0)]):
        s, t = random_digraph(n, dens, rec, 100 + k)
        rng_graphs.append(graphs.build_csr(n, s, t))
    B = concat(rng_graphs)
    d = triad.batch_to_device(B)
    got = triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d)
    for g, m in enumerate(rng_graphs):
        assert got[g] == oracle.census(m), g


def test_graph_replays(torch):
    B = graphs.null_ensemble(G=32, seed=6, nmin=64, nmax=400, dmin=4, dmax=16)
    want = [oracle.census(B.graph(g)) for g in range(B.G)]
    d = triad.batch_to_device(B)
    plan = triad.BatchPlan(B.G, int(B.vbase[-1]), B.nnz, *d)
    for rep in range(4):
        plan.launch()
        assert plan.result() == want, rep
        # eager work on the same stream between replays
        x = torch.arange(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert int(x) == (1 << 20) * ((1 << 20) - 1) // 2
    plan.close()


def test_batch_validation_error(torch):
    B = graphs.null_ensemble(G=4, seed=7, nmin=64, nmax=100, dmin=4, dmax=8)
    nb = B.nbrs.copy()
    nb[5] = 100000  # out of its graph's range
    d = list(triad.batch_to_device(B))
    d[2] = torch.from_numpy(nb).cuda()
    with pytest.raises(triad.TriadError) as e:
        triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d)
    assert e.value.status == triad.ERANGE


@pytest.mark.parametrize("case", ["first", "last", "order", "too_large"])
def test_batch_rejects_bad_bases(torch, case):
    """Graph bases are checked on the host before any launch: a bad vbase is
    TRIAD_EINVAL and nothing is written."""
    B = graphs.null_ensemble(G=4, seed=7, nmin=64, nmax=100, dmin=4, dmax=8)
    vb = B.vbase.copy()
    nv, nnz = int(vb[-1]), B.nnz
    if case == "first":
        vb[0] = 1
    elif case == "last":
        vb[-1] = nv - 1
    elif case == "order":
        vb[2] = vb[1] - 1
    else:
        # one member of 4,801,281 vertices and no arcs: its C(n,3) exceeds 2^64
        vb = np.array([0, 4801281], np.int64)
        nv, nnz = 4801281, 0
    d = [torch.from_numpy(vb).cuda()] + list(triad.batch_to_device(B))[1:]
    if case == "too_large":
        d[1] = torch.zeros(nv + 1, dtype=torch.int64, device="cuda")
    G = vb.size - 1
    out = torch.full((G, 16), 7, dtype=torch.int64, device="cuda")
    for call in ("plan", "tune"):
        with pytest.raises(triad.TriadError) as e:
            if call == "plan":
                triad.BatchPlan(G, nv, nnz, *d, d_out=out)
            else:
                triad.batch_autotune(G, nv, nnz, *d)
        assert e.value.status == triad.EINVAL, (call, str(e.value))
    assert torch.all(out == 7), "output written on error"
    # a member of 4,801,280 vertices is accepted
    if case == "too_large":
        vb = np.array([0, 4801280], np.int64)
        d = [torch.from_numpy(vb).cuda(), torch.zeros(4801281, dtype=torch.int64, device="cuda"), d[2], d[3]]
        got = triad.triad_census_batch(1, 4801280, 0, *d)
        assert got[0] == oracle.census(graphs.build_csr(4801280, np.zeros(0, np.int32), np.zeros(0, np.int32)))


def test_autotune_and_cache(torch, tmp_path):
    B = graphs.null_ensemble(G=64, seed=8, nmin=64, nmax=900, dmin=4, dmax=24)
    want = [oracle.census(B.graph(g)) for g in range(B.G)]
    d = triad.batch_to_device(B)
    cache = str(tmp_path / "tune.jsonl")
    best = triad.batch_autotune(B.G, int(B.vbase[-1]), B.nnz, *d, cache_path=cache)
    assert best["kernel_variant"] > 0 and best["waves_per_group"] in (1, 2)
    again = triad.batch_autotune(B.G, int(B.vbase[-1]), B.nnz, *d, cache_path=cache)
    assert again == best
    assert len(open(cache).read().strip().splitlines()) == 1
    # another batch of the same sizes (member 0's ids reversed, so its degree
    # sequence moves) has another signature: it is tuned again and appended
    m0 = B.graph(0)
    s0, t0 = m0.arcs()
    r0 = graphs.build_csr(m0.n, m0.n - 1 - s0, m0.n - 1 - t0)
    B2 = concat([r0] + [B.graph(g) for g in range(1, B.G)])
    assert (B2.G, int(B2.vbase[-1]), B2.nnz) == (B.G, int(B.vbase[-1]), B.nnz)
    assert not np.array_equal(B2.offsets, B.offsets)
    d2 = triad.batch_to_device(B2)
    triad.batch_autotune(B2.G, int(B2.vbase[-1]), B2.nnz, *d2, cache_path=cache)
    assert len(open(cache).read().strip().splitlines()) == 2
    # a cached line whose launch shape is not a candidate is ignored (tuned again)
    lines = open(cache).read().strip().splitlines()
    bad = json.loads(lines[0])
    bad["waves_per_group"] = 3
    with open(cache, "w") as f:
        f.write(json.dumps(bad) + "\n")
    third = triad.batch_autotune(B.G, int(B.vbase[-1]), B.nnz, *d, cache_path=cache)
    assert third["waves_per_group"] in (1, 2)
    assert len(open(cache).read().strip().splitlines()) == 2
    assert triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d, **best) == want


def test_full_ensemble_golden(torch):
    path = os.path.join(GOLDEN, "census_nullens.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    rec = json.load(open(path))
    p = rec["params"]
    B = graphs.null_ensemble(G=p["G"], seed=p["seed"], nmin=p["nmin"], nmax=p["nmax"], dmin=p["dmin"],
                             dmax=p["dmax"], rmax=p["rmax"], swap_factor=p["swap_factor"])
    assert B.content_hash() == rec["content_hash"]
    d = triad.batch_to_device(B)
    for short_tasks in (0, -1):
        got = triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *d, short_tasks=short_tasks)
        assert [[str(x) for x in row] for row in got] == rec["census"], short_tasks
