"""CSR construction on the device (the compact structure of Sec. 6, Fig. 7)
against the host builder of the input generators: the same offsets, ids and
packed flags, byte for byte, from the same arc lists (duplicates, self-loops,
isolated vertices, empty inputs), and the census of the result."""
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


def _gpu_build(torch, n, src, dst):
    ds = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int32)).cuda()
    dd = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.int32)).cuda()
    off, nbr, flg = triad.csr_from_arcs(n, ds, dd)
    return graphs.CSR(n, off.cpu().numpy(), nbr.cpu().numpy(), flg.cpu().numpy())


def _same(a, b):
    assert a.n == b.n
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.nbrs, b.nbrs)
    assert np.array_equal(a.flags, b.flags)


@pytest.mark.parametrize("n,density,recip,seed", [(2, 1.0, 1.0, 1), (17, 0.3, 0.2, 2), (200, 0.05, 0.3, 3),
                                                  (700, 0.02, 0.0, 4)])
def test_random_digraphs_with_duplicates_and_loops(torch, n, density, recip, seed):
    s, t = random_digraph(n, density, recip, seed)
    rng = np.random.default_rng(seed)
    # repeat some arcs (in shuffled order) and add self-loops
    k = s.size
    rep = rng.integers(0, max(k, 1), size=k // 2 + 1) if k else np.zeros(0, np.int64)
    loops = rng.integers(0, n, size=5)
    src = np.concatenate([s, s[rep] if k else [], loops]).astype(np.int32)
    dst = np.concatenate([t, t[rep] if k else [], loops]).astype(np.int32)
    p = rng.permutation(src.size)
    src, dst = src[p], dst[p]
    got = _gpu_build(torch, n, src, dst)
    _same(got, graphs.build_csr(n, src, dst))


@pytest.mark.parametrize("n,arcs", [(0, []), (1, []), (5, []), (3, [(1, 1)]), (4, [(3, 0)]),
                                    (6, [(5, 0), (0, 5), (0, 5), (2, 2)])])
def test_degenerate_inputs(torch, n, arcs):
    a = np.array(arcs, dtype=np.int32).reshape(-1, 2)
    got = _gpu_build(torch, n, a[:, 0], a[:, 1])
    _same(got, graphs.build_csr(n, a[:, 0], a[:, 1]))


def test_rmat_and_chung_lu_raw_arcs(torch):
    for n, (src, dst) in ((1 << 12, graphs.rmat_arcs(12, 16 << 12, seed=3)),
                          (1 << 14, graphs.chung_lu_arcs(1 << 14, 2.1, 12.0, 2000.0, 12 << 14, seed=2))):
        g = _gpu_build(torch, n, src, dst)
        _same(g, graphs.build_csr(n, src, dst))
        d = triad.to_device(g)
        assert triad.triad_census_device(g.n, g.nnz, *d, validate=1)[0] == oracle.census(g)


def test_range_error_writes_nothing(torch):
    src = torch.tensor([0, 1, 7], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(triad.TriadError) as e:
        triad.csr_from_arcs(5, src, dst)
    assert e.value.status == triad.ERANGE


def _golden(name):
    path = os.path.join(GOLDEN, f"census_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["cl22", "rmat24"])
def test_full_size_content_hash(torch, name):
    """The device build of the full-size raw arc lists has the content hash of
    the host-built workload the goldens were made from."""
    rec = _golden(name)
    w = graphs.WORKLOADS[name]
    if w["kind"] == "rmat":
        n = 1 << w["scale"]
        src, dst = graphs.rmat_arcs(w["scale"], w["edge_factor"] * n, seed=w["seed"])
    else:
        n = w["n"]
        src, dst = graphs.chung_lu_arcs(n, w["gamma"], w["mean"], w["w0"], int(round(w["mean"] * n)), seed=w["seed"])
    ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    del src, dst
    off, nbr, flg, ms = triad.csr_from_arcs(n, ds, dd, timed=True)
    g = graphs.CSR(n, off.cpu().numpy(), nbr.cpu().numpy(), flg.cpu().numpy())
    assert g.content_hash() == rec["content_hash"], ms
