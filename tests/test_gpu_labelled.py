"""64-state labelled census on the GPU (the states of triples a < b < c by
id order, Sec. 3) against the oracle's labelled sweep, bit-exact, over both
round paths of the merge kernel, hub splits and degenerate graphs; and its
condensation into the 16 classes against the 16-class census."""
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


def _lab(g, **kw):
    d = triad.to_device(g)
    return triad.labelled_census_device(g.n, g.nnz, *d, **kw)


@pytest.mark.parametrize("n,density,recip,seed", [(3, 1.0, 0.5, 1), (10, 0.4, 0.3, 2), (64, 0.2, 0.5, 3),
                                                  (130, 0.1, 0.2, 4), (600, 0.3, 0.1, 5)])
def test_random_small(torch, n, density, recip, seed):
    s, d = random_digraph(n, density, recip, seed)
    g = graphs.build_csr(n, s, d)
    got, st, _ = _lab(g)
    assert got == oracle.labelled_census(g)


@pytest.mark.parametrize("hub", [(-1, 0), (0, 0), (64, 256), (300, 1000)])
def test_rmat_hub_splits(torch, hub):
    # scale 12: long lists (both round paths), split tasks with small chunks
    g = graphs.rmat(12, 8, seed=5, recip_p=0.15)
    got, st, _ = _lab(g, hub_threshold=hub[0], chunk=hub[1])
    assert got == oracle.labelled_census(g)


def test_degenerate(torch):
    for n, arcs in ((0, []), (1, []), (2, [(0, 1)]), (3, [(2, 0)]), (7, [])):
        a = np.array(arcs, np.int32).reshape(-1, 2)
        g = graphs.build_csr(n, a[:, 0], a[:, 1])
        assert _lab(g)[0] == oracle.labelled_census(g)


def test_condenses_to_the_census(torch):
    g = graphs.rmat(13, 8, seed=6, recip_p=0.2)
    lab, _, _ = _lab(g)
    lut = oracle.lut()
    cond = [0] * 16
    for st, c in enumerate(lab):
        cond[int(lut[st])] += c
    d = triad.to_device(g)
    assert cond == triad.triad_census_device(g.n, g.nnz, *d)[0]


def test_schedules_and_wrapped_state0(torch):
    g = graphs.rmat(11, 8, seed=2, recip_p=0.3)
    want = oracle.labelled_census(g)
    for sched in ("heuristic",):
        assert _lab(g, schedule=sched, tail_share=-1)[0] == want
    n = 4801300
    g = graphs.from_arcs(n, [(0, 1), (1, 0), (7, 3), (n - 1, 2)])
    got, st, _ = _lab(g)
    assert got == oracle.labelled_census(g)
    assert st == triad.OK_003_WRAPPED


@pytest.mark.parametrize("name", ["rmat20", "rmat24"])
def test_condensed_golden(torch, name):
    """Full size: R-MAT scales 20 and 24 (the benchmark workload, 003 above
    2^64); the condensed labelled census equals the oracle's stored 16-class
    census of the same graph."""
    path = os.path.join(GOLDEN, f"census_{name}.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    rec = json.load(open(path))
    g = graphs.workload(name)
    assert g.content_hash() == rec["content_hash"]
    lab, _, _ = _lab(g)
    lut = oracle.lut()
    cond = [0] * 16
    for st, c in enumerate(lab):
        cond[int(lut[st])] += c
    assert [str(x) for x in cond] == rec["census"]
