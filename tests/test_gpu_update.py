"""Incremental census (arc insertions and deletions in batches, Sec. 3)
against the oracle: after each batch the census equals the oracle's census of
the updated arc set, bit-exact, and the CSR after the batch equals the host
builder's, byte for byte."""
import numpy as np
import pytest

import oracle
from oracle.update import apply_updates
from paper_1209_6308_amd import graphs, triad

from _helpers import random_digraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


def _random_batch(rng, n, src, dst, k, p_delete=0.4, p_reverse=0.2):
    """k updates: deletions of existing arcs, insertions of reverse arcs of
    existing ones (pairs turning mutual), insertions between random vertices,
    and repeats of earlier updates (so some arcs get several operations)."""
    us, ud, ui = [], [], []
    m = src.size
    for _ in range(k):
        r = rng.random()
        if m and r < p_delete:
            i = rng.integers(m)
            us.append(src[i]); ud.append(dst[i]); ui.append(0)
        elif m and r < p_delete + p_reverse:
            i = rng.integers(m)
            us.append(dst[i]); ud.append(src[i]); ui.append(1)
        elif us and r < 0.9:
            a, b = rng.integers(n), rng.integers(n)
            if a == b:
                b = (a + 1) % n
            us.append(a); ud.append(b); ui.append(1)
        else:
            j = rng.integers(len(us)) if us else None
            if j is None:
                a, b = 0, 1 % n
                us.append(a); ud.append(b); ui.append(1)
            else:
                us.append(us[j]); ud.append(ud[j]); ui.append(1 - ui[j])
    return np.array(us, np.int32), np.array(ud, np.int32), np.array(ui, np.uint8)


def _run_series(torch, n, src, dst, batches, seed):
    rng = np.random.default_rng(seed)
    g = graphs.build_csr(n, src, dst)
    s, d = g.arcs()
    census = oracle.census(g)
    dev = triad.to_device(g)
    nnz = g.nnz
    for k in batches:
        us, ud, ui = _random_batch(rng, n, s, d, k)
        t = [torch.from_numpy(a).cuda() for a in (us, ud, ui)]
        got, new, changed = triad.census_update(n, nnz, *dev, census, *t)
        s, d = apply_updates(s, d, us, ud, ui)
        want_g = graphs.build_csr(n, s, d)
        assert got == oracle.census(want_g), k
        off, nb, fl = (x.cpu().numpy() for x in new)
        assert np.array_equal(off, want_g.offsets)
        assert np.array_equal(nb, want_g.nbrs)
        assert np.array_equal(fl, want_g.flags)
        census, dev, nnz = got, new, int(nb.size)
    return census


@pytest.mark.parametrize("n,density,recip,seed", [(12, 0.4, 0.3, 1), (60, 0.1, 0.2, 2), (300, 0.02, 0.5, 3)])
def test_random_digraph_series(torch, n, density, recip, seed):
    s, d = random_digraph(n, density, recip, seed)
    _run_series(torch, n, s, d, [1, 5, 40, 200, 0, 7], seed)


def test_rmat_with_hubs(torch):
    # R-MAT scale 12: updates land on hub rows (long neighbour lists, many
    # changed pairs per row)
    src, dst = graphs.rmat_arcs(12, 8 << 12, seed=4)
    _run_series(torch, 1 << 12, src, dst, [3000, 1, 500], 11)


def test_long_pairs_and_sparse_rows(torch):
    """Two hub rows (20,000 and 15,000 neighbours): their changed pairs merge
    more than 8,192 positions and are cut into several work items; the CSR copy
    meets tiles inside a hub row (one changed row), a tile holding the end of
    one hub row and the start of the other, and tiles over thousands of short
    or empty rows (the per-entry row search)."""
    n = 120_000
    rng = np.random.default_rng(21)
    h0 = rng.choice(np.arange(2, 60_000), 20_000, replace=False)
    h1 = rng.choice(np.arange(2, 60_000), 15_000, replace=False)
    sp = np.arange(60_000, n, 97)
    src = np.concatenate([np.zeros(h0.size), np.ones(h1.size), [0], sp[:-1]]).astype(np.int32)
    dst = np.concatenate([h0, h1, [1], sp[1:]]).astype(np.int32)
    _run_series(torch, n, src, dst, [50, 400, 3000], 5)


def test_from_empty_and_to_empty(torch):
    n = 9
    arcs = [(0, 1), (1, 2), (2, 0), (3, 4), (4, 3), (5, 6), (6, 7), (7, 5), (8, 0)]
    s = np.array([a for a, _ in arcs], np.int32)
    d = np.array([b for _, b in arcs], np.int32)
    empty = graphs.build_csr(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    dev = triad.to_device(empty)
    t = [torch.from_numpy(a).cuda() for a in (s, d, np.ones(s.size, np.uint8))]
    got, new, changed = triad.census_update(n, 0, *dev, oracle.census(empty), *t)
    full = graphs.build_csr(n, s, d)
    assert got == oracle.census(full)
    assert changed == 8  # 3-4 / 4-3 is one pair
    t = [torch.from_numpy(a).cuda() for a in (s, d, np.zeros(s.size, np.uint8))]
    got2, new2, _ = triad.census_update(n, full.nnz, *new, got, *t)
    assert got2 == oracle.census(empty)
    assert int(new2[1].numel()) == 0 and np.all(new2[0].cpu().numpy() == 0)


def test_wrapped_003(torch):
    # 003 above 2^64 before and after
    n = 4801300
    g = graphs.from_arcs(n, [(0, 1), (5, 6)])
    dev = triad.to_device(g)
    us, ud, ui = np.array([1, 5, 7], np.int32), np.array([0, 6, 9], np.int32), np.array([1, 0, 1], np.uint8)
    t = [torch.from_numpy(a).cuda() for a in (us, ud, ui)]
    got, new, _ = triad.census_update(n, g.nnz, *dev, oracle.census(g), *t, new_csr=False)
    s, d = apply_updates(*g.arcs(), us, ud, ui)
    assert new is None
    assert got == oracle.census(graphs.build_csr(n, s, d))


def test_update_errors(torch):
    g = graphs.rmat(6, 4, seed=1)
    dev = triad.to_device(g)
    c = oracle.census(g)
    for us, ud, ui, status in (([3], [3], [1], triad.ESELFLOOP), ([0], [g.n], [1], triad.ERANGE),
                               ([0], [1], [2], triad.ERANGE)):
        t = [torch.tensor(a, dtype=dt, device="cuda") for a, dt in ((us, torch.int32), (ud, torch.int32),
                                                                   (ui, torch.uint8))]
        with pytest.raises(triad.TriadError) as e:
            triad.census_update(g.n, g.nnz, *dev, c, *t)
        assert e.value.status == status


def test_rmat24_batch_and_its_inverse(torch):
    """Full size (R-MAT scale 24, the benchmark workload): a batch of 100,000
    updates, each touching a different arc (deletions of present arcs,
    insertions of absent ones), gives the census a full census of the
    resulting CSR gives; the inverse batch (every deletion re-inserted, every
    insertion deleted) from there returns the oracle's stored census and the
    original CSR, byte for byte."""
    import json
    import os

    from _helpers import GOLDEN
    path = os.path.join(GOLDEN, "census_rmat24.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    rec = json.load(open(path))
    g = graphs.workload("rmat24")
    assert g.content_hash() == rec["content_hash"]
    want = [int(x) for x in rec["census"]]
    off, nbr, flg = triad.to_device(g)
    n, nnz, k = g.n, g.nnz, 100000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    # arcs of the graph as sorted keys row * n + col (an entry with bit0 set is the arc row -> col)
    rows = torch.repeat_interleave(torch.arange(n, device="cuda"), off[1:] - off[:-1])
    j = torch.arange(nnz, device="cuda")
    f = (flg[j >> 2].to(torch.int64) >> (2 * (j & 3))) & 3
    akey = (rows * n + nbr.to(torch.int64))[(f & 1) != 0]
    del rows, j, f
    dkey = torch.unique(akey[torch.randint(0, akey.numel(), (k // 2,), device="cuda", generator=gen)])
    a = torch.randint(0, n, (k,), device="cuda", generator=gen)
    b = (a + torch.randint(1, n, (k,), device="cuda", generator=gen)) % n
    ikey = torch.unique(a * n + b)
    pos = torch.searchsorted(akey, ikey).clamp(max=akey.numel() - 1)
    ikey = ikey[akey[pos] != ikey][: k - dkey.numel()]
    del akey
    keys = torch.cat([dkey, ikey])
    ins = torch.cat([torch.zeros(dkey.numel(), dtype=torch.uint8, device="cuda"),
                     torch.ones(ikey.numel(), dtype=torch.uint8, device="cuda")])
    perm = torch.randperm(keys.numel(), device="cuda", generator=gen)
    keys, ins = keys[perm], ins[perm].contiguous()
    us, ud = (keys // n).to(torch.int32).contiguous(), (keys % n).to(torch.int32).contiguous()
    c1, csr1, chg = triad.census_update(n, nnz, off, nbr, flg, want, us, ud, ins)
    assert chg > 0.9 * keys.numel()
    nnz1 = int(csr1[1].numel())
    full, st, _ = triad.triad_census_device(n, nnz1, *csr1, validate=1)
    assert c1 == full
    c2, csr2, _ = triad.census_update(n, nnz1, *csr1, c1, us, ud, (1 - ins).contiguous())
    assert c2 == want
    assert torch.equal(csr2[0], off) and torch.equal(csr2[1], nbr) and torch.equal(csr2[2], flg)


def test_sliding_window_series(torch):
    """Windowed census: a stream of timestamped arcs (R-MAT endpoints, uniform
    times), a window of 20 time units moved by 5; each step's batch (arcs that
    left the window deleted, arcs that entered inserted) brings the census of
    the previous window to the oracle's census of the new window's arc set."""
    n = 1 << 9
    src, dst = graphs.rmat_arcs(9, 40000, seed=4)
    times = np.random.default_rng(6).uniform(0.0, 100.0, src.size)
    g = graphs.build_csr(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    dev, nnz = triad.to_device(g), 0
    census = oracle.census(g)
    steps = 0
    for t, us, ud, ui in graphs.window_batches(n, src, dst, times, 20.0, 5.0, 100.0):
        args = [torch.from_numpy(a).cuda() for a in (us, ud, ui)]
        census, dev, _ = triad.census_update(n, nnz, *dev, census, *args)
        nnz = int(dev[1].numel())
        sel = (times >= t) & (times < t + 20.0)
        want = graphs.build_csr(n, src[sel], dst[sel])
        assert census == oracle.census(want), t
        assert np.array_equal(dev[0].cpu().numpy(), want.offsets)
        steps += 1
    assert steps == 17
