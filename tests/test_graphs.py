"""Seeded input generators and the CSR builder (input contract of the census)."""
import ctypes

import numpy as np
import pytest

from paper_1209_6308_amd import graphs


def check_csr(g: graphs.CSR):
    off, nb = g.offsets, g.nbrs
    assert off[0] == 0 and off[-1] == g.nnz and np.all(np.diff(off) >= 0)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    assert np.all(nb >= 0) and np.all(nb < g.n)
    assert np.all(nb != rows), "self-loop"
    same_row = rows[1:] == rows[:-1]
    assert np.all(nb[1:][same_row] > nb[:-1][same_row]), "row not strictly increasing"
    f = g.flag_array()
    assert np.all(f != 0)
    # symmetry with mirrored flags: (x,y,f) present iff (y,x,swap(f)) present
    key = rows * g.n + nb
    rkey = nb.astype(np.int64) * g.n + rows
    order = np.argsort(key)
    pos = np.searchsorted(key[order], rkey)
    assert np.all(pos < key.size)
    assert np.all(key[order][pos] == rkey)
    fm = f[order][pos]
    swapped = ((f & 1) << 1) | ((f >> 1) & 1)
    assert np.array_equal(fm, swapped)


@pytest.mark.parametrize("name", ["rmat10"])
def test_workload_valid_and_deterministic(name):
    a = graphs.workload(name)
    b = graphs.workload(name)
    check_csr(a)
    assert a.content_hash() == b.content_hash()


def test_rmat_thread_count_independent():
    L = graphs.lib()
    outs = []
    for t in (1, 3, 8):
        s = np.empty(1 << 16, dtype=np.int32)
        d = np.empty(1 << 16, dtype=np.int32)
        L.tg_rmat(12, s.size, 0.57, 0.19, 0.19, 5, ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(d.ctypes.data), t)
        outs.append((s, d))
    for s, d in outs[1:]:
        assert np.array_equal(s, outs[0][0]) and np.array_equal(d, outs[0][1])


def test_rmat_quadrant_frequencies():
    s, d = graphs.rmat_arcs(1, 200000, seed=11)
    q = s * 2 + d
    freq = np.bincount(q, minlength=4) / q.size
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_csr_round_trip_and_recip():
    g = graphs.rmat(12, 8, seed=2)
    check_csr(g)
    s, d = g.arcs()
    h = graphs.build_csr(g.n, s, d)
    assert h.content_hash() == g.content_hash()
    r = graphs.rmat(12, 8, seed=2, recip_p=0.5)
    check_csr(r)
    assert r.stats()["mutual_pairs"] > g.stats()["mutual_pairs"]
    assert r.stats()["m_sym"] == g.stats()["m_sym"]


def test_csr_drops_loops_and_duplicates():
    g = graphs.from_arcs(4, [(0, 1), (0, 1), (1, 0), (2, 2), (3, 1)])
    check_csr(g)
    assert g.offsets.tolist() == [0, 1, 3, 3, 4]
    assert g.nbrs.tolist() == [1, 0, 3, 1]
    assert g.flag_array().tolist() == [3, 3, 2, 1]


def test_chung_lu_small():
    g = graphs.chung_lu(1 << 12, 2.1, 8.0, 256.0, seed=3)
    check_csr(g)
    d = np.diff(g.offsets)
    assert d.max() > 20 * np.median(d[d > 0])


def _degrees(n, s, d):
    arcs = set(zip(s.tolist(), d.tolist()))
    od = np.zeros(n, int); idg = np.zeros(n, int); mu = np.zeros(n, int)
    for a, b in arcs:
        od[a] += 1; idg[b] += 1
        if (b, a) in arcs:
            mu[a] += 1
    return od, idg, mu


def test_swaps_preserve_degrees():
    n = 200
    s, d = graphs.erdos_renyi_arcs(n, 1500, seed=4)
    keep = s != d
    a = np.unique(np.stack([s[keep], d[keep]], 1), axis=0)
    # reciprocate some
    extra = a[:200][:, ::-1]
    a = np.unique(np.concatenate([a, extra]), axis=0)
    s, d = a[:, 0].astype(np.int32), a[:, 1].astype(np.int32)
    s2, d2, acc = graphs.degree_preserving_swaps(s, d, 20000, seed=5)
    assert acc > 1000
    assert len(set(zip(s2.tolist(), d2.tolist()))) == s2.size
    assert np.all(s2 != d2)
    for x, y in zip(_degrees(n, s, d), _degrees(n, s2, d2)):
        assert np.array_equal(x, y)
    assert set(zip(s.tolist(), d.tolist())) != set(zip(s2.tolist(), d2.tolist()))


def test_null_ensemble_small():
    B = graphs.null_ensemble(G=16, seed=3, nmin=64, nmax=300, dmin=4, dmax=12)
    assert B.vbase[0] == 0 and B.offsets[-1] == B.nnz
    for g in range(B.G):
        m = B.graph(g)
        check_csr(m)
        kind, n, mean, recip, gamma, arcs = B.params[g]
        assert 64 <= n <= 300 and 4 <= mean <= 12 and 0 <= recip <= 0.3 and 2.1 <= gamma <= 3.0
        assert m.n == n
        assert kind == (g & 1)
    C = graphs.null_ensemble(G=16, seed=3, nmin=64, nmax=300, dmin=4, dmax=12)
    assert C.content_hash() == B.content_hash()


def test_randomised_ensemble_keeps_degrees():
    g = graphs.rmat(9, 8, seed=4, recip_p=0.3)
    B = graphs.randomised_ensemble(g, 6, seed=2)
    assert B.G == 6 and np.array_equal(np.diff(B.vbase), np.full(6, g.n))

    def degs(h):
        f = h.flag_array()
        rows = np.repeat(np.arange(h.n), np.diff(h.offsets))
        out = np.bincount(rows[(f & 1) != 0], minlength=h.n)
        inn = np.bincount(rows[(f & 2) != 0], minlength=h.n)
        mut = np.bincount(rows[f == 3], minlength=h.n)
        return out, inn, mut

    want = degs(g)
    changed = 0
    for k in range(B.G):
        m = B.graph(k)
        for a, b in zip(degs(m), want):
            assert np.array_equal(a, b)
        changed += int(not np.array_equal(m.nbrs, g.nbrs))
    assert changed == B.G  # every copy was rewired
    again = graphs.randomised_ensemble(g, 6, seed=2)
    assert again.content_hash() == B.content_hash()


def test_window_batches_follow_the_window():
    """Applying each step's batch to a set of arcs (delete, then insert) gives
    exactly the arc set of the new window; no batch touches an arc twice."""
    n = 1 << 9
    src, dst = graphs.rmat_arcs(9, 20000, seed=4)
    times = np.random.default_rng(6).uniform(0.0, 100.0, src.size)
    cur, steps = set(), 0
    for t, us, ud, ui in graphs.window_batches(n, src, dst, times, 20.0, 5.0, 100.0):
        pairs = list(zip(us.tolist(), ud.tolist()))
        assert len(set(pairs)) == len(pairs)
        for (a, b), i in zip(pairs, ui.tolist()):
            if i:
                assert (a, b) not in cur
                cur.add((a, b))
            else:
                cur.remove((a, b))
        sel = (times >= t) & (times < t + 20.0) & (src != dst)
        assert cur == set(zip(src[sel].tolist(), dst[sel].tolist()))
        steps += 1
    assert steps == 17
