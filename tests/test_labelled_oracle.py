"""Pins of the 64-state labelled census oracle (CPU): its sweep against the
definition (every triple a < b < c, by brute force, exhaustively on small
vertex sets), closed forms, the relabelling that reverses id order, and the
condensation of the 64 states into the 16 classes by the class table."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1209_6308_amd import graphs

from _helpers import random_digraph

STATES = 64


def mirror(f):
    return ((f & 1) << 1) | (f >> 1)


def _arcs_of_pairs(n, states):
    """Arc list of the digraph whose unordered pair k (itertools order) has
    state states[k] (bit0 = lower -> higher id, bit1 = higher -> lower)."""
    src, dst = [], []
    for (a, b), s in zip(itertools.combinations(range(n), 2), states):
        if s & 1:
            src.append(a); dst.append(b)
        if s & 2:
            src.append(b); dst.append(a)
    return np.array(src, np.int32), np.array(dst, np.int32)


@pytest.mark.parametrize("n", [3, 4])
def test_exhaustive_against_definition(n):
    pairs = n * (n - 1) // 2
    for code in range(4 ** pairs):
        states = [(code >> (2 * k)) & 3 for k in range(pairs)]
        s, d = _arcs_of_pairs(n, states)
        g = graphs.build_csr(n, s, d)
        assert oracle.labelled_census(g) == oracle.brute64(n, s, d), states


@pytest.mark.parametrize("n,density,recip,seed", [(5, 0.7, 0.3, 1), (12, 0.5, 0.5, 2), (30, 0.2, 0.1, 3),
                                                  (61, 0.1, 0.0, 4), (45, 0.9, 0.9, 5)])
def test_random_against_definition(n, density, recip, seed):
    s, d = random_digraph(n, density, recip, seed)
    g = graphs.build_csr(n, s, d)
    assert oracle.labelled_census(g) == oracle.brute64(n, s, d)


def test_rmat10_against_definition():
    g = graphs.workload("rmat10")
    s, d = g.arcs()
    got = oracle.labelled_census(g)
    assert got == oracle.brute64(g.n, s, d)
    assert sum(got) == g.n * (g.n - 1) * (g.n - 2) // 6


def test_condensed_by_class_table():
    lut = oracle.lut()
    for g in (graphs.workload("rmat10"), graphs.rmat(11, 8, seed=3, recip_p=0.3)):
        lab = oracle.labelled_census(g)
        cond = [0] * 16
        for st, c in enumerate(lab):
            cond[int(lut[st])] += c
        assert cond == oracle.census(g)


@pytest.mark.parametrize("n", [3, 4, 9])
def test_closed_forms(n):
    c3 = n * (n - 1) * (n - 2) // 6
    up = [(i, j) for i in range(n) for j in range(i + 1, n)]
    cases = {21: up,                                # transitive tournament, lower -> higher: 1 | 1<<2 | 1<<4
             42: [(j, i) for i, j in up],           # the reverse: 2 | 2<<2 | 2<<4
             63: up + [(j, i) for i, j in up],      # complete mutual
             0: []}
    for state, arcs in cases.items():
        g = graphs.from_arcs(n, arcs) if arcs else graphs.build_csr(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
        want = [0] * STATES
        want[state] = c3
        assert oracle.labelled_census(g) == want, state


@pytest.mark.parametrize("a,b,n", [(2, 5, 9), (0, 1, 4), (0, 7, 8), (3, 4, 8)])
def test_single_arc_by_position(a, b, n):
    """One arc a -> b, a < b: the triples with a third vertex below a, between,
    and above b are in states 1<<4, 1<<2 and 1 (the pair's flag sits at the
    position of the pair within the triple)."""
    lab = oracle.labelled_census(graphs.from_arcs(n, [(a, b)]))
    want = [0] * STATES
    want[1 << 4] = a
    want[1 << 2] = b - a - 1
    want[1] = n - 1 - b
    want[0] = n * (n - 1) * (n - 2) // 6 - (n - 2)
    assert lab == want


def test_reversed_ids():
    """Relabelling x -> n-1-x turns (a, b, c) into (c', b', a'): the state
    (f_ab, f_ac, f_bc) becomes (mirror f_bc, mirror f_ac, mirror f_ab)."""
    n = 40
    s, d = random_digraph(n, 0.25, 0.3, 9)
    g = graphs.build_csr(n, s, d)
    r = graphs.build_csr(n, (n - 1 - s).astype(np.int32), (n - 1 - d).astype(np.int32))
    lab, rev = oracle.labelled_census(g), oracle.labelled_census(r)
    for st in range(STATES):
        fab, fac, fbc = st & 3, (st >> 2) & 3, st >> 4
        assert rev[mirror(fbc) | mirror(fac) << 2 | mirror(fab) << 4] == lab[st]


def test_state0_high_word():
    n = 4801290
    g = graphs.from_arcs(n, [(0, 1), (n - 1, 3)])
    lab = oracle.labelled_census(g)
    assert lab[0] >= 1 << 64
    assert sum(lab) == n * (n - 1) * (n - 2) // 6
