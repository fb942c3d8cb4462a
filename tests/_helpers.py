"""Shared test helpers: fixtures parsing, small random digraphs, and per-graph
quantities computed straight from the arc list (no census code involved)."""
from __future__ import annotations

import itertools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
TYPES = ["003", "012", "102", "021D", "021U", "021C", "111D", "111U",
         "030T", "030C", "201", "120D", "120U", "120C", "210", "300"]


def prototypes():
    """{type: set of arcs on vertices 0,1,2} from tests/golden/triad_prototypes.txt."""
    out = {}
    idx = {"A": 0, "B": 1, "C": 2}
    with open(os.path.join(GOLDEN, "triad_prototypes.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            arcs = set()
            for tok in parts[1:]:
                if ">" in tok:
                    a, b = tok.split(">")
                    arcs.add((idx[a], idx[b]))
                else:
                    a, b = tok.split("=")
                    arcs.add((idx[a], idx[b]))
                    arcs.add((idx[b], idx[a]))
            out[parts[0]] = arcs
    assert list(out) == TYPES
    return out


def code_of(arcs, u=0, v=1, w=2):
    """6-bit triad code with bit0 u->v, bit1 v->u, bit2 u->w, bit3 w->u, bit4 v->w, bit5 w->v."""
    bits = [(u, v), (v, u), (u, w), (w, u), (v, w), (w, v)]
    return sum(1 << k for k, a in enumerate(bits) if a in arcs)


def arcs_of_code(code):
    bits = [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)]
    return {a for k, a in enumerate(bits) if (code >> k) & 1}


def type_coefficients():
    """Per type: M, A, N dyads; out2 / in2 = pairs sharing a sender / receiver;
    path2 = directed 2-paths a->b->c (a != c). Counted on the prototype digraphs."""
    co = {}
    for t, arcs in prototypes().items():
        pairs = [(0, 1), (0, 2), (1, 2)]
        M = sum(1 for a, b in pairs if (a, b) in arcs and (b, a) in arcs)
        A = sum(1 for a, b in pairs if ((a, b) in arcs) != ((b, a) in arcs))
        N = 3 - M - A
        od = [sum(1 for (a, b) in arcs if a == x) for x in range(3)]
        idg = [sum(1 for (a, b) in arcs if b == x) for x in range(3)]
        out2 = sum(d * (d - 1) // 2 for d in od)
        in2 = sum(d * (d - 1) // 2 for d in idg)
        path2 = sum(1 for (a, b) in arcs for (b2, c) in arcs if b2 == b and c != a)
        co[t] = dict(M=M, A=A, N=N, out2=out2, in2=in2, path2=path2)
    return co


def random_digraph(n, density, recip, seed):
    """Arc list of a random simple digraph: each unordered pair is connected with
    probability `density`; a connected pair is mutual with probability `recip`,
    otherwise one arc in a random direction."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < density:
                if rng.random() < recip:
                    src += [a, b]
                    dst += [b, a]
                elif rng.random() < 0.5:
                    src.append(a); dst.append(b)
                else:
                    src.append(b); dst.append(a)
    return np.array(src, dtype=np.int32), np.array(dst, dtype=np.int32)


def graph_quantities(n, src, dst):
    """Right-hand sides of the linear census identities, from the arcs alone."""
    arcs = set(zip(src.tolist(), dst.tolist()))
    arcs = {(a, b) for a, b in arcs if a != b}
    und = {(min(a, b), max(a, b)) for a, b in arcs}
    M = sum(1 for a, b in und if (a, b) in arcs and (b, a) in arcs)
    A = len(und) - M
    od = np.zeros(n, dtype=np.int64)
    idg = np.zeros(n, dtype=np.int64)
    mut = np.zeros(n, dtype=np.int64)
    for a, b in arcs:
        od[a] += 1
        idg[b] += 1
        if (b, a) in arcs:
            mut[a] += 1
    adj = [set() for _ in range(n)]
    for a, b in und:
        adj[a].add(b)
        adj[b].add(a)
    T = 0
    for a, b in und:
        T += sum(1 for c in adj[a] & adj[b] if c > b)
    deg = np.array([len(s) for s in adj], dtype=np.int64)
    return dict(
        M=M, A=A, N=n * (n - 1) // 2 - M - A,
        out2=int(sum(int(d) * (int(d) - 1) // 2 for d in od)),
        in2=int(sum(int(d) * (int(d) - 1) // 2 for d in idg)),
        path2=int(sum(int(i) * int(o) - int(m) for i, o, m in zip(idg, od, mut))),
        T=T, wedges=int(sum(int(d) * (int(d) - 1) // 2 for d in deg)),
    )


def check_identities(n, census, q):
    co = type_coefficients()
    c = dict(zip(TYPES, census))
    assert sum(census) == n * (n - 1) * (n - 2) // 6
    for key, side in (("M", q["M"]), ("A", q["A"]), ("N", q["N"])):
        assert sum(co[t][key] * c[t] for t in TYPES) == side * (n - 2), key
    assert sum(co[t]["out2"] * c[t] for t in TYPES) == q["out2"]
    assert sum(co[t]["in2"] * c[t] for t in TYPES) == q["in2"]
    assert sum(co[t]["path2"] * c[t] for t in TYPES) == q["path2"]
    tri = ["030T", "030C", "120D", "120U", "120C", "210", "300"]
    opn = ["021D", "021U", "021C", "111D", "111U", "201"]
    assert sum(c[t] for t in tri) == q["T"]
    assert sum(c[t] for t in opn) == q["wedges"] - 3 * q["T"]


def permutations3():
    return list(itertools.permutations(range(3)))
