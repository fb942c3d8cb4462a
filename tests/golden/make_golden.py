"""Write the stored expected censuses of the large synthetic workloads.

Every number written here comes from the CPU oracle only (``oracle/``): the
Batagelj-Mrvar sweep of Fig. 5 run on all host threads, confirmed by the
independent wedge/triangle decomposition. The graphs are regenerated from
their seeds by ``paper_1209_6308_amd.graphs`` and identified by a content hash,
so a test can check it is looking at the same graph.

    python tests/golden/make_golden.py rmat20 cl22 rmat24 nullens
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1209_6308_amd import graphs  # noqa: E402


def threads():
    return max(1, len(os.sched_getaffinity(0)))


def single(name):
    t0 = time.time()
    g = graphs.workload(name)
    tgen = time.time() - t0
    h = g.content_hash()
    st = g.stats()
    print(f"[{name}] generated in {tgen:.1f}s hash={h} {st}", flush=True)
    t0 = time.time()
    a = oracle.census_mt(g, threads())
    ta = time.time() - t0
    print(f"[{name}] sweep {ta:.1f}s on {threads()} threads", flush=True)
    t0 = time.time()
    b = oracle.wedge_census(g, threads())
    tb = time.time() - t0
    print(f"[{name}] wedge/triangle {tb:.1f}s agree={a == b}", flush=True)
    if a != b:
        raise SystemExit(f"{name}: sweep and decomposition disagree:\n{a}\n{b}")
    rec = {
        "workload": name,
        "params": graphs.WORKLOADS[name],
        "content_hash": h,
        "stats": st,
        "census": [str(x) for x in a],
        "types": oracle.TYPES,
        "oracle": {"sweep_seconds": round(ta, 1), "wedge_seconds": round(tb, 1), "threads": threads()},
    }
    with open(os.path.join(HERE, f"census_{name}.json"), "w") as f:
        json.dump(rec, f, indent=1)


def ensemble(G=4096, seed=1):
    t0 = time.time()
    B = graphs.null_ensemble(G, seed)
    print(f"[nullens] generated {G} graphs in {time.time() - t0:.1f}s nnz={B.nnz}", flush=True)
    out = []
    t0 = time.time()
    for g in range(G):
        m = B.graph(g)
        a = oracle.census(m)
        if g % 64 == 0:
            b = oracle.wedge_census(m, 1)
            if a != b:
                raise SystemExit(f"member {g}: sweep and decomposition disagree")
        out.append([str(x) for x in a])
    print(f"[nullens] oracle {time.time() - t0:.1f}s", flush=True)
    rec = {
        "workload": "nullens",
        "params": {"G": G, "seed": seed, "nmin": 64, "nmax": 8192, "dmin": 4.0, "dmax": 32.0, "rmax": 0.3,
                   "swap_factor": 10.0},
        "content_hash": B.content_hash(),
        "nnz": B.nnz,
        "sum_d2": B.sum_d2(),
        "census": out,
        "types": oracle.TYPES,
    }
    with open(os.path.join(HERE, "census_nullens.json"), "w") as f:
        json.dump(rec, f)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        if name == "nullens":
            ensemble()
        else:
            single(name)
