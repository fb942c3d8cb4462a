"""Checkpointed runs of the CPU oracle. TEST INFRASTRUCTURE ONLY.

A single-threaded oracle census of a large graph (hours at R-MAT scale 24) is
cut into chunks of consecutive CSR entries. Each chunk runs the tasks of
Fig. 5 whose entry lies in it (the edge sweep of the oracle, unchanged) and
adds its partial census (classes 012..300) to the running sums. After every
chunk the sums, the number of chunks done, the chunk size and a SHA-256 of the
graph go to a JSON file, written under a temporary name and renamed into
place, so an interrupted run leaves the last complete checkpoint. A run
started again on the same graph and chunk size resumes after the last chunk
done; the counts are exact integers whose sum does not depend on where the run
was cut. 003 is formed at the end as C(n,3) minus the rest (Fig. 5, steps 3-5).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import _csr_args, _p, choose3, lib

FORMAT = 1


def graph_digest(g):
    """SHA-256 of n and the three CSR arrays."""
    off, nb, fl = _csr_args(g)
    h = hashlib.sha256()
    h.update(np.int64(g.n).tobytes())
    for a in (off, nb, fl):
        h.update(a.tobytes())
    return h.hexdigest()


def _chunk(g, off, nb, fl, j0, j1, nthreads):
    out = np.zeros(16, dtype=np.uint64)
    if nthreads <= 1:
        lib().oracle_census_entries(g.n, _p(off), _p(nb), _p(fl), j0, j1, _p(out))
    else:
        j = np.arange(j0, j1, dtype=np.int64)
        rows = np.searchsorted(off, j, side="right") - 1
        tasks = np.ascontiguousarray(j[nb[j0:j1] > rows])
        lib().oracle_census_tasks_mt(g.n, _p(off), _p(nb), _p(fl), tasks.size, _p(tasks), nthreads, _p(out))
    return [int(x) for x in out]


def _write(path, state):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(state, f)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def census_resumable(g, path, chunk_entries=1 << 22, nthreads=1, max_chunks=None):
    """Census of graph `g` with a checkpoint at `path` after every chunk of
    `chunk_entries` CSR entries. Resumes from an existing checkpoint of the
    same graph and chunk size (ValueError for another graph or size). Runs at
    most `max_chunks` chunks in this call (None: to the end); returns the 16
    counts (003 with its high word) when the census is complete, else None."""
    if chunk_entries < 1:
        raise ValueError("chunk_entries must be >= 1")
    off, nb, fl = _csr_args(g)
    nnz = int(off[g.n]) if g.n > 0 else 0
    digest = graph_digest(g)
    nchunks = (nnz + chunk_entries - 1) // chunk_entries
    state = {"format": FORMAT, "graph_sha256": digest, "n": int(g.n), "nnz": nnz, "chunk_entries": int(chunk_entries),
             "chunks": nchunks, "chunks_done": 0, "partial": [0] * 16, "census": None}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("format") != FORMAT or old.get("graph_sha256") != digest:
            raise ValueError(f"{path} is a checkpoint of another graph")
        if old.get("chunk_entries") != chunk_entries:
            raise ValueError(f"{path} was written with chunks of {old.get('chunk_entries')} entries")
        state = old
    if state["census"] is not None:
        return [int(x) for x in state["census"]]
    ran = 0
    while state["chunks_done"] < nchunks:
        if max_chunks is not None and ran >= max_chunks:
            return None
        k = state["chunks_done"]
        j0, j1 = k * chunk_entries, min(nnz, (k + 1) * chunk_entries)
        part = _chunk(g, off, nb, fl, j0, j1, nthreads)
        state["partial"] = [a + b for a, b in zip(state["partial"], part)]
        state["chunks_done"] = k + 1
        _write(path, state)
        ran += 1
    res = [0] * 16
    if g.n >= 3:
        res[1:] = state["partial"][1:]
        res[0] = choose3(g.n) - sum(res[1:])
    state["census"] = res
    _write(path, state)
    return res
