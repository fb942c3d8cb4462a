"""The checkpointed oracle run: stopped after k chunks and resumed, in one or
several pieces, single- or multi-threaded, it gives the uninterrupted census;
a checkpoint of another graph or chunk size is refused; a half-written
temporary file is ignored. Pinned against the brute force on a small graph."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import checkpoint
from paper_1209_6308_amd import graphs

from _helpers import random_digraph


@pytest.fixture(scope="module")
def g():
    return graphs.rmat(11, 8, seed=21, recip_p=0.2)


def test_uninterrupted_run_equals_census(g, tmp_path):
    path = str(tmp_path / "c.json")
    got = checkpoint.census_resumable(g, path, chunk_entries=5000)
    assert got == oracle.census(g)
    st = json.load(open(path))
    assert st["chunks_done"] == st["chunks"] == (g.nnz + 4999) // 5000
    assert [int(x) for x in st["census"]] == got
    # a finished checkpoint answers at once
    assert checkpoint.census_resumable(g, path, chunk_entries=5000, max_chunks=0) == got


@pytest.mark.parametrize("pieces,threads", [((3,), (1, 1)), ((1, 2, 4), (1, 4)), ((5, 5, 5), (4, 1))])
def test_stop_and_resume(g, tmp_path, pieces, threads):
    path = str(tmp_path / "r.json")
    done = 0
    for i, k in enumerate(pieces):
        r = checkpoint.census_resumable(g, path, chunk_entries=3000, nthreads=threads[i % 2], max_chunks=k)
        done += k
        if r is None:
            st = json.load(open(path))
            assert st["chunks_done"] == done and st["census"] is None
    got = checkpoint.census_resumable(g, path, chunk_entries=3000, nthreads=threads[-1])
    assert got == oracle.census(g)


def test_refuses_other_graph_or_chunk_size(g, tmp_path):
    path = str(tmp_path / "x.json")
    assert checkpoint.census_resumable(g, path, chunk_entries=4000, max_chunks=2) is None
    with pytest.raises(ValueError, match="another graph"):
        checkpoint.census_resumable(graphs.rmat(11, 8, seed=22), path, chunk_entries=4000)
    with pytest.raises(ValueError, match="chunks of 4000"):
        checkpoint.census_resumable(g, path, chunk_entries=5000)


def test_half_written_temporary_is_ignored(g, tmp_path):
    path = str(tmp_path / "t.json")
    assert checkpoint.census_resumable(g, path, chunk_entries=6000, max_chunks=2) is None
    with open(path + ".tmp", "w") as f:
        f.write('{"format": 1, "chunks_do')  # a write cut short
    assert checkpoint.census_resumable(g, path, chunk_entries=6000) == oracle.census(g)


def test_pinned_to_brute_force(tmp_path):
    s, d = random_digraph(60, 0.3, 0.3, 5)
    h = graphs.build_csr(60, s, d)
    got = checkpoint.census_resumable(h, str(tmp_path / "b.json"), chunk_entries=37, max_chunks=None)
    assert got == oracle.brute(60, s, d)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_tiny_graphs(tmp_path, n):
    h = graphs.build_csr(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert checkpoint.census_resumable(h, str(tmp_path / f"{n}.json"), chunk_entries=10) == oracle.census(h)
