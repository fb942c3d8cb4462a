"""The benchmark's algorithmic byte count (CPU): the closed-form sums that
bench.py evaluates on the device equal the entries the merge reads, counted
task by task from the CSR (N(u) from its first id above u, N(v) from u on)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from paper_1209_6308_amd import graphs  # noqa: E402


def _entries_by_task(g):
    off, nbr = g.offsets, g.nbrs
    a_sum = b_sum = 0
    for u in range(g.n):
        row = nbr[off[u]:off[u + 1]]
        above = row[row > u]
        for v in above.tolist():
            rv = nbr[off[v]:off[v + 1]]
            a_sum += above.size                         # ids of N(u) above u
            b_sum += int(rv.size - np.searchsorted(rv, u))  # ids of N(v) from u on
    return a_sum, b_sum


def test_list_byte_sums_match_task_counts():
    import torch
    for g in (graphs.rmat(9, 8, seed=3, recip_p=0.2), graphs.chung_lu(600, 2.1, 8.0, 60.0, seed=2)):
        want = _entries_by_task(g)
        got = bench.list_byte_sums(torch.from_numpy(g.offsets), torch.from_numpy(g.nbrs), g.n)
        assert got == want
