"""Arc updates applied to a digraph, by their definition. TEST INFRASTRUCTURE
ONLY (same rules as the rest of the oracle package).

A batch of updates is a sequence of arc operations applied in order to the
set of arcs: an insertion adds the arc (nothing happens if it is present), a
deletion removes it (nothing happens if it is absent). The census of a graph
that changes over time (Sec. 3 of the paper: triad censuses taken at fixed
intervals of a traffic graph) is then the census of the arc set after each
batch, which the oracle's census computes from scratch."""
from __future__ import annotations

import numpy as np


def apply_updates(src, dst, upd_src, upd_dst, upd_insert):
    """Arc list (src, dst) after the updates, as two sorted int32 arrays
    (self-loops and duplicates of the input dropped)."""
    arcs = {(int(a), int(b)) for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()) if a != b}
    for a, b, ins in zip(np.asarray(upd_src).tolist(), np.asarray(upd_dst).tolist(),
                         np.asarray(upd_insert).tolist()):
        if a == b:
            raise ValueError("an update of a self-loop")
        if ins:
            arcs.add((int(a), int(b)))
        else:
            arcs.discard((int(a), int(b)))
    out = sorted(arcs)
    return (np.array([a for a, _ in out], dtype=np.int32), np.array([b for _, b in out], dtype=np.int32))
