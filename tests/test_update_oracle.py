"""Pins of the update semantics the incremental census is checked against
(CPU): hand-worked batches whose outcome the definition fixes."""
import numpy as np
import pytest

from oracle.update import apply_updates


def _set(s, d):
    return set(zip(s.tolist(), d.tolist()))


@pytest.mark.parametrize("start,ops,want", [
    ([], [(0, 1, 1)], {(0, 1)}),                               # insert
    ([(0, 1)], [(0, 1, 1)], {(0, 1)}),                         # insert a present arc: no change
    ([(0, 1)], [(1, 0, 1)], {(0, 1), (1, 0)}),                 # the reverse arc makes the pair mutual
    ([(0, 1), (1, 0)], [(0, 1, 0)], {(1, 0)}),                 # delete one direction of a mutual pair
    ([], [(2, 3, 0)], set()),                                  # delete an absent arc: no change
    ([], [(0, 1, 1), (0, 1, 0)], set()),                       # insert then delete
    ([(0, 1)], [(0, 1, 0), (0, 1, 1)], {(0, 1)}),              # delete then insert
    ([(0, 1)], [(0, 1, 0), (1, 0, 1), (0, 1, 1), (1, 0, 0)], {(0, 1)}),  # the last operation of each arc decides
    ([(5, 4), (4, 2)], [(4, 5, 1), (2, 4, 1), (4, 2, 0)], {(5, 4), (4, 5), (2, 4)}),
])
def test_hand_worked_batches(start, ops, want):
    s = np.array([a for a, _ in start], np.int32)
    d = np.array([b for _, b in start], np.int32)
    us = np.array([o[0] for o in ops], np.int32)
    ud = np.array([o[1] for o in ops], np.int32)
    ui = np.array([o[2] for o in ops], np.uint8)
    assert _set(*apply_updates(s, d, us, ud, ui)) == want


def test_self_loop_update_rejected():
    with pytest.raises(ValueError):
        apply_updates(np.zeros(0, np.int32), np.zeros(0, np.int32), [3], [3], [1])


def test_order_matters_only_within_an_arc():
    rng = np.random.default_rng(5)
    us = rng.integers(0, 6, 40).astype(np.int32)
    ud = rng.integers(0, 6, 40).astype(np.int32)
    keep = us != ud
    us, ud = us[keep], ud[keep]
    ui = rng.integers(0, 2, us.size).astype(np.uint8)
    base = _set(*apply_updates(np.zeros(0, np.int32), np.zeros(0, np.int32), us, ud, ui))
    # a stable reordering that keeps each arc's operations in order gives the same set
    order = np.argsort(us.astype(np.int64) * 100 + ud, kind="stable")
    assert _set(*apply_updates(np.zeros(0, np.int32), np.zeros(0, np.int32), us[order], ud[order], ui[order])) == base
