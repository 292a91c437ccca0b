"""The order-tolerant projection comparison (tests/projcheck.py) on hand cases: it marks exactly the
paths whose link-phase order FP32 scores cannot decide, and it still catches a wrong trim."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from projcheck import ambiguous_paths, check_projection


def _one_link(x):
    n = len(x)
    inst = W.make_instance("one-link", 2 * n + 2, [0], [1], [1.0], list(range(2, n + 2)),
                           list(range(n + 2, 2 * n + 2)), [10.0] * n, [[[0]] for _ in range(n)])
    return inst, np.asarray(x, np.float64)


def test_near_tie_marked_and_clear_order_not():
    # one link of capacity 1; three single-path demands; alpha = 1: score = ln S_c
    inst, x = _one_link([0.5, 0.5 * (1 + 1e-9), 0.2])
    _, xm, sc = O.project(inst, x, 1.0, stages=True)
    amb = ambiguous_paths(inst, xm, sc, 1.0)
    assert amb.tolist() == [True, True, False]
    # identical key inputs (same S, same count) tie by path index on both sides: not ambiguous
    inst2, x2 = _one_link([0.5, 0.5, 0.2])
    _, xm2, sc2 = O.project(inst2, x2, 1.0, stages=True)
    assert not ambiguous_paths(inst2, xm2, sc2, 1.0).any()
    # alpha = 0: the score is ln C_p alone, equal counts tie by index on both sides
    _, xm3, sc3 = O.project(inst, x, 0.0, stages=True)
    assert not ambiguous_paths(inst, xm3, sc3, 0.0).any()


def test_near_tie_next_to_a_tie_group_marks_the_group():
    # paths 0 and 1 have identical key inputs (equal sums), path 2 is a near-tie of both: FP32 may put
    # path 2 above or below the whole group, which changes the rate above each member of the group
    # (the 2-path group alone would keep its index order on both sides)
    inst, x = _one_link([0.5, 0.5, 0.5 * (1 + 1e-9), 0.2])
    _, xm, sc = O.project(inst, x, 1.0, stages=True)
    assert ambiguous_paths(inst, xm, sc, 1.0).tolist() == [True, True, True, False]
    # the same near-tie, its partner clearly apart from the group: only the near-tie pair is marked
    inst2, x2 = _one_link([0.5, 0.4, 0.5 * (1 + 1e-9), 0.2])
    _, xm2, sc2 = O.project(inst2, x2, 1.0, stages=True)
    assert ambiguous_paths(inst2, xm2, sc2, 1.0).tolist() == [True, False, True, False]


def test_check_projection_accepts_the_oracle_and_rejects_a_wrong_trim():
    inst, x = _one_link([0.6, 0.5, 0.2])
    ref = O.project(inst, x, 1.0)
    # the largest score (0.6) gives up the whole excess 0.3
    np.testing.assert_allclose(ref, [0.3, 0.5, 0.2])
    check_projection(inst, x, ref, 1.0)
    wrong = np.array([0.6, 0.2, 0.2])  # feasible, but the trim went to the wrong path
    with pytest.raises(AssertionError):
        check_projection(inst, x, wrong, 1.0)
