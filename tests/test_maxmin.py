"""Pins for the exact max-min checker (the ground truth of the paper's optimality metric)."""
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import coo_matrix

import oracle as O
import workloads as W


def test_parking_lot_maxmin_is_half():
    S, _ = O.maxmin_exact(W.parking_lot(4))
    np.testing.assert_allclose(S, 0.5, atol=1e-9)


def test_shared_link_waterfilling():
    S, _ = O.maxmin_exact(W.shared_link([0.1, 0.2, 0.5, 0.9]))
    np.testing.assert_allclose(S, [0.1, 0.2, 0.35, 0.35], atol=1e-9)


def test_two_level_hand_case():
    """f1 on A (cap 1), f2 on A then B (cap 3), f3 on B: levels 0.5, 0.5, 2.5."""
    inst = W.make_instance("two_level", 3, [0, 1], [1, 2], [1.0, 3.0], [0, 0, 1], [1, 2, 2], [9.0, 9.0, 9.0],
                           [[[0]], [[0, 1]], [[1]]])
    S, _ = O.maxmin_exact(inst)
    np.testing.assert_allclose(S, [0.5, 0.5, 2.5], atol=1e-9)


def _max_single(inst, c, lower):
    """max S_c s.t. S_c' >= lower_c' (given), S <= D, loads <= C, x >= 0."""
    E, P, D = inst.n_links, inst.n_paths, inst.n_demands
    dem_of_path = np.repeat(np.arange(D), np.diff(inst.demand_path_ptr))
    path_of_inc = np.repeat(np.arange(P), np.diff(inst.path_ptr))
    A_cap = coo_matrix((np.ones(inst.nnz), (inst.path_links, path_of_inc)), shape=(E, P))
    A_sum = coo_matrix((np.ones(P), (dem_of_path, np.arange(P))), shape=(D, P)).tocsr()
    from scipy.sparse import vstack
    A = vstack([A_cap, A_sum, -A_sum]).tocsr()
    b = np.concatenate([inst.capacity, inst.demand, -lower])
    cost = -A_sum[c].toarray().ravel()
    res = linprog(cost, A_ub=A, b_ub=b, bounds=(0, None), method="highs")
    assert res.status == 0
    return -res.fun


@pytest.mark.parametrize("which", ["waxman20", "tiny0", "tiny1"])
def test_definition_no_commodity_can_rise(which):
    """The max-min definition itself: raising any S_c forces lowering some S_c' <= S_c.
    For each c: max S_c subject to every c' with OPT_c' <= OPT_c keeping OPT_c' equals OPT_c."""
    if which == "waxman20":
        inst = W.waxman20(0)
    else:
        import sys
        import os
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        from test_oracle_pins import _tiny_random
        inst = _tiny_random(int(which[-1]))
    S, _ = O.maxmin_exact(inst)
    rng = np.random.default_rng(0)
    cs = np.arange(inst.n_demands) if inst.n_demands <= 60 else rng.choice(inst.n_demands, 60, replace=False)
    # include every commodity that is not demand-satisfied
    cs = np.union1d(cs, np.nonzero(S < inst.demand * (1 - 1e-7))[0])
    for c in cs:
        lower = np.where(S <= S[c] * (1 + 1e-9), S * (1 - 1e-9), 0.0)
        lower[c] = 0.0
        best = _max_single(inst, c, lower)
        assert best <= S[c] * (1 + 1e-6) + 1e-9, (c, best, S[c])


def test_drift_golden_matches_generator():
    """The stored exact max-min allocations of the drifted 150-node states belong to the states the
    generator produces (same fingerprints), one rate per demand within its demand."""
    import os
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "maxmin_waxman150_drift_s0.npz"))
    states = W.drift_path(W.waxman150(0), [float(t) for t in g["t"]], seed=0)
    for i, s in enumerate(states):
        assert str(g[f"fp{i}"]) == s.fingerprint()
        S = g[f"S{i}"]
        assert S.shape == (s.n_demands,)
        assert np.all(S >= 0) and np.all(S <= s.demand * (1 + 1e-9))
