"""GPU checks of Algorithm 2 applied to given rates under a drifted network state (te_project_rates)
and of the drift-adjusted optimality built on it (section 4.1), against the FP64 oracle's Algorithm 2
and exact max-min allocations of the drifted states.

The bar for the applied rates is the one of the projection tests: the oracle's Algorithm 2 on the
same FP32 input rates, to 2e-6 relative (the GPU rounds its FP32 outputs toward zero), except for
paths whose trim order FP32 scores do not resolve (tests/projcheck.py).
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from projcheck import check_projection

pytestmark = pytest.mark.gpu

THETA = 1e-9


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def te(torch):
    import paper_2605_01748_amd as te_mod
    te_mod.library()
    return te_mod


@pytest.fixture(scope="module")
def c1():
    return W.waxman20(0)


@pytest.fixture(scope="module")
def solved_c1(te, c1):
    """A max-min solve of the 20-node instance at T_0 (adaptive stop, projection)."""
    prob = te.Problem(c1)
    x, S, st = prob.solve(te.Options(engine=te.ENGINE_GRAPH))
    return x.cpu().numpy(), float(st["final_alpha"])


# capacity events at 2,000 per day so that the later states include degraded links
TIMES = [0.0, 30.0, 300.0, 3000.0]


@pytest.fixture(scope="module")
def drifted_c1(c1):
    return W.drift_path(c1, TIMES, seed=3, cap_events_per_day=2000.0)


def _check_feasible(inst, x, x0):
    assert np.all(x >= 0)
    assert np.all(x <= np.maximum(x0, 0) * (1 + 1e-7) + 1e-30)
    assert np.all(O.link_loads(inst, x) <= inst.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(inst, x) <= inst.demand * (1 + 1e-7))


def test_project_rates_matches_oracle_under_drift(te, c1, solved_c1, drifted_c1):
    x0, alpha = solved_c1
    assert drifted_c1[-1].meta["drift"]["cap_events"] > 0
    prob = te.Problem(c1)
    for inst in drifted_c1:
        prob.update(capacity=inst.capacity, demand=inst.demand)
        xa, Sa = prob.project_rates(x0, alpha)
        xa = xa.cpu().numpy().astype(np.float64)
        print(f"{inst.name}: applied throughput {xa.sum():.4f} of {x0.sum():.4f}")
        _check_feasible(inst, xa, x0)
        check_projection(inst, x0, xa, alpha, tag=inst.name)
        np.testing.assert_allclose(Sa.cpu().numpy(), O.demand_sums(inst, xa), rtol=1e-6)
    # at T_0 the solve's own (feasible) allocation comes back unchanged
    prob.update(capacity=c1.capacity, demand=c1.demand)
    xa, _ = prob.project_rates(x0, alpha)
    np.testing.assert_allclose(xa.cpu().numpy(), x0, rtol=1e-6, atol=0)


def test_project_rates_waxman150(te):
    c2 = W.waxman150(0)
    prob = te.Problem(c2)
    x0, _, st = prob.solve(te.Options(fixed_iters=128))
    x0 = x0.cpu().numpy()
    inst = W.drift_path(c2, [300.0], seed=5, cap_events_per_day=20000.0)[0]
    assert inst.meta["drift"]["cap_events"] > 0
    prob.update(capacity=inst.capacity, demand=inst.demand)
    xa, Sa = prob.project_rates(x0, st["final_alpha"])
    xa = xa.cpu().numpy().astype(np.float64)
    _check_feasible(inst, xa, x0)
    check_projection(inst, x0, xa, st["final_alpha"], tag="waxman150 drifted 300 s")


def test_project_rates_ragged_and_in_place(te, torch):
    """Arbitrary rates (negative entries, far above the demands) on the edge-case instance: demands
    of 1 to 64 paths, a hot link on 40 % of the paths, unused zero-capacity links.  x_out may be
    x_in itself."""
    inst = W.ragged(0)
    rng = np.random.default_rng(2)
    dem_of = np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))
    x0 = (rng.uniform(-0.2, 1.5, inst.n_paths) * inst.demand[dem_of]).astype(np.float32)
    prob = te.Problem(inst)
    for alpha in (0.0, 1.0, 4.0):
        xa, _ = prob.project_rates(x0, alpha)
        xa = xa.cpu().numpy().astype(np.float64)
        _check_feasible(inst, xa, x0.astype(np.float64))
        check_projection(inst, x0, xa, alpha, tag=f"ragged alpha={alpha}")
        xt = torch.tensor(x0, device="cuda")
        xi, _ = prob.project_rates(xt, alpha, x_out=xt)
        assert xi.data_ptr() == xt.data_ptr()
        np.testing.assert_array_equal(xi.cpu().numpy(), xa.astype(np.float32))


def test_project_rates_rejects_bad_arguments(te, c1, solved_c1):
    x0, _ = solved_c1
    prob = te.Problem(c1)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(te.TEError):
            prob.project_rates(x0, bad)
    with pytest.raises(ValueError):
        prob.project_rates(x0[:-1], 1.0)


def test_project_rates_leaves_solver_state(te, c1, solved_c1):
    """te_project_rates uses the projection buffers only: a warm continuation after it is the same
    as one without it."""
    x0, alpha = solved_c1
    opts = dict(engine=te.ENGINE_GRAPH, project=False)
    runs = []
    for interleave in (False, True):
        prob = te.Problem(c1)
        prob.solve(te.Options(fixed_iters=40, **opts))
        if interleave:
            prob.project_rates(x0 * 3.0, alpha)
        x, _, _ = prob.solve(te.Options(fixed_iters=40, warm=True, **opts))
        runs.append(x.cpu().numpy())
    np.testing.assert_array_equal(runs[0], runs[1])


def test_drift_adjusted_optimality_matches_oracle(te, c1, solved_c1, drifted_c1):
    """DAO_K of the T_0 allocation at each drifted state, scored against the exact max-min allocation
    of that state: the GPU harness equals the oracle's Algorithm 2 + metric, DAO_0 is the plain
    optimality of the solve, and a state drifted for 50 minutes scores lower than T_0."""
    from paper_2605_01748_amd import dao
    x0, alpha = solved_c1
    prob = te.Problem(c1)
    vals = []
    for inst in drifted_c1:
        scale = float(inst.capacity[np.unique(inst.path_links)].max())
        opt, _ = O.maxmin_exact(inst)
        prob.update(capacity=inst.capacity, demand=inst.demand)
        v, xa, Sa = dao.drift_adjusted_optimality(prob, x0, alpha, opt, THETA * scale)
        ref = O.optimality(O.demand_sums(inst, O.project(inst, x0.astype(np.float64), alpha)), opt,
                           THETA * scale)
        print(f"DAO at t = {inst.meta['drift']['t']:g} s: {v:.5f} (oracle {ref:.5f})")
        assert abs(v - ref) <= 1e-5
        vals.append(v)
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "maxmin_waxman20_s0.npz"))["S"]
    scale0 = float(c1.capacity[np.unique(c1.path_links)].max())
    plain = O.optimality(O.demand_sums(c1, x0.astype(np.float64)), gold, THETA * scale0)
    assert abs(vals[0] - plain) <= 1e-5
    assert vals[-1] < vals[0]
