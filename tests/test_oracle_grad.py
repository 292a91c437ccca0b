"""Pins for the oracle's FP64 reverse pass: central finite differences of the oracle's own forward
sweeps (same schedule, unit scale frozen), and closed-form derivatives of a trivial instance."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _fd(inst, sb, sa, w, scale, h):
    fdC = np.zeros(inst.n_links)
    fdD = np.zeros(inst.n_demands)
    for e in range(inst.n_links):
        c = inst.capacity.copy()
        c[e] += h
        Sp, _, _ = O.grad(inst, sb, sa, w, scale=scale, capacity=c)
        c[e] -= 2 * h
        Sm, _, _ = O.grad(inst, sb, sa, w, scale=scale, capacity=c)
        fdC[e] = w @ (Sp - Sm) / (2 * h)
    for k in range(inst.n_demands):
        d = inst.demand.copy()
        d[k] += h
        Sp, _, _ = O.grad(inst, sb, sa, w, scale=scale, demand=d)
        d[k] -= 2 * h
        Sm, _, _ = O.grad(inst, sb, sa, w, scale=scale, demand=d)
        fdD[k] = w @ (Sp - Sm) / (2 * h)
    return fdC, fdD


@pytest.mark.parametrize("seed,K", [(0, 25), (1, 40), (3, 60)])
def test_reverse_pass_matches_central_differences(seed, K):
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_pins import _tiny_random
    inst = _tiny_random(seed)
    r = O.solve(inst, O.Options(fixed_iters=K, project=False), want_state=False)
    sb, sa = r.schedule
    w = np.random.default_rng(seed).uniform(0.5, 1.5, inst.n_demands)
    S, dC, dD = O.grad(inst, sb, sa, w)
    np.testing.assert_allclose(S, r.S_raw * r.scale, rtol=1e-10, atol=1e-12)
    s = O.used_scale(inst)
    fdC, fdD = _fd(inst, sb, sa, w, s, 1e-6 * s)
    tol = 1e-5 * max(np.abs(dC).max(), np.abs(dD).max(), 1.0)
    np.testing.assert_allclose(dC, fdC, atol=tol)
    np.testing.assert_allclose(dD, fdD, atol=tol)


def test_reverse_pass_sum_log_objective():
    """Cotangent 1/S gives the gradient of sum_c log S_c (the proportional-fairness utility)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_pins import _tiny_random
    inst = _tiny_random(0)
    K = 60
    r = O.solve(inst, O.Options(fixed_iters=K, project=False), want_state=False)
    sb, sa = r.schedule
    S0, _, _ = O.grad(inst, sb, sa, np.ones(inst.n_demands))
    assert S0.min() > 0  # the unprojected sums must be positive for the logarithm
    w = 1.0 / S0
    S, dC, dD = O.grad(inst, sb, sa, w)
    s = O.used_scale(inst)
    h = 1e-6 * s
    for e in range(0, inst.n_links, 3):
        c = inst.capacity.copy()
        c[e] += h
        Sp, _, _ = O.grad(inst, sb, sa, w, scale=s, capacity=c)
        c[e] -= 2 * h
        Sm, _, _ = O.grad(inst, sb, sa, w, scale=s, capacity=c)
        fd = (np.log(Sp).sum() - np.log(Sm).sum()) / (2 * h)
        assert dC[e] == pytest.approx(fd, rel=1e-4, abs=1e-5)


def test_one_sweep_single_link_closed_form():
    """One demand on one single-link path, alpha = 0 (U = S), beta = 1, one sweep from x^0 = y^0 = D.
    The sum equation is F(S) = (a - h(S)) - S with a = y^0 = D and h(S) = [S - D]_+ - 1: for S <= D,
    F = D + 1 - S > 0; above, F = 2D + 1 - 2S, so S = D + 1/2.  Hence dS/dD = 1 (half through a, half
    through h) and dS/dC = 0 (the capacity enters only the link step, after the rates are set)."""
    inst = W.make_instance("one", 2, [0], [1], [1.0], [0], [1], [0.5], [[[0]]])
    S, dC, dD = O.grad(inst, [1.0], [0.0], [1.0])
    assert S[0] == pytest.approx(0.5 + 0.5, abs=1e-12)
    assert dD[0] == pytest.approx(1.0, abs=1e-12)
    assert dC[0] == pytest.approx(0.0, abs=1e-12)
