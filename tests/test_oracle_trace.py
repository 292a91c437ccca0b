"""Pins for the oracle's residuals, penalty rescale, stop rule, warm state and trim scores, each
against values derived by hand from the paper's definitions (not by re-running the oracle's
formulas) or against invariants that any correct implementation satisfies.

* Two sweeps on one link shared by two single-path demands, worked out by hand from the block
  minimisations (section 3.3 with the slacks of appendix B.1), the dual updates (section 3.3) and
  the residuals of section 3.4: every variable and both residuals after each sweep, with beta held
  at 1 and with beta doubled after the first sweep (the scaled duals divided by 2).
* The unscaled multipliers beta * u are unchanged by a rescale (every dual family), and the rate
  suggestions are not rescaled.
* The stagnation stop of Algorithm 1: an instance whose optimum does not depend on alpha stops on
  the first sweep after the first increment.
* Warm state (Algorithm 1's optional inputs): continuing a solve from its own state reproduces the
  uninterrupted run, including a penalty change at the seam and a change of units.
* Residual balancing with back-off: the beta sequence of a run on which the rule reverses is the
  rule's output for the residuals recorded, and the run converges where the rule without rests
  cycles; the back-off crosses a warm seam.
* Algorithm 2's score in FP64: scores closer than single precision resolves are still ordered.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _two_demands_one_link():
    # link 0 with capacity 1 shared by two demands of 1 (one path each): twice oversubscribed
    return W.shared_link([1.0, 1.0], cap=1.0)


# ------------------------------------------------------------------------------------------
# Hand trace, beta = 1, alpha = 0.
#   Start: x = y = 1 (x^0 = D / |P|), every dual 0.
#   Sweep 1.  a_r = y - u_con = 1; h(S) = [S - 1]_+ - 1 (S^-0 / beta = 1).  For 1 < S < 3 the rate
#   is xi(a - h) = 3 - S and F(S) = 3 - 2S, root S = 3/2: x = (3/2, 3/2).
#   Link: V = sum (x + u_con) = 3, g = [u_cap + V - C]_+ / (1 + n_e) = 2/3, y = x + u_con - g = 5/6.
#   Duals: u_dem = [0 + 3/2 - 1]_+ = 1/2, u_cap = [0 + 5/3 - 1]_+ = 2/3, u_con = [0 + 3/2 - 5/6]_+
#   = 2/3, u_neg = [0 - 3/2]_+ = 0.
#   s = ||x^1 - x^0|| = sqrt(2 (1/2)^2); r^2 = 2 (1/2)^2 + (2/3)^2 + 2 (2/3)^2 = 11/6.
#   Sweep 2.  a = 5/6 - 2/3 = 1/6; h(S) = [S - 1/2]_+ - 1; F(S) = 5/3 - 2S, S = 5/6: x = (5/6, 5/6).
#   V = 2 (5/6 + 2/3) = 3, g = (2/3 + 3 - 1) / 3 = 8/9, y = 5/6 + 2/3 - 8/9 = 11/18.
#   u_dem = [1/2 + 5/6 - 1]_+ = 1/3, u_cap = [2/3 + 11/9 - 1]_+ = 8/9, u_con = [2/3 + 5/6 - 11/18]_+ = 8/9.
#   s = sqrt(2 (2/3)^2); r^2 = 2 (1/6)^2 + 3 (2/9)^2.
# ------------------------------------------------------------------------------------------
HAND = {
    1: dict(x=1.5, y=5 / 6, udem=0.5, ucap=2 / 3, ucon=2 / 3, s=math.sqrt(0.5), r=math.sqrt(11 / 6)),
    2: dict(x=5 / 6, y=11 / 18, udem=1 / 3, ucap=8 / 9, ucon=8 / 9, s=math.sqrt(8 / 9),
            r=math.sqrt(2 / 36 + 3 * 4 / 81)),
}


@pytest.mark.parametrize("collapsed", [False, True])
@pytest.mark.parametrize("K", [1, 2])
def test_two_sweep_hand_trace(collapsed, K):
    inst = _two_demands_one_link()
    r = O.solve(inst, O.Options(fixed_iters=K, project=False, adapt_beta=False, alpha_target=0.0,
                                collapsed=collapsed))
    h = HAND[K]
    assert r.scale == 1.0
    np.testing.assert_allclose(r.x_raw, [h["x"]] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.S_raw, [h["x"]] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.y, [h["y"]] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_dem, [h["udem"]] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_cap, [h["ucap"]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_con, [h["ucon"]] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_neg, [0.0, 0.0], rtol=0, atol=0)
    for k in range(1, K + 1):
        assert r.trace[k - 1, 3] == pytest.approx(HAND[k]["s"], rel=1e-13)   # s_k
        assert r.trace[k - 1, 2] == pytest.approx(HAND[k]["r"], rel=1e-13)   # r_k
        assert r.trace[k - 1, 1] == 1.0 and r.trace[k - 1, 0] == 0.0


# ------------------------------------------------------------------------------------------
# Hand trace with beta doubled after sweep 1 (replayed schedule beta = (1, 2)): the scaled duals are
# divided by 2 before sweep 2 (u_dem 1/4, u_cap = u_con = 1/3), y stays 5/6.
#   Sweep 2.  a = 5/6 - 1/3 = 1/2; h(S) = [S - 3/4]_+ - 1/2; F(S) = 7/4 - 2S, S = 7/8.
#   V = 2 (7/8 + 1/3) = 29/12, g = (1/3 + 29/12 - 1) / 3 = 7/12, y = 7/8 + 1/3 - 7/12 = 5/8.
#   u_dem = [1/4 + 7/8 - 1]_+ = 1/8, u_cap = [1/3 + 5/4 - 1]_+ = 7/12, u_con = [1/3 + 7/8 - 5/8]_+ = 7/12.
#   r^2 = 2 (1/8)^2 + 3 (1/4)^2 = 7/32 (differences from the rescaled values), s = sqrt(2) 5/8.
# Without the rescale the root would be 7/12 instead of 7/8.
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("collapsed", [False, True])
def test_two_sweep_hand_trace_with_rescale(collapsed):
    inst = _two_demands_one_link()
    r = O.solve(inst, O.Options(fixed_iters=2, project=False, collapsed=collapsed,
                                sched_beta=np.array([1.0, 2.0]), sched_alpha=np.array([0.0, 0.0])))
    np.testing.assert_allclose(r.x_raw, [7 / 8] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.y, [5 / 8] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_dem, [1 / 8] * 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_cap, [7 / 12], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r.dual_con, [7 / 12] * 2, rtol=0, atol=1e-14)
    assert r.beta == 2.0
    assert r.trace[0, 2] == pytest.approx(math.sqrt(11 / 6), rel=1e-13)
    assert r.trace[1, 2] == pytest.approx(math.sqrt(7 / 32), rel=1e-13)
    assert r.trace[1, 3] == pytest.approx(math.sqrt(2) * 5 / 8, rel=1e-13)


@pytest.mark.parametrize("collapsed", [False, True])
def test_rescale_keeps_unscaled_multipliers(collapsed):
    """A change of beta after sweep K divides every scaled dual by the same factor, so the
    multipliers beta * u are continuous across it, and leaves the rates and rate suggestions."""
    inst = W.waxman20(0)
    K = 37
    sb = np.ones(K + 1)
    sb[K] = 4.0
    sa = np.zeros(K + 1)
    kw = dict(fixed_iters=K, project=False, collapsed=collapsed)
    before = O.solve(inst, O.Options(sched_beta=sb[:K], sched_alpha=sa[:K], **kw))
    after = O.solve(inst, O.Options(sched_beta=sb, sched_alpha=sa, **kw))
    assert before.beta == 1.0 and after.beta == 4.0
    for name in ("dual_dem", "dual_cap", "dual_neg", "dual_con"):
        u0, u1 = getattr(before, name), getattr(after, name)
        assert np.any(u0 != 0.0), name
        np.testing.assert_allclose(after.beta * u1, before.beta * u0, rtol=1e-15, atol=0, err_msg=name)
    np.testing.assert_array_equal(after.x_raw, before.x_raw)
    np.testing.assert_array_equal(after.y, before.y)


def test_stagnation_stop_when_optimum_does_not_move():
    """One demand on one link with D = C (1 in normalised units): S = 1 is optimal for every alpha
    (S^-alpha = 1 there), so the iterate does not move when alpha rises.  Algorithm 1 with the
    stagnation reading stops on the first sweep after the increment to alpha = 1 instead of
    climbing to alpha_max."""
    inst = W.shared_link([3.0], cap=3.0)
    r = O.solve(inst, O.Options(gamma=1e-6, max_iters=100000, project=False))
    alphas = r.trace[:, 0]
    assert r.flags & O.CONVERGED and not (r.flags & (O.HIT_ALPHA_MAX | O.HIT_MAX_ITERS))
    assert r.final_alpha == 1.0
    k_inc = int(np.argmax(alphas > 0.0))          # first sweep at alpha = 1
    assert k_inc > 0 and np.all(alphas[:k_inc] == 0.0)
    assert r.iters == k_inc + 1 and r.stop_iter == k_inc + 1
    assert r.trace[k_inc - 1, 2] <= 1e-6 and r.trace[k_inc - 1, 3] <= 1e-6
    assert r.S_raw[0] == pytest.approx(1.0, abs=1e-6)


# ------------------------------------------------------------------------------------------
# warm state
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("collapsed", [False, True])
def test_warm_continuation_replayed(collapsed):
    """K1 + K2 replayed sweeps in one run equal K1 sweeps, then K2 more from the state they left,
    with a penalty change exactly at the seam (the warm state's duals are scaled for the penalty
    of sweep K1 - 1 and are divided by the factor before sweep K1)."""
    inst = W.waxman20(0)
    K1, K2 = 30, 50
    ref = O.solve(inst, O.Options(fixed_iters=K1 + K2, project=False))
    sb, sa = ref.schedule
    sb = sb.copy()
    sb[K1:] *= 2.0  # the seam carries a change of beta
    kw = dict(project=False, collapsed=collapsed)
    full = O.solve(inst, O.Options(fixed_iters=K1 + K2, sched_beta=sb, sched_alpha=sa, **kw))
    first = O.solve(inst, O.Options(fixed_iters=K1, sched_beta=sb[:K1], sched_alpha=sa[:K1], **kw))
    assert first.beta == sb[K1 - 1]
    second = O.solve(inst, O.Options(fixed_iters=K2, sched_beta=sb[K1:], sched_alpha=sa[K1:], **kw),
                     warm=first.warm_state())
    # the state passes through caller units (x 100 and / 100): rounding only
    np.testing.assert_allclose(second.x_raw, full.x_raw, rtol=0, atol=1e-11)
    np.testing.assert_allclose(second.S_raw, full.S_raw, rtol=0, atol=1e-11)


def test_warm_continuation_adaptive():
    """Adaptive beta and alpha: 128 sweeps then 102 warm sweeps (a beta change decided after sweep
    128, an alpha increment after 131) follow the uninterrupted 230-sweep run, schedule included."""
    inst = W.waxman20(0)
    o = dict(project=False, gamma=3e-2)
    full = O.solve(inst, O.Options(fixed_iters=230, **o))
    first = O.solve(inst, O.Options(fixed_iters=128, **o))
    second = O.solve(inst, O.Options(fixed_iters=102, **o), warm=first.warm_state())
    b, a = full.trace[:, 1], full.trace[:, 0]
    assert b[128] != b[127] and a[131] != a[130]
    np.testing.assert_array_equal(second.trace[:, 1], b[128:])
    np.testing.assert_array_equal(second.trace[:, 0], a[128:])
    np.testing.assert_allclose(second.x_raw, full.x_raw, rtol=0, atol=1e-11)


def test_warm_state_converts_units():
    """Every capacity and demand doubled (the unit scale doubles): the warm state of the original
    instance, doubled, continues on the doubled instance exactly as the original continues (the
    normalised problems and states coincide), i.e. duals are converted like rates."""
    inst = W.waxman20(0)
    big = W.Instance(**{**inst.__dict__, "capacity": 2.0 * inst.capacity, "demand": 2.0 * inst.demand})
    first = O.solve(inst, O.Options(fixed_iters=25, project=False))
    ws = first.warm_state()
    ws2 = {k: (2.0 * v if isinstance(v, np.ndarray) else v) for k, v in ws.items()}
    o = O.Options(fixed_iters=40, project=False)
    a = O.solve(inst, o, warm=ws)
    b = O.solve(big, o, warm=ws2)
    assert b.scale == 2.0 * a.scale
    np.testing.assert_array_equal(b.x_raw, a.x_raw)
    np.testing.assert_array_equal(b.trace, a.trace)


# ------------------------------------------------------------------------------------------
# Algorithm 2's score in FP64
# ------------------------------------------------------------------------------------------
def test_projection_orders_scores_closer_than_single_precision():
    """Two single-path demands on link 0 (capacity 1) with rates 0.6 (1 + 1e-9) and 0.6: the scores
    S^alpha C_p (alpha = 1, C_p = 1) differ by one part in 1e9, which single precision does not
    resolve (it would see a tie and trim the higher path index).  The larger score is trimmed:
    path 0 gives up the whole excess."""
    inst = W.make_instance("near_tie", 3, [0, 0], [1, 2], [1.0, 5.0], [0, 0], [1, 2], [5.0, 5.0],
                           [[[0]], [[0]]])
    x = np.array([0.6 * (1 + 1e-9), 0.6])
    xp = O.project(inst, x, 1.0)
    np.testing.assert_allclose(xp, [1.0 - 0.6, 0.6], rtol=0, atol=1e-15)
    # with the order reversed the other path is trimmed
    xp2 = O.project(inst, x[::-1].copy(), 1.0)
    np.testing.assert_allclose(xp2, [0.6, 1.0 - 0.6], rtol=0, atol=1e-15)


def test_projection_stages():
    """The stage outputs: rates after the demand trims (sums capped at the demands, no rate raised)
    and the link phase's log-scores alpha ln S_c + ln C_p (-inf for paths off violated links)."""
    inst = W.waxman20(0)
    rng = np.random.default_rng(9)
    x = rng.uniform(0.0, 2.0, inst.n_paths) * inst.demand[np.repeat(np.arange(inst.n_demands),
                                                                    np.diff(inst.demand_path_ptr))]
    xp, xm, sc = O.project(inst, x, 2.0, stages=True)
    np.testing.assert_array_equal(xp, O.project(inst, x, 2.0))
    assert np.all(xm <= x) and np.all(O.demand_sums(inst, xm) <= inst.demand * (1 + 1e-12))
    L = O.link_loads(inst, xm)
    viol = L > inst.capacity
    path_of_inc = np.repeat(np.arange(inst.n_paths), np.diff(inst.path_ptr))
    Cp = np.bincount(path_of_inc, weights=viol[inst.path_links], minlength=inst.n_paths)
    S = O.demand_sums(inst, xm)[np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))]
    on = Cp > 0
    np.testing.assert_allclose(sc[on], 2.0 * np.log(S[on]) + np.log(Cp[on]), rtol=1e-15, atol=1e-15)
    assert np.all(np.isneginf(sc[~on]))


# ------------------------------------------------------------------------------------------
# Residual balancing with back-off.  The 2-link parking lot at alpha = 1 is an instance on which
# the rule applied after every sweep keeps beta cycling between two values and the iterate never
# settles; with the back-off (after the n-th reversal of beta's direction the rule rests for the
# next 2^n - 1 sweeps) it converges to the alpha-fair optimum (closed form in test_oracle_pins).
# ------------------------------------------------------------------------------------------
def _expected_betas(tr, beta0, A=10.0, C=2.0, every=1):
    """The beta of every sweep from the residuals the trace recorded, by the rule as defined: after
    sweep k (1-based count k + 1), if the cadence admits it and no rest is due, multiply by C when
    r > A s, divide by C when s > A r; a change against the previous direction is a reversal."""
    betas = [beta0]
    last, nrev, rest_until = 0, 0, 0
    for k in range(len(tr) - 1):
        b, r, s = betas[-1], tr[k, 2], tr[k, 3]
        d = 0
        if (k + 1) % every == 0 and k + 1 >= rest_until:
            d = 1 if r > A * s else (-1 if s > A * r else 0)
        if d != 0:
            if last != 0 and d != last:
                nrev += 1
                rest_until = k + 1 + 2 ** nrev
            last = d
        betas.append(b * C ** d)
    return np.array(betas)


def test_backoff_schedule_follows_the_rule():
    inst = W.parking_lot(2)
    r = O.solve(inst, O.Options(alpha_target=1.0, gamma=1e-10, max_iters=300000, project=False))
    tr = r.trace
    np.testing.assert_array_equal(tr[:, 1], _expected_betas(tr, 1.0))
    b = tr[:, 1]
    d = np.sign(np.diff(b))
    d = d[d != 0]
    assert np.count_nonzero(d[1:] != d[:-1]) >= 3      # the rule did reverse, several times
    # a rest was taken: some sweep had r > A s or s > A r while beta stayed
    ratio_hit = (tr[:-1, 2] > 10 * tr[:-1, 3]) | (tr[:-1, 3] > 10 * tr[:-1, 2])
    assert np.any(ratio_hit & (b[1:] == b[:-1]))
    assert r.flags & O.CONVERGED and r.final_alpha == 1.0


def test_backoff_cadence_and_warm_seam():
    """The cadence composes with the back-off, and a warm continuation carries the back-off: K1 + (400 -
    K1) sweeps equal 400 uninterrupted ones on the 2-link parking lot, the seam inside a rest after
    several reversals (K1 a multiple of the cadence, which counts from the start of each solve)."""
    inst = W.parking_lot(2)
    o = dict(alpha_target=1.0, gamma=1e-10, project=False)
    for every, K1 in ((1, 160), (3, 159)):
        full = O.solve(inst, O.Options(fixed_iters=400, beta_every=every, **o))
        np.testing.assert_array_equal(full.trace[:, 1], _expected_betas(full.trace, 1.0, every=every))
        first = O.solve(inst, O.Options(fixed_iters=K1, beta_every=every, **o))
        assert first.backoff[1] >= 3 and first.backoff[2] > 0
        second = O.solve(inst, O.Options(fixed_iters=400 - K1, beta_every=every, **o), warm=first.warm_state())
        np.testing.assert_array_equal(second.trace[:, 1], full.trace[K1:, 1])
        np.testing.assert_allclose(second.x_raw, full.x_raw, rtol=0, atol=1e-12)
