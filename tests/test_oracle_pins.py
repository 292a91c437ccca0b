"""Pins for the FP64 oracle against facts fixed independently of its own formulas.

* per-commodity and per-link block minimisations vs scipy's bounded quasi-Newton solver on
  the augmented-Lagrangian sub-problems written with explicit slack variables (section 3.2
  augmented Lagrangian, appendix B.1 slacks);
* closed forms: the alpha = 1 quadratic and alpha = 2 cubic of the sum equation with every
  hinge active (appendix B.2), the parking-lot alpha-fair optimum, water-filling on one shared
  link, one demand over parallel paths;
* the KKT conditions of the original TE problem (section 3.1) at a converged iterate (the
  approximate-KKT statement of the convergence proof, appendix C);
* Algorithm 2 hand cases and invariants (section 3.5);
* internal identities of the reading: the consensus duals equal the capacity dual of their link
  after every sweep, and the per-link collapsed bookkeeping reproduces the per-incidence one.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import workloads as W


def U(S, alpha):
    if alpha == 1.0:
        return math.log(S)
    return (S ** (1.0 - alpha) - 1.0) / (1.0 - alpha)


# ------------------------------------------------------------------------------------------
# x-block: one commodity
# ------------------------------------------------------------------------------------------
def _commodity_problem(rng, m):
    n = rng.integers(1, 5, m)                       # links per path
    y = [rng.uniform(0.0, 0.6, k) for k in n]      # rate suggestions y_{e,r}
    ucon = [rng.uniform(0.0, 0.2, k) for k in n]   # consensus duals
    uneg = rng.uniform(0.0, 0.3, m) * (rng.uniform(size=m) < 0.5)
    D = rng.uniform(0.2, 1.5)
    udem = rng.uniform(0.0, 0.3) * (rng.uniform() < 0.5)
    return n, y, ucon, uneg, D, udem


def _alm_commodity_min(n, y, ucon, uneg, D, udem, alpha, beta, x_start):
    """min over x, slack_dem >= 0, nu >= 0 of the commodity's augmented-Lagrangian terms."""
    m = len(n)

    def f(z):
        x, sig, nu = z[:m], z[m], z[m + 1:]
        S = x.sum()
        if alpha > 0 and S <= 1e-12:
            return 1e30
        val = -U(S, alpha) / beta + 0.5 * (udem + S - D + sig) ** 2
        val += 0.5 * np.sum((uneg - x + nu) ** 2)
        for r in range(m):
            val += 0.5 * np.sum((ucon[r] + x[r] - y[r]) ** 2)
        return val

    z0 = np.concatenate([x_start, [0.0], np.maximum(x_start, 0.0)])
    bounds = [(None, None)] * m + [(0.0, None)] + [(0.0, None)] * m
    res = minimize(f, z0, method="L-BFGS-B", bounds=bounds,
                   options=dict(ftol=1e-16, gtol=1e-12, maxiter=20000, maxfun=200000))
    return res.x[:m], res.fun


@pytest.mark.parametrize("alpha", [0.0, 1.0, 2.0, 3.5])
@pytest.mark.parametrize("seed", range(5))
def test_x_block_is_exact_minimiser(alpha, seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(1, 6))
    n, y, ucon, uneg, D, udem = _commodity_problem(rng, m)
    beta = float(rng.choice([0.5, 1.0, 4.0]))
    a = np.array([np.sum(y[r] - ucon[r]) for r in range(m)])
    S, x, _ = O.sum_root(a, n, uneg, D, udem, alpha, beta, D)
    assert S == pytest.approx(x.sum(), rel=1e-10, abs=1e-12)
    x_ref, f_ref = _alm_commodity_min(n, y, ucon, uneg, D, udem, alpha, beta, np.full(m, max(D, 0.1) / m))
    # the oracle's point must be at least as good as the generic solver's, and close to it
    _, f_or = _alm_commodity_min(n, y, ucon, uneg, D, udem, alpha, beta, x)
    assert f_or <= f_ref + 1e-9
    np.testing.assert_allclose(x, x_ref, atol=2e-5)


def test_sum_root_alpha1_quadratic():
    """All hinges active: (1+w) S - K - (w/beta) / S = 0, w = sum 1/(1+n_r),
    K = sum (a_r + u_r)/(1+n_r) + w (D - udem)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        m = int(rng.integers(1, 6))
        n = rng.integers(1, 5, m)
        uneg = rng.uniform(0.5, 1.0, m)        # large dual_neg: every path on the (n+1) branch
        a = rng.uniform(-0.5, 0.2, m)
        D = rng.uniform(0.0, 0.05)             # tiny demand: the demand hinge is active
        udem = rng.uniform(0.0, 0.1)
        beta = float(rng.uniform(0.5, 3.0))
        S, x, _ = O.sum_root(a, n, uneg, D, udem, 1.0, beta, 0.3)
        w = np.sum(1.0 / (1 + n))
        K = np.sum((a + uneg) / (1 + n)) + w * (D - udem)
        S_cf = (K + math.sqrt(K * K + 4 * (1 + w) * w / beta)) / (2 * (1 + w))
        # the closed form holds only if the hinges it assumes are active at S_cf
        h = (S_cf - D + udem) - 1.0 / (beta * S_cf)
        if S_cf - D + udem > 0 and np.all(a - h < n * uneg):
            assert S == pytest.approx(S_cf, rel=1e-11)


def test_sum_root_alpha2_cubic():
    """All hinges active, alpha = 2: (1+w) S^3 - K S^2 - w/beta = 0 (numpy.roots)."""
    rng = np.random.default_rng(8)
    checked = 0
    for _ in range(40):
        m = int(rng.integers(1, 6))
        n = rng.integers(1, 5, m)
        uneg = rng.uniform(0.5, 1.0, m)
        a = rng.uniform(-0.5, 0.2, m)
        D = rng.uniform(0.0, 0.05)
        udem = rng.uniform(0.0, 0.1)
        beta = float(rng.uniform(0.5, 3.0))
        S, x, _ = O.sum_root(a, n, uneg, D, udem, 2.0, beta, 0.3)
        w = np.sum(1.0 / (1 + n))
        K = np.sum((a + uneg) / (1 + n)) + w * (D - udem)
        roots = np.roots([1 + w, -K, 0.0, -w / beta])
        real = [z.real for z in roots if abs(z.imag) < 1e-9 and z.real > 0]
        assert len(real) == 1
        S_cf = real[0]
        h = (S_cf - D + udem) - 1.0 / (beta * S_cf ** 2)
        if S_cf - D + udem > 0 and np.all(a - h < n * uneg):
            assert S == pytest.approx(S_cf, rel=1e-10)
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("alpha", [0.0, 1.0, 3.0])
def test_sum_root_any_warm_start_and_brute_force(alpha):
    """The safeguarded Newton root does not depend on its warm start (bracket growth from far below
    and far above, halving towards 0 for alpha > 0), and equals a plain 300-step bisection of the
    sum equation (F decreasing; appendix B.2) on the same data."""
    rng = np.random.default_rng(11 + int(alpha))
    for _ in range(25):
        m = int(rng.integers(1, 9))
        n = rng.integers(1, 9, m)
        uneg = rng.uniform(0.0, 0.5, m) * (rng.uniform(size=m) < 0.5)
        a = rng.uniform(-1.0, 2.0, m)
        D = float(rng.uniform(0.01, 2.0))
        udem = float(rng.uniform(0.0, 0.5)) * float(rng.uniform() < 0.5)
        beta = float(10.0 ** rng.uniform(-2, 2))

        def F(S):
            h = max(S - D + udem, 0.0) - (S ** -alpha if alpha > 0 else 1.0) / beta
            b = a - h
            x = np.where(b >= n * uneg, b / n, (b + uneg) / (n + 1))
            return x.sum() - S

        lo, hi = (1e-60, 1e6) if alpha > 0 else (-1e6, 1e6)
        assert F(lo) > 0 > F(hi)
        for _ in range(300):
            mid = 0.5 * (lo + hi)
            if F(mid) > 0:
                lo = mid
            else:
                hi = mid
        roots = [O.sum_root(a, n, uneg, D, udem, alpha, beta, S0)[0] for S0 in (1e-9, 1e-3, 1.0, 1e3, 1e6)]
        for r in roots:
            assert r == pytest.approx(lo, rel=1e-10, abs=1e-13)


# ------------------------------------------------------------------------------------------
# y-block: one link, read back from the oracle after one and two sweeps
# ------------------------------------------------------------------------------------------
def _link_min(C, ucap, ucon, x):
    """min over y, slack_cap >= 0 of 1/2 (ucap + sum y - C + tau)^2 + sum 1/2 (ucon + x - y)^2."""
    m = len(x)

    def f(z):
        yv, tau = z[:m], z[m]
        return 0.5 * (ucap + yv.sum() - C + tau) ** 2 + 0.5 * np.sum((ucon + x - yv) ** 2)

    res = minimize(f, np.concatenate([x, [0.0]]), method="L-BFGS-B", bounds=[(None, None)] * m + [(0, None)],
                   options=dict(ftol=1e-16, gtol=1e-13, maxiter=20000))
    return res.x[:m]


def test_y_block_is_exact_minimiser(waxman20):
    inst = waxman20
    opt = O.Options(fixed_iters=1, project=False, adapt_beta=False)
    r1 = O.solve(inst, opt)
    r2 = O.solve(inst, O.Options(fixed_iters=2, project=False, adapt_beta=False))
    C = inst.capacity / r1.scale
    path_of_inc = np.repeat(np.arange(inst.n_paths), np.diff(inst.path_ptr))
    rng = np.random.default_rng(0)
    links = rng.choice(inst.n_links, 25, replace=False)
    for e in links:
        inc = np.nonzero(inst.path_links == e)[0]
        if len(inc) == 0:
            continue
        # sweep 1: duals start at zero
        y_ref = _link_min(C[e], 0.0, np.zeros(len(inc)), r1.x_raw[path_of_inc[inc]])
        np.testing.assert_allclose(r1.y[inc], y_ref, atol=1e-7)
        # sweep 2: duals from sweep 1, x from sweep 2
        y_ref2 = _link_min(C[e], r1.dual_cap[e], r1.dual_con[inc], r2.x_raw[path_of_inc[inc]])
        np.testing.assert_allclose(r2.y[inc], y_ref2, atol=1e-7)


# ------------------------------------------------------------------------------------------
# closed-form optima
# ------------------------------------------------------------------------------------------
def _fixed_alpha(K, alpha, beta=1.0):
    return O.Options(sched_beta=np.full(K, beta), sched_alpha=np.full(K, float(alpha)), fixed_iters=K,
                     project=False)


def _to_target(alpha):
    """The paper's loop (adaptive beta, alpha-continuation) run to a finite target."""
    return O.Options(alpha_target=float(alpha), gamma=1e-10, max_iters=300000, project=False)


@pytest.mark.parametrize("L", [2, 3, 5])
@pytest.mark.parametrize("alpha", [1.0, 2.0, 4.0])
def test_parking_lot_alpha_fair(L, alpha):
    inst = W.parking_lot(L)
    r = O.solve(inst, _to_target(alpha))
    assert r.flags & O.CONVERGED and r.final_alpha == alpha
    x0 = 1.0 / (1.0 + L ** (1.0 / alpha))
    assert r.S_raw[0] == pytest.approx(x0, abs=2e-6)
    np.testing.assert_allclose(r.S_raw[1:], 1.0 - x0, atol=2e-6)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 3.0])
def test_shared_link_waterfilling(alpha):
    """Single shared link with demand caps: water-filling, the same for every alpha > 0."""
    inst = W.shared_link([0.1, 0.2, 0.5, 0.9], cap=1.0)
    r = O.solve(inst, _to_target(alpha))
    assert r.flags & O.CONVERGED
    np.testing.assert_allclose(r.S_raw * r.scale, [0.1, 0.2, 0.35, 0.35], atol=2e-6)


@pytest.mark.parametrize("D", [0.3, 0.5, 2.0])
def test_parallel_paths(D):
    inst = W.parallel_paths([0.2, 0.3], D)
    r = O.solve(inst, _fixed_alpha(3000, 1.0, beta=16.0))
    assert r.S_raw[0] * r.scale == pytest.approx(min(D, 0.5), abs=2e-6)


def _tiny_random(seed, n=7, links=12, k=3):
    rng = np.random.default_rng(np.random.SeedSequence([99, seed]))
    pos, edges = W.waxman(n, links, rng, tol=0.35)
    cap = rng.choice([1.0, 2.0, 5.0], size=len(edges))
    src, dst, capa, _ = W.arcs_from_edges(edges, cap)
    wts = rng.lognormal(0, 1, n)
    pairs = [(s, t) for s in range(n) for t in range(n) if s != t]
    base = W.gravity(wts, np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]))
    paths = W.k_shortest_paths(n, src, dst, np.ones(len(src)), [p[0] for p in pairs], [p[1] for p in pairs], k)
    inst = W.make_instance("tiny", n, src, dst, capa, [p[0] for p in pairs], [p[1] for p in pairs], base, paths)
    lam = W.max_concurrent_flow(inst, base)
    inst.demand = 2.0 * lam * base
    return inst


@pytest.mark.parametrize("seed,alpha", [(0, 1.0), (1, 1.0), (2, 1.0), (3, 1.0), (1, 2.0), (3, 2.0)])
def test_kkt_at_convergence(seed, alpha):
    """At a converged iterate the scaled duals times beta are KKT multipliers of the TE problem:
    S_c^-alpha = mu_c + sum_{e in r} lambda_e - eta_r on every path, with complementary slackness.
    (Cases chosen to converge to gamma = 1e-9 within the sweep budget; demand-capped small
    commodities need multipliers D^-alpha, which the bounded beta reaches slowly at large alpha.)"""
    inst = _tiny_random(seed)
    r = O.solve(inst, O.Options(alpha_target=alpha, gamma=1e-9, max_iters=200000, project=False))
    assert r.final_alpha == alpha and r.flags & O.CONVERGED
    b = r.beta
    lam = b * r.dual_cap
    mu = b * r.dual_dem
    eta = b * r.dual_neg
    S = r.S_raw
    x = r.x_raw
    dem_of = np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))
    for p in range(inst.n_paths):
        links = inst.path_links[inst.path_ptr[p]:inst.path_ptr[p + 1]]
        c = dem_of[p]
        lhs = S[c] ** -alpha
        rhs = mu[c] + lam[links].sum() - eta[p]
        assert lhs == pytest.approx(rhs, rel=1e-4, abs=1e-6)
        assert eta[p] * max(x[p], 0.0) == pytest.approx(0.0, abs=1e-6)
    C = inst.capacity / r.scale
    Dn = inst.demand / r.scale
    L = O.link_loads(inst, x)
    assert np.all(L <= C * (1 + 1e-5))
    assert np.all(S <= Dn * (1 + 1e-5))
    # complementary slackness, scale-free: a multiplier is ~0 or its constraint is ~tight
    assert np.all(np.minimum(lam / lam.max(), (C - L) / C) < 1e-6)
    assert np.all(np.minimum(mu / mu.max(), (Dn - S) / Dn) < 1e-6)
    assert np.all(x >= -1e-6)


# ------------------------------------------------------------------------------------------
# Algorithm 2
# ------------------------------------------------------------------------------------------
def test_projection_hand_case_link_phase():
    """Link 0 (cap 1) carries path A of commodity a (x=0.6, S_a=0.8 via path A2 on link 1)
    and path B of commodity b (x=0.5, S_b=0.5): violation 0.1, alpha = 1, score_A = 0.8 > 0.5,
    so A is trimmed by 0.1."""
    inst = W.make_instance("hand", 3, [0, 0], [1, 2], [1.0, 1.0], [0, 0], [1, 1], [5.0, 5.0],
                           [[[0], [1]], [[0]]])
    x = np.array([0.6, 0.2, 0.5])
    xp = O.project(inst, x, 1.0)
    np.testing.assert_allclose(xp, [0.5, 0.2, 0.5], atol=1e-15)


def test_projection_hand_case_demand_phase():
    """Commodity with D = 1 and x = (0.5, 0.4, 0.3): excess 0.2 is trimmed from the path
    crossing the most violated links first (path 2 crosses the violated link 1)."""
    inst = W.make_instance("hand", 3, [0, 0, 1], [1, 1, 2], [5.0, 0.1, 5.0], [0, 1], [1, 2], [1.0, 5.0],
                           [[[0], [0], [1]], [[2]]])
    x = np.array([0.5, 0.4, 0.3, 0.1])
    xp = O.project(inst, x, 1.0)
    # demand phase: path 2 (C_p = 1) first: trimmed by 0.2 -> 0.1; link 1 then carries 0.1 = cap
    np.testing.assert_allclose(xp, [0.5, 0.4, 0.1, 0.1], atol=1e-15)


def test_projection_parallel_links_take_max():
    """Two violated links share one path; each trims from the same snapshot and the path gives
    up the larger trim."""
    inst = W.make_instance("hand", 3, [0, 1], [1, 2], [1.0, 1.0], [0, 0, 1], [2, 1, 2], [9.0, 9.0, 9.0],
                           [[[0, 1]], [[0]], [[1]]])
    x = np.array([0.6, 0.6, 0.45])   # link 0: 1.2 (V=0.2), link 1: 1.05 (V=0.05)
    xp = O.project(inst, x, 0.0)
    # alpha = 0: score = C_p; path 0 crosses both violated links (C=2) -> trimmed first on both;
    # link 0 asks 0.2, link 1 asks 0.05 -> path 0 loses max = 0.2
    np.testing.assert_allclose(xp, [0.4, 0.6, 0.45], atol=1e-15)


def test_projection_invariants_random(waxman20):
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.5, 3.0, waxman20.n_paths) * rng.uniform(size=waxman20.n_paths) ** 2 * 10
    xp = O.project(waxman20, x, 2.0)
    assert np.all(xp >= 0)
    S = O.demand_sums(waxman20, xp)
    L = O.link_loads(waxman20, xp)
    assert np.all(S <= waxman20.demand * (1 + 1e-12))
    assert np.all(L <= waxman20.capacity * (1 + 1e-9))
    assert np.all(xp <= np.maximum(x, 0) + 1e-15)


def test_projection_under_demand_drift_closed_form(waxman20):
    """Rates that fit the capacities, applied under drifted demands with unchanged capacities (the
    drift-adjusted optimality of section 4.1): only demand trims act, so every demand gets exactly
    min(S_c, D_c') and no path rises."""
    r = O.solve(waxman20, O.Options(fixed_iters=400))
    later = W.drift_path(waxman20, [300.0], seed=2, cap_events_per_day=0.0)[0]
    assert np.any(later.demand < r.S) and np.any(later.demand > r.S)
    xa = O.project(later, r.x, 2.0)
    np.testing.assert_allclose(O.demand_sums(later, xa), np.minimum(r.S, later.demand), rtol=1e-12, atol=1e-15)
    assert np.all(xa <= r.x)


def test_projection_under_capacity_cut(waxman20):
    """The same rates after one link's capacity is halved: feasible, no demand gains, and the
    demands none of whose paths cross an over-full link keep their rates (up to the last-bit
    demand trims of rates whose sum rounds above the demand)."""
    r = O.solve(waxman20, O.Options(fixed_iters=400))
    L = O.link_loads(waxman20, r.x)
    e = int(np.argmax(L))
    cap = waxman20.capacity.copy()
    cap[e] *= 0.5
    later = W.Instance(**{**waxman20.__dict__, "capacity": cap})
    xa = O.project(later, r.x, 2.0)
    Sa = O.demand_sums(later, xa)
    assert np.all(O.link_loads(later, xa) <= cap * (1 + 1e-12))
    assert np.all(Sa <= r.S * (1 + 1e-15))
    over = O.link_loads(later, r.x) > cap
    S0 = O.demand_sums(waxman20, r.x)
    for c in range(waxman20.n_demands):
        ps = range(waxman20.demand_path_ptr[c], waxman20.demand_path_ptr[c + 1])
        if not any(over[waxman20.path_links[waxman20.path_ptr[p]:waxman20.path_ptr[p + 1]]].any() for p in ps):
            assert abs(Sa[c] - S0[c]) <= 1e-14 * S0[c]
    assert Sa.sum() < r.S.sum()


# ------------------------------------------------------------------------------------------
# whole-solve invariants and identities
# ------------------------------------------------------------------------------------------
def test_consensus_duals_collapse(waxman20):
    r = O.solve(waxman20, O.Options(fixed_iters=300, project=False))
    assert r.collapse_dev < 1e-12
    # after each sweep y_{e,r} = x_r + q_e with one offset q_e per link
    path_of_inc = np.repeat(np.arange(waxman20.n_paths), np.diff(waxman20.path_ptr))
    q = r.y - r.x_raw[path_of_inc]
    for e in range(waxman20.n_links):
        qe = q[waxman20.path_links == e]
        if len(qe):
            assert np.ptp(qe) < 1e-12


def test_collapsed_matches_full(waxman20):
    full = O.solve(waxman20, O.Options(fixed_iters=300, project=False))
    sb, sa = full.schedule
    opts = dict(fixed_iters=300, project=False, sched_beta=sb, sched_alpha=sa)
    a = O.solve(waxman20, O.Options(**opts))
    b = O.solve(waxman20, O.Options(collapsed=True, **opts))
    np.testing.assert_allclose(a.x_raw, full.x_raw, rtol=0, atol=1e-13)
    # same algebra, different summation order: agreement to rounding accumulated over 300 sweeps
    np.testing.assert_allclose(b.x_raw, a.x_raw, rtol=0, atol=1e-9)
    np.testing.assert_allclose(b.S_raw, a.S_raw, rtol=0, atol=1e-9)


def test_projected_solution_feasible_and_near_maxmin(waxman20):
    gold = np.load(_golden("maxmin_waxman20_s0.npz"))
    assert str(gold["fingerprint"]) == waxman20.fingerprint()
    r = O.solve(waxman20, O.Options(fixed_iters=1500))
    L = O.link_loads(waxman20, r.x)
    assert np.all(r.x >= 0)
    assert np.max((L - waxman20.capacity) / waxman20.capacity) <= 1e-9
    assert np.all(r.S <= waxman20.demand * (1 + 1e-9))
    assert O.optimality(r.S, gold["S"], 1e-9) >= 0.99
    # bottleneck property: every unsatisfied demand has, on each path, a nearly saturated link
    unsat = r.S < (1 - 1e-6) * waxman20.demand
    for c in np.nonzero(unsat)[0]:
        for p in range(waxman20.demand_path_ptr[c], waxman20.demand_path_ptr[c + 1]):
            links = waxman20.path_links[waxman20.path_ptr[p]:waxman20.path_ptr[p + 1]]
            assert np.max(L[links] / waxman20.capacity[links]) >= 1 - 1e-3


def test_slater_point_feasible(waxman20):
    """Appendix C Part I(b): x_r = eps / m_c is strictly feasible for small eps."""
    m = np.diff(waxman20.demand_path_ptr)
    dem_of = np.repeat(np.arange(waxman20.n_demands), m)
    kappa = O.link_loads(waxman20, 1.0 / m[dem_of])
    used = kappa > 0
    eps = 0.5 * min(waxman20.demand.min(), np.min(waxman20.capacity[used] / kappa[used]))
    x = eps / m[dem_of]
    assert np.all(O.link_loads(waxman20, x) < waxman20.capacity)
    assert np.all(O.demand_sums(waxman20, x) < waxman20.demand)


def test_schedule_replay_is_exact(waxman20):
    a = O.solve(waxman20, O.Options(fixed_iters=200))
    sb, sa = a.schedule
    b = O.solve(waxman20, O.Options(fixed_iters=200, sched_beta=sb, sched_alpha=sa))
    np.testing.assert_array_equal(a.x, b.x)


def test_alpha_continuation_and_stop():
    """alpha rises 0, 1, 2, ... each time the residuals drop below gamma, and a finite target stops
    the solve once converged at that target."""
    inst = W.parking_lot(3)
    r = O.solve(inst, O.Options(alpha_target=3.0, gamma=1e-6, max_iters=100000, project=False))
    assert r.flags & O.CONVERGED and r.final_alpha == 3.0
    alphas = r.trace[:, 0]
    steps = np.unique(alphas)
    np.testing.assert_array_equal(steps, [0.0, 1.0, 2.0, 3.0])
    assert np.all(np.diff(alphas) >= 0)
    # the iteration before each increment had both residuals at or below gamma
    for k in np.nonzero(np.diff(alphas))[0]:
        assert r.trace[k, 2] <= 1e-6 and r.trace[k, 3] <= 1e-6
    x0 = 1.0 / (1.0 + 3 ** (1.0 / 3.0))
    assert r.S_raw[0] == pytest.approx(x0, abs=1e-4)


def _golden(name):
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
