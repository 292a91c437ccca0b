"""Pins for the oracle's per-link adaptive penalties (the paper's future-work direction of learning
rates adaptive across parts of the topology; reading: link e's consensus and capacity constraints
carry the penalty beta * w_e, and the residual-balancing rule of section 3.4, applied per link on
that link's own residuals, moves w_e).  Each pin is independent of the oracle's formulas: a generic
minimiser of the weighted augmented Lagrangian, closed-form optima, KKT conditions with the
per-link multipliers, the full per-incidence form against the collapsed one, and the continuity of
the unscaled multipliers across a per-link change."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import workloads as W
from test_oracle_pins import U, _tiny_random


def _weighted_alm_min(w, y, ucon, uneg, D, udem, alpha, beta, x_start):
    """min over x, slack_dem >= 0, nu >= 0 of one commodity's augmented-Lagrangian terms in units of
    beta, the terms of link e on path r weighted by w_e (its penalty beta * w_e over beta)."""
    m = len(w)

    def f(z):
        x, sig, nu = z[:m], z[m], z[m + 1:]
        S = x.sum()
        if alpha > 0 and S <= 1e-12:
            return 1e30
        val = -U(S, alpha) / beta + 0.5 * (udem + S - D + sig) ** 2
        val += 0.5 * np.sum((uneg - x + nu) ** 2)
        for r in range(m):
            val += 0.5 * np.sum(w[r] * (ucon[r] + x[r] - y[r]) ** 2)
        return val

    z0 = np.concatenate([x_start, [0.0], np.maximum(x_start, 0.0)])
    bounds = [(None, None)] * m + [(0.0, None)] + [(0.0, None)] * m
    res = minimize(f, z0, method="L-BFGS-B", bounds=bounds,
                   options=dict(ftol=1e-16, gtol=1e-12, maxiter=20000, maxfun=200000))
    return res.x[:m], res.fun


@pytest.mark.parametrize("alpha", [0.0, 1.0, 2.5])
@pytest.mark.parametrize("seed", range(4))
def test_weighted_x_block_is_exact_minimiser(alpha, seed):
    rng = np.random.default_rng(300 + seed)
    m = int(rng.integers(1, 6))
    n = rng.integers(1, 5, m)
    w = [2.0 ** rng.integers(-3, 4, k) for k in n]  # per-link factors, powers of two as the rule makes
    y = [rng.uniform(0.0, 0.6, k) for k in n]
    ucon = [rng.uniform(0.0, 0.2, k) for k in n]
    uneg = rng.uniform(0.0, 0.3, m) * (rng.uniform(size=m) < 0.5)
    D, udem = rng.uniform(0.2, 1.5), rng.uniform(0.0, 0.3) * (rng.uniform() < 0.5)
    beta = float(rng.choice([0.5, 1.0, 4.0]))
    a = np.array([np.sum(w[r] * (y[r] - ucon[r])) for r in range(m)])
    Wr = np.array([np.sum(w[r]) for r in range(m)])
    S, x, _ = O.sum_root(a, Wr, uneg, D, udem, alpha, beta, D)
    # a generic minimiser from a generic start and from the oracle's point: the oracle's point is at
    # least as good as either, and the minimiser does not move away from it (the minimum is unique)
    _, f_gen = _weighted_alm_min(w, y, ucon, uneg, D, udem, alpha, beta, np.full(m, max(D, 0.1) / m))
    x_pol, f_pol = _weighted_alm_min(w, y, ucon, uneg, D, udem, alpha, beta, x)
    assert f_pol <= f_gen + 1e-9
    np.testing.assert_allclose(x, x_pol, atol=2e-5)


def _to_target(alpha, **kw):
    return O.Options(alpha_target=float(alpha), gamma=1e-10, max_iters=300000, project=False, per_link=True, **kw)


@pytest.mark.parametrize("L", [2, 3, 5])
@pytest.mark.parametrize("alpha", [1.0, 2.0])
def test_per_link_parking_lot_alpha_fair(L, alpha):
    inst = W.parking_lot(L)
    r = O.solve(inst, _to_target(alpha))
    assert r.flags & O.CONVERGED and r.final_alpha == alpha
    x0 = 1.0 / (1.0 + L ** (1.0 / alpha))
    assert r.S_raw[0] == pytest.approx(x0, abs=2e-6)
    np.testing.assert_allclose(r.S_raw[1:], 1.0 - x0, atol=2e-6)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 3.0])
def test_per_link_shared_link_waterfilling(alpha):
    inst = W.shared_link([0.1, 0.2, 0.5, 0.9], cap=1.0)
    r = O.solve(inst, _to_target(alpha))
    assert r.flags & O.CONVERGED
    np.testing.assert_allclose(r.S_raw * r.scale, [0.1, 0.2, 0.35, 0.35], atol=2e-6)


@pytest.mark.parametrize("D", [0.3, 0.5, 2.0])
def test_per_link_parallel_paths(D):
    inst = W.parallel_paths([0.2, 0.3], D)
    r = O.solve(inst, O.Options(sched_beta=np.full(3000, 16.0), sched_alpha=np.full(3000, 1.0), fixed_iters=3000,
                                project=False, per_link=True))
    assert r.S_raw[0] * r.scale == pytest.approx(min(D, 0.5), abs=2e-6)


@pytest.mark.parametrize("seed,alpha", [(0, 1.0), (1, 1.0), (3, 2.0)])
def test_per_link_kkt_at_convergence(seed, alpha):
    """KKT of the TE problem with the per-link multipliers lambda_e = beta * w_e * g_e:
    S_c^-alpha = mu_c + sum_{e in r} lambda_e - eta_r on every path, with complementary slackness."""
    inst = _tiny_random(seed)
    r = O.solve(inst, O.Options(alpha_target=alpha, gamma=1e-9, max_iters=200000, project=False, per_link=True))
    assert r.final_alpha == alpha and r.flags & O.CONVERGED
    assert np.any(r.w != 1.0)  # the rule did act
    b = r.beta
    lam = b * r.w * r.dual_cap
    mu = b * r.dual_dem
    eta = b * r.dual_neg
    S, x = r.S_raw, r.x_raw
    dem_of = np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))
    for p in range(inst.n_paths):
        links = inst.path_links[inst.path_ptr[p]:inst.path_ptr[p + 1]]
        assert S[dem_of[p]] ** -alpha == pytest.approx(mu[dem_of[p]] + lam[links].sum() - eta[p], rel=1e-4, abs=1e-6)
        assert eta[p] * max(x[p], 0.0) == pytest.approx(0.0, abs=1e-6)
    C = inst.capacity / r.scale
    L = O.link_loads(inst, x)
    assert np.all(L <= C * (1 + 1e-5))
    assert np.all(np.minimum(lam / lam.max(), (C - L) / C) < 1e-6)


def test_per_link_full_matches_collapsed(waxman20):
    """The collapse (dual_con_{e,r} = dual_cap_e, y_{e,r} = x_r + q_e) survives per-link factors."""
    opts = dict(fixed_iters=300, project=False, per_link=True)
    full = O.solve(waxman20, O.Options(**opts))
    col = O.solve(waxman20, O.Options(collapsed=True, **opts))
    assert full.collapse_dev < 1e-12
    assert np.any(full.w != 1.0)
    np.testing.assert_array_equal(full.w, col.w)
    np.testing.assert_allclose(col.x_raw, full.x_raw, rtol=0, atol=1e-9)


def test_per_link_rescale_keeps_unscaled_multipliers(waxman20):
    """With the cadence 5 the rule first acts after sweep 5: with it, every link's w_e * u_cap_e after
    that sweep equals u_cap_e of the same 5 sweeps with the factors pinned at 1 (w in [1, 1]); rates
    are untouched."""
    base = dict(fixed_iters=5, project=False, per_link=True, adapt_beta=False, beta_every=5)
    a = O.solve(waxman20, O.Options(**base))
    b = O.solve(waxman20, O.Options(w_min=1.0, w_max=1.0, **base))
    assert np.any(a.w != 1.0) and np.all(b.w == 1.0)
    assert set(np.unique(a.w)) <= {0.5, 1.0, 2.0}
    np.testing.assert_array_equal(a.x_raw, b.x_raw)
    np.testing.assert_allclose(a.w * a.dual_cap, b.dual_cap, rtol=1e-15, atol=0)
    path_of_inc = np.repeat(np.arange(waxman20.n_paths), np.diff(waxman20.path_ptr))
    np.testing.assert_allclose(a.w[waxman20.path_links] * a.dual_con, b.dual_con, rtol=1e-15, atol=0)
    assert path_of_inc.size == a.dual_con.size


def test_per_link_pinned_factors_equal_global(waxman20):
    """w pinned at 1 (bounds [1, 1]): per-link penalties are exactly the global iteration."""
    a = O.solve(waxman20, O.Options(fixed_iters=200, project=False))
    b = O.solve(waxman20, O.Options(fixed_iters=200, project=False, per_link=True, w_min=1.0, w_max=1.0))
    np.testing.assert_array_equal(a.x_raw, b.x_raw)
    np.testing.assert_array_equal(a.trace, b.trace)
