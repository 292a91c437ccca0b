"""Exact max-min fair allocation by progressive filling of LPs.

TEST INFRASTRUCTURE ONLY.  This is the ground truth the paper measures
optimality against (section 4.1, "Optimality": distance to the max-min fair
allocation OPT), and the alpha -> infinity end of the alpha-fair family
(section 3.1, objective table).

Definition used (textbook max-min fairness over the TE polytope of section
3.1, paths fixed): the vector of demand sums S is max-min fair when no S_c can
be raised without lowering some S_c' <= S_c.  Water-filling computes it level
by level.  Each round, with F the frozen commodities (fixed at f_c) and A the
active ones:

  1. bulk step: the largest threshold T among the active demands such that
     every active c can get min(T, D_c) at once.  It is found by galloping and
     bisection over the sorted active demands with the always-feasible LP
        theta(T) = max theta  s.t.  S_c >= theta * min(T, D_c)  (c in A),
                                    S_c >= f_c (c in F), S_c <= D_c, loads <= C, x >= 0
     (T passes iff theta(T) >= 1; the predicate is monotone in T).  Every
     active c with D_c <= T is then demand-satisfied in the max-min allocation
     and is frozen at D_c.
  2. bottleneck step: t* = max t  s.t.  S_c >= t (c in A), S_c >= f_c (c in F),
     S_c <= D_c, loads <= C.  Every active c whose row S_c >= t has a non-zero
     dual cannot exceed t* (complementary slackness holds in every optimal
     solution, and every allocation keeping all active commodities >= t* is
     optimal); those are frozen at t*.  The duals of these rows sum to one, so
     at least one commodity is frozen per round.

The LPs are solved with HiGHS through scipy.optimize.linprog.
"""
from __future__ import annotations

import time

import numpy as np


def maxmin_exact(inst, dual_tol: float = 1e-7, rel_tol: float = 1e-9, verbose: bool = False):
    """Returns (S_opt [D] in original units, info dict)."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix, csr_matrix, hstack, vstack

    E, P, D = inst.n_links, inst.n_paths, inst.n_demands
    used = np.zeros(E, bool)
    used[inst.path_links] = True
    scale = float(inst.capacity[used].max())
    C = inst.capacity / scale
    Dm = inst.demand / scale
    dem_of_path = np.repeat(np.arange(D), np.diff(inst.demand_path_ptr))
    path_of_inc = np.repeat(np.arange(P), np.diff(inst.path_ptr))
    cap_rows = coo_matrix((np.ones(inst.nnz), (inst.path_links, path_of_inc)), shape=(E, P)).tocsr()
    sum_rows = coo_matrix((np.ones(P), (dem_of_path, np.arange(P))), shape=(D, P)).tocsr()

    active = np.ones(D, bool)
    level = np.zeros(D)
    lps = 0
    rounds = 0
    t0 = time.time()

    def solve_level(coef_t, lower):
        """max t s.t. S_c - coef_t[c] t >= lower[c], S_c <= D_c, loads <= C, x >= 0.
        Returns (t*, duals of the level rows)."""
        nonlocal lps
        level_rows = hstack([-sum_rows, csr_matrix(coef_t.reshape(-1, 1))])
        A = vstack([hstack([cap_rows, csr_matrix((E, 1))]), hstack([sum_rows, csr_matrix((D, 1))]),
                    level_rows]).tocsr()
        b = np.concatenate([C, Dm, -lower])
        c = np.zeros(P + 1)
        c[P] = -1.0
        res = linprog(c, A_ub=A, b_ub=b, bounds=(0, None), method="highs-ds")
        lps += 1
        if res.status != 0:
            raise RuntimeError(f"max-min LP failed: {res.message}")
        return float(res.x[P]), np.abs(res.ineqlin.marginals[E + D:])

    def frozen_lower():
        low = np.zeros(D)
        fz = ~active
        low[fz] = level[fz] * (1 - rel_tol)
        return low

    def theta(T):
        coef = np.where(active, np.minimum(T, Dm), 0.0)
        th, _ = solve_level(coef, frozen_lower())
        return th

    while active.any():
        act = np.nonzero(active)[0]
        order = act[np.argsort(Dm[act], kind="stable")]
        vals = Dm[order]
        ok = lambda j: theta(vals[j]) >= 1.0 - rel_tol  # noqa: E731
        good, step, bad = -1, 1, None
        while True:
            j = min(good + step, len(order) - 1)
            if j <= good:
                break
            if ok(j):
                good = j
                if j == len(order) - 1:
                    break
                step *= 2
            else:
                bad = j
                break
        if bad is not None:
            lo = good
            while bad - lo > 1:
                mid = (lo + bad) // 2
                if ok(mid):
                    lo = mid
                else:
                    bad = mid
            good = lo
        n_bulk = good + 1
        if n_bulk > 0:
            idx = order[:n_bulk]
            level[idx] = Dm[idx]
            active[idx] = False
        if not active.any():
            rounds += 1
            break
        coef = active.astype(np.float64)
        tstar, duals = solve_level(coef, frozen_lower())
        fz = active & ((duals > dual_tol) | (Dm <= tstar * (1 + rel_tol)))
        if not fz.any():
            raise RuntimeError("max-min LP: no commodity frozen (dual degeneracy)")
        idx = np.nonzero(fz)[0]
        level[idx] = np.minimum(tstar, Dm[idx])
        active[idx] = False
        rounds += 1
        if verbose:
            print(f"round {rounds}: demand-satisfied {n_bulk}, t*={tstar:.9g} froze {len(idx)}, "
                  f"active {int(active.sum())}, lps {lps} ({time.time() - t0:.1f}s)", flush=True)
    return level * scale, dict(rounds=rounds, lps=lps, seconds=time.time() - t0, scale=scale)
