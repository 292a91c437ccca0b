"""Optimality and drift-adjusted optimality (section 4.1) of an allocation.

Optimality of per-demand rates X against the optimal allocation OPT of the objective is the mean over
demands of min(X_d / max(OPT_d, theta), 1).  The drift-adjusted optimality DAO_K of a solver whose
runtime is K scores the rates it computed from the network state at T_0 under the state at T_0 + K:
the handle is updated to the later capacities and demands (``Problem.update``), Algorithm 2 applies
the earlier path rates to them on the GPU (``Problem.project_rates``: every path keeps at most its
T_0 rate, demands that shrank are trimmed, links whose capacity fell drop the excess), and the
resulting per-demand rates are scored against the optimum of the later state, which the caller
supplies (an exact max-min allocation, for instance).
"""
from __future__ import annotations

import numpy as np


def optimality(S, opt, theta: float) -> float:
    """Mean over demands of min(S_d / max(OPT_d, theta), 1)."""
    S = np.asarray(S, np.float64)
    opt = np.asarray(opt, np.float64)
    if S.shape != opt.shape:
        raise ValueError(f"{S.shape} rates against {opt.shape} optimal rates")
    if S.size == 0:
        raise ValueError("no demands")
    return float(np.mean(np.minimum(S / np.maximum(opt, theta), 1.0)))


def drift_adjusted_optimality(problem_K, x_T0, alpha: float, opt_K, theta: float, stream=None):
    """DAO of path rates x_T0 (computed for an earlier state, caller units, [n_paths]) under the
    state that `problem_K` holds now, with Algorithm 2's trim order at `alpha` (the final alpha of
    the solve that produced x_T0).  Returns (dao, x_applied, S_applied); the tensors stay on the GPU."""
    import torch
    x, S = problem_K.project_rates(x_T0, alpha, stream=stream)
    torch.cuda.synchronize(S.device)  # the work may be on a stream other than torch's current one
    return optimality(S.cpu().numpy(), opt_K, theta), x, S
