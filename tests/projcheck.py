"""Order-tolerant comparison of a GPU projection (Algorithm 2, section 3.5) with the oracle's.

The paper fixes no precision for the trim score S_c^alpha * C_p.  The oracle orders paths by the
score in FP64; the GPU by an FP32 log-score.  Where two paths on a violated link have FP64 scores
closer than FP32 resolves, the two sides may trim them in opposite order, and both orders are
valid readings of Algorithm 2.  Such a swap changes only the trims of the two paths involved on
that link (every other path on the link sees the same rate above it), so:

* every path whose order against its neighbours is decided on every violated link it uses must
  get the oracle's rate (to the rounding of the FP32 output);
* an ambiguous path must keep a rate between 0 and its rate after the demand phase;
* the output must be feasible (checked by the callers).
"""
import numpy as np

import oracle as O

SCORE_TOL = 4e-6  # relative resolution of the GPU's FP32 log-score, with margin


def ambiguous_paths(inst, xm, scores, alpha):
    """Boolean mask of paths whose link-phase order is not decided at FP32 resolution.
    xm: rates after the demand phase; scores: the oracle's FP64 log-scores of the link phase (at
    alpha = 0 they depend on the violated-link count alone).

    On each violated link the entries sorted by FP64 score fall into clusters: maximal runs in
    which each neighbour is within the FP32 resolution of the next.  Entries with the same score
    inputs (violated-link count and, for alpha > 0, demand sum) get equal scores on both sides and
    keep their path-index order; entries with different inputs may be reordered within their
    cluster, which can move one across a whole group of equal entries and change the rates above
    every member.  So every member of a cluster that holds more than one class of inputs is
    ambiguous."""
    P = inst.n_paths
    L = O.link_loads(inst, xm)
    viol = L > inst.capacity
    path_of_inc = np.repeat(np.arange(P), np.diff(inst.path_ptr))
    links = np.asarray(inst.path_links)
    on = viol[links]
    pi, li = path_of_inc[on], links[on]
    sc = scores[pi]
    # the exact inputs of a score: the demand sum and the violated-link count
    dem_of = np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))
    S = O.demand_sums(inst, xm)
    cp = np.bincount(path_of_inc[on], minlength=P)
    order = np.lexsort((sc, li))
    pi, li, sc = pi[order], li[order], sc[order]
    amb = np.zeros(P, bool)
    if pi.size < 2:
        return amb
    same = li[1:] == li[:-1]
    fin = np.isfinite(sc[1:]) & np.isfinite(sc[:-1])
    with np.errstate(invalid="ignore"):
        close = np.abs(sc[1:] - sc[:-1]) <= SCORE_TOL * np.maximum(1.0, np.maximum(np.abs(sc[1:]), np.abs(sc[:-1])))
    link_ = same & fin & close
    cluster = np.concatenate([[0], np.cumsum(~link_)])  # entries i, i + 1 share a cluster iff link_[i]
    # class of an entry's score inputs
    cls_S = S[dem_of[pi]] if alpha != 0.0 else np.zeros(pi.size)
    _, cls = np.unique(np.stack([cp[pi].astype(np.float64), cls_S]), axis=1, return_inverse=True)
    cls = np.asarray(cls).ravel()
    # clusters holding more than one class
    pairs = np.unique(np.stack([cluster, cls]), axis=1)
    n_cls = np.bincount(pairs[0], minlength=cluster.max() + 1)
    amb[pi[n_cls[cluster] > 1]] = True
    return amb


def check_projection(inst, x_in, x_gpu, alpha, tag="", rtol=2e-6, per_demand=False):
    """Compare the GPU's projection x_gpu of rates x_in (caller units) with the oracle's Algorithm 2.
    per_demand: compare per-demand sums (large instances) instead of every path."""
    ref, xm, sc = O.project(inst, np.asarray(x_in, np.float64), alpha, stages=True)
    amb = ambiguous_paths(inst, xm, sc, alpha)
    x_gpu = np.asarray(x_gpu, np.float64)
    atol = 1e-6 * inst.capacity.max()
    assert np.all(x_gpu[amb] >= 0)
    assert np.all(x_gpu[amb] <= xm[amb] * (1 + rtol) + atol)
    if per_demand:
        dem_of = np.repeat(np.arange(inst.n_demands), np.diff(inst.demand_path_ptr))
        amb_dem = np.zeros(inst.n_demands, bool)
        amb_dem[dem_of[amb]] = True
        Sg, Sr = O.demand_sums(inst, x_gpu), O.demand_sums(inst, ref)
        d = np.abs(Sg - Sr)[~amb_dem]
        print(f"{tag} projection: {amb.sum()} of {inst.n_paths} paths in near-ties ({amb_dem.sum()} demands); "
              f"max |dS| elsewhere {d.max() if d.size else 0:.3e}")
        np.testing.assert_allclose(Sg[~amb_dem], Sr[~amb_dem], rtol=10 * rtol, atol=atol)
    else:
        d = np.abs(x_gpu - ref)[~amb]
        print(f"{tag} projection: {amb.sum()} of {inst.n_paths} paths in near-ties; "
              f"max |dx| elsewhere {d.max() if d.size else 0:.3e}")
        np.testing.assert_allclose(x_gpu[~amb], ref[~amb], rtol=rtol, atol=atol)
    return amb
