"""FP64 CPU oracle of GATE's decomposition, and exact checkers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the GPU product path.  It shares no
code with the HIP library.

* ``solve``      -- the iteration of section 3 (Algorithm 1) in FP64, C library
                    ``libgate_oracle.so`` built from ``gate_oracle.c``.
* ``sum_root``   -- one commodity's sum equation (appendix B.2).
* ``project``    -- Algorithm 2 (section 3.5).
* ``grad``       -- FP64 reverse pass (vector-Jacobian product) through K sweeps.
* ``maxmin``     -- exact max-min fair allocation by progressive filling of LPs
                    (``maxmin.py``).
* ``optimality`` -- the paper's optimality metric (section 4.1).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgate_oracle.so")
_lib = None

CONVERGED, HIT_MAX_ITERS, HIT_ALPHA_MAX, HIT_BETA_BOUND, NUMERIC = 1, 2, 4, 8, 16


def build(openmp: bool = True) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-Wextra",
           os.path.join(_HERE, "gate_oracle.c"), "-o", _LIB_PATH, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.check_call(cmd)
    return _LIB_PATH


class _Options(ctypes.Structure):
    _fields_ = [("alpha_target", ctypes.c_double), ("gamma", ctypes.c_double), ("beta0", ctypes.c_double),
                ("A", ctypes.c_double), ("C", ctypes.c_double), ("beta_min", ctypes.c_double),
                ("beta_max", ctypes.c_double), ("max_iters", ctypes.c_int32), ("alpha_max", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("adapt_beta", ctypes.c_int32), ("project", ctypes.c_int32),
                ("collapsed", ctypes.c_int32), ("sched_beta", ctypes.c_void_p), ("sched_alpha", ctypes.c_void_p),
                ("sched_len", ctypes.c_int32), ("root_max_steps", ctypes.c_int32),
                ("dual_res_scaled", ctypes.c_int32), ("beta_every", ctypes.c_int32), ("warm", ctypes.c_void_p),
                ("per_link", ctypes.c_int32), ("w_min", ctypes.c_double), ("w_max", ctypes.c_double)]


class _Warm(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("S", ctypes.c_void_p), ("y", ctypes.c_void_p), ("ucon", ctypes.c_void_p),
                ("ucap", ctypes.c_void_p), ("udem", ctypes.c_void_p), ("uneg", ctypes.c_void_p),
                ("beta", ctypes.c_double), ("alpha", ctypes.c_double), ("w", ctypes.c_void_p),
                ("last_dir", ctypes.c_int32), ("n_rev", ctypes.c_int32), ("rule_rest", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("stop_iter", ctypes.c_int32),
                ("final_alpha", ctypes.c_double), ("beta", ctypes.c_double), ("r", ctypes.c_double),
                ("s", ctypes.c_double), ("max_cap_viol_rel", ctypes.c_double),
                ("max_dem_viol_rel", ctypes.c_double), ("collapse_dev", ctypes.c_double),
                ("root_steps_mean", ctypes.c_double), ("root_steps_max", ctypes.c_int32),
                ("last_dir", ctypes.c_int32), ("n_rev", ctypes.c_int32), ("rule_rest", ctypes.c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("dual_dem", ctypes.c_void_p), ("dual_cap", ctypes.c_void_p), ("dual_neg", ctypes.c_void_p),
                ("dual_con", ctypes.c_void_p), ("y", ctypes.c_void_p), ("x_raw", ctypes.c_void_p),
                ("S_raw", ctypes.c_void_p), ("trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int32),
                ("scale", ctypes.c_double), ("w", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gate_oracle_solve.restype = ctypes.c_int
        lib.gate_oracle_solve.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, P, P,
                                          ctypes.POINTER(_Options), P, P, P, ctypes.POINTER(_State),
                                          ctypes.POINTER(_Stats)]
        lib.gate_oracle_sum_root.restype = ctypes.c_int
        lib.gate_oracle_sum_root.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P]
        lib.gate_oracle_grad.restype = ctypes.c_int
        lib.gate_oracle_grad.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, P, P, ctypes.c_double,
                                         ctypes.c_int, P, P, P, P, P, P]
        lib.gate_oracle_threads.restype = ctypes.c_int
        lib.gate_oracle_threads.argtypes = [ctypes.c_int]
        lib.gate_oracle_project.restype = ctypes.c_int
        lib.gate_oracle_project.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, P, P,
                                            ctypes.c_double, P, P, P]
        _lib = lib
    return _lib


@dataclass
class Options:
    alpha_target: float = math.inf
    gamma: float = 1e-3
    beta0: float = 1.0
    A: float = 10.0
    C: float = 2.0
    beta_min_rel: float = 1e-3
    beta_max_rel: float = 1e3
    max_iters: int = 20000
    alpha_max: int = 64
    fixed_iters: int = 0
    adapt_beta: bool = True
    project: bool = True
    collapsed: bool = False
    sched_beta: np.ndarray | None = None
    sched_alpha: np.ndarray | None = None
    root_max_steps: int = 200
    dual_res_scaled: bool = False
    beta_every: int = 1
    per_link: bool = False   # per-link penalties beta * w_e, w_e adapted per link
    w_min: float = 0.25      # bounds on w_e (wider bounds let the rule starve a link's penalty: with
    w_max: float = 4.0       # [1e-2, 1e2] a 7-node instance stalled at alpha = 0)


@dataclass
class Result:
    x: np.ndarray            # projected (if requested) path rates, original units
    S: np.ndarray            # per-demand sums of x
    x_raw: np.ndarray        # unprojected rates, normalised units
    S_raw: np.ndarray        # unprojected sums, normalised units
    scale: float
    iters: int
    flags: int
    stop_iter: int
    final_alpha: float
    beta: float
    r: float
    s: float
    max_cap_viol_rel: float
    max_dem_viol_rel: float
    collapse_dev: float
    root_steps_mean: float
    root_steps_max: int
    trace: np.ndarray        # [iters, 5]: alpha, beta, r, s, flags
    dual_dem: np.ndarray
    dual_cap: np.ndarray
    dual_neg: np.ndarray
    dual_con: np.ndarray
    y: np.ndarray
    w: np.ndarray            # [E] per-link penalty factors at the end (ones without per_link)
    backoff: tuple = (0, 0, 0)  # balancing rule: last direction, reversals, sweeps still at rest

    @property
    def schedule(self):
        return self.trace[:, 1].copy(), self.trace[:, 0].copy()

    def warm_state(self):
        """The iterate this solve left (unprojected rates, last sums, rate suggestions, every scaled
        dual, the penalty and alpha), in caller units: the `warm` input of a later solve."""
        if self.dual_dem is None:
            raise ValueError("solve(..., want_state=True) keeps the duals")
        s = self.scale
        return dict(x=self.x_raw * s, S=self.S_raw * s, y=self.y * s, ucon=self.dual_con * s,
                    ucap=self.dual_cap * s, udem=self.dual_dem * s, uneg=self.dual_neg * s,
                    beta=self.beta, alpha=self.final_alpha, w=self.w.copy(), backoff=self.backoff)


def _p(a):
    return None if a is None else a.ctypes.data


def solve(inst, opts: Options | None = None, x0=None, want_state: bool = True, warm=None) -> Result:
    """Run the oracle on a workloads.Instance.  warm: a state from Result.warm_state() (caller units)
    to continue from instead of initialising (x0 is then ignored)."""
    opts = opts or Options()
    lib = _load()
    E, P, D, nnz = inst.n_links, inst.n_paths, inst.n_demands, inst.nnz
    cap = np.ascontiguousarray(inst.capacity, np.float64)
    pptr = np.ascontiguousarray(inst.path_ptr, np.int64)
    plinks = np.ascontiguousarray(inst.path_links, np.int32)
    dptr = np.ascontiguousarray(inst.demand_path_ptr, np.int32)
    dem = np.ascontiguousarray(inst.demand, np.float64)
    o = _Options()
    o.alpha_target = opts.alpha_target
    o.gamma = opts.gamma
    o.beta0 = opts.beta0
    o.A = opts.A
    o.C = opts.C
    o.beta_min = opts.beta0 * opts.beta_min_rel
    o.beta_max = opts.beta0 * opts.beta_max_rel
    o.max_iters = opts.max_iters
    o.alpha_max = opts.alpha_max
    o.fixed_iters = opts.fixed_iters
    o.adapt_beta = int(opts.adapt_beta)
    o.project = int(opts.project)
    o.collapsed = int(opts.collapsed)
    o.root_max_steps = opts.root_max_steps
    o.dual_res_scaled = int(opts.dual_res_scaled)
    o.beta_every = int(opts.beta_every)
    o.per_link = int(opts.per_link)
    o.w_min = float(opts.w_min)
    o.w_max = float(opts.w_max)
    sb = sa = None
    if opts.sched_beta is not None:
        sb = np.ascontiguousarray(opts.sched_beta, np.float64)
        sa = np.ascontiguousarray(opts.sched_alpha, np.float64)
        o.sched_beta = sb.ctypes.data
        o.sched_alpha = sa.ctypes.data
        o.sched_len = sb.shape[0]
    n_iter_cap = opts.fixed_iters if opts.fixed_iters > 0 else opts.max_iters
    x_out = np.zeros(P)
    S_out = np.zeros(D)
    x_raw = np.zeros(P)
    S_raw = np.zeros(D)
    trace = np.zeros((max(n_iter_cap, 1), 5))
    st = _State()
    st.x_raw = x_raw.ctypes.data
    st.S_raw = S_raw.ctypes.data
    st.trace = trace.ctypes.data
    st.trace_cap = trace.shape[0]
    w_out = np.ones(E)
    st.w = w_out.ctypes.data
    dd = dc = dn = dcon = yy = None
    if want_state:
        dd, dc, dn, dcon, yy = np.zeros(D), np.zeros(E), np.zeros(P), np.zeros(max(nnz, 1)), np.zeros(max(nnz, 1))
        st.dual_dem, st.dual_cap, st.dual_neg, st.dual_con, st.y = (dd.ctypes.data, dc.ctypes.data, dn.ctypes.data,
                                                                    dcon.ctypes.data, yy.ctypes.data)
    x0a = None if x0 is None else np.ascontiguousarray(x0, np.float64)
    wkeep = []
    if warm is not None:
        w = _Warm()
        for name, n in (("x", P), ("S", D), ("y", nnz), ("ucon", nnz), ("ucap", E), ("udem", D), ("uneg", P)):
            a = np.ascontiguousarray(warm[name], np.float64)
            if a.shape != (n,):
                raise ValueError(f"warm[{name!r}] has shape {a.shape}, expected ({n},)")
            wkeep.append(a)
            setattr(w, name, a.ctypes.data)
        w.beta = float(warm["beta"])
        w.alpha = float(warm["alpha"])
        w.last_dir, w.n_rev, w.rule_rest = (int(v) for v in warm.get("backoff", (0, 0, 0)))
        if warm.get("w") is not None:
            wa = np.ascontiguousarray(warm["w"], np.float64)
            if wa.shape != (E,):
                raise ValueError(f"warm['w'] has shape {wa.shape}, expected ({E},)")
            wkeep.append(wa)
            w.w = wa.ctypes.data
        wkeep.append(w)
        o.warm = ctypes.addressof(w)
    stats = _Stats()
    rc = lib.gate_oracle_solve(E, cap.ctypes.data, P, pptr.ctypes.data, plinks.ctypes.data, D, dptr.ctypes.data,
                               dem.ctypes.data, ctypes.byref(o), _p(x0a), x_out.ctypes.data, S_out.ctypes.data,
                               ctypes.byref(st), ctypes.byref(stats))
    if rc != 0:
        raise RuntimeError(f"oracle solve failed rc={rc}")
    it = stats.iters
    return Result(x=x_out, S=S_out, x_raw=x_raw, S_raw=S_raw, scale=st.scale, iters=it, flags=stats.flags,
                  stop_iter=stats.stop_iter, final_alpha=stats.final_alpha, beta=stats.beta, r=stats.r, s=stats.s,
                  max_cap_viol_rel=stats.max_cap_viol_rel, max_dem_viol_rel=stats.max_dem_viol_rel,
                  collapse_dev=stats.collapse_dev, root_steps_mean=stats.root_steps_mean,
                  root_steps_max=stats.root_steps_max, trace=trace[:it].copy(), dual_dem=dd, dual_cap=dc,
                  dual_neg=dn, dual_con=None if dcon is None else dcon[:nnz], y=None if yy is None else yy[:nnz],
                  w=w_out, backoff=(stats.last_dir, stats.n_rev, stats.rule_rest))


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP threads for later calls (n > 0); returns the threads in use."""
    return int(_load().gate_oracle_threads(int(n)))


def sum_root(a, n_links, uneg, D, udem, alpha, beta, S0):
    """Root S of one commodity's sum equation and the rates x_r (appendix B.2).  n_links: links per
    path, or with per-link penalties the weights W_r = sum of the factors w_e of the path's links."""
    lib = _load()
    a = np.ascontiguousarray(a, np.float64)
    n = np.ascontiguousarray(n_links, np.float64)
    u = np.ascontiguousarray(uneg, np.float64)
    x = np.zeros(a.shape[0])
    S = ctypes.c_double(0.0)
    steps = lib.gate_oracle_sum_root(a.shape[0], a.ctypes.data, n.ctypes.data, u.ctypes.data, float(D), float(udem),
                                     float(alpha), float(beta), float(S0), ctypes.addressof(S), x.ctypes.data)
    return S.value, x, steps


def project(inst, x, alpha, stages: bool = False):
    """Algorithm 2 on rates x (original units); returns the projected copy, or with stages=True
    (projected, rates after the demand trims, log-scores of the link phase)."""
    lib = _load()
    xx = np.array(x, dtype=np.float64, copy=True)
    xm = np.zeros_like(xx) if stages else None
    sc = np.zeros_like(xx) if stages else None
    cap = np.ascontiguousarray(inst.capacity, np.float64)
    pptr = np.ascontiguousarray(inst.path_ptr, np.int64)
    plinks = np.ascontiguousarray(inst.path_links, np.int32)
    dptr = np.ascontiguousarray(inst.demand_path_ptr, np.int32)
    dem = np.ascontiguousarray(inst.demand, np.float64)
    lib.gate_oracle_project(inst.n_links, cap.ctypes.data, inst.n_paths, pptr.ctypes.data, plinks.ctypes.data,
                            inst.n_demands, dptr.ctypes.data, dem.ctypes.data, float(alpha), xx.ctypes.data,
                            _p(xm), _p(sc))
    return (xx, xm, sc) if stages else xx


def used_scale(inst):
    """The unit scale s: the largest capacity of a link used by some path."""
    return float(inst.capacity[np.unique(inst.path_links)].max())


def grad(inst, sched_beta, sched_alpha, dS, scale=None, capacity=None, demand=None):
    """FP64 reverse pass: S^(K) (unprojected, caller units) and the vector-Jacobian products
    dC = dS . dS^(K)/dC, dD = dS . dS^(K)/dD for K = len(sched_beta) sweeps with the schedule and
    the unit scale held fixed.  capacity / demand override the instance's values (for finite
    differences at a frozen scale)."""
    lib = _load()
    sb = np.ascontiguousarray(sched_beta, np.float64)
    sa = np.ascontiguousarray(sched_alpha, np.float64)
    cap = np.ascontiguousarray(inst.capacity if capacity is None else capacity, np.float64)
    dem = np.ascontiguousarray(inst.demand if demand is None else demand, np.float64)
    pptr = np.ascontiguousarray(inst.path_ptr, np.int64)
    plinks = np.ascontiguousarray(inst.path_links, np.int32)
    dptr = np.ascontiguousarray(inst.demand_path_ptr, np.int32)
    w = np.ascontiguousarray(dS, np.float64)
    S = np.zeros(inst.n_demands)
    dC = np.zeros(inst.n_links)
    dD = np.zeros(inst.n_demands)
    s = used_scale(inst) if scale is None else float(scale)
    rc = lib.gate_oracle_grad(inst.n_links, cap.ctypes.data, inst.n_paths, pptr.ctypes.data, plinks.ctypes.data,
                              inst.n_demands, dptr.ctypes.data, dem.ctypes.data, s, sb.shape[0], sb.ctypes.data,
                              sa.ctypes.data, w.ctypes.data, S.ctypes.data, dC.ctypes.data, dD.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle grad failed")
    return S, dC, dD


def demand_sums(inst, x):
    return np.add.reduceat(np.asarray(x, np.float64), inst.demand_path_ptr[:-1]) if inst.n_paths else np.zeros(0)


def link_loads(inst, x):
    path_of_inc = np.repeat(np.arange(inst.n_paths), np.diff(inst.path_ptr))
    return np.bincount(inst.path_links, weights=np.asarray(x, np.float64)[path_of_inc], minlength=inst.n_links)


def optimality(S, opt, theta):
    """Section 4.1: mean over demands of min(X_d / max(OPT_d, theta), 1)."""
    S = np.asarray(S, np.float64)
    opt = np.asarray(opt, np.float64)
    return float(np.mean(np.minimum(S / np.maximum(opt, theta), 1.0)))


from .maxmin import maxmin_exact  # noqa: E402,F401
