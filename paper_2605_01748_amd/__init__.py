"""Python binding of the GATE TE solver library (libte_gate.so, C ABI in include/te.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.  PyTorch
provides device memory and the current HIP stream.  There is no CPU fallback: if the library is
missing, importing the solver raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libte_gate.so")

TE_OK, TE_ERR_INVALID, TE_ERR_OOM, TE_ERR_DEVICE, TE_ERR_NUMERIC, TE_ERR_STATE = range(6)
TE_CONVERGED, TE_HIT_MAX_ITERS, TE_HIT_ALPHA_MAX, TE_HIT_BETA_BOUND = 1, 2, 4, 8
ENGINE_AUTO, ENGINE_GRAPH, ENGINE_BLOCK = 0, 1, 2
LINK_SUMS_AUTO, LINK_SUMS_PRIVATE, LINK_SUMS_CSC, LINK_SUMS_PRIVATE_ATOMIC = 0, 1, 2, 3

API = ["te_default_options", "te_validate", "te_create", "te_update", "te_solve", "te_grad", "te_create_batch",
       "te_solve_batch", "te_kernel_times", "te_project", "te_project_rates", "te_project_rates_static", "te_get_state", "te_trace", "te_destroy", "te_destroy_batch",
       "te_info", "te_last_error"]


class TEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"te status {status}: {msg}")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("alpha_target", ctypes.c_double), ("gamma", ctypes.c_double), ("beta0", ctypes.c_double),
                ("A", ctypes.c_double), ("C", ctypes.c_double), ("beta_min", ctypes.c_double),
                ("beta_max", ctypes.c_double), ("max_iters", ctypes.c_int32), ("alpha_max", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("adapt_beta", ctypes.c_int32), ("beta_every", ctypes.c_int32),
                ("project", ctypes.c_int32), ("engine", ctypes.c_int32), ("record", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("paths_per_lane", ctypes.c_int32), ("warm", ctypes.c_int32), ("sched_beta", ctypes.c_void_p),
                ("sched_alpha", ctypes.c_void_p), ("sched_len", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("link_sums", ctypes.c_int32), ("per_link", ctypes.c_int32), ("w_min", ctypes.c_double),
                ("w_max", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("stop_iter", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("paths_per_lane", ctypes.c_int32), ("final_alpha", ctypes.c_double),
                ("beta", ctypes.c_double),
                ("r", ctypes.c_double), ("s", ctypes.c_double), ("max_cap_viol_rel", ctypes.c_double),
                ("max_dem_viol_rel", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def library(path: str = LIB_PATH):
    """Load libte_gate.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2605_01748_amd.build` "
                          f"(hipcc, gfx950); there is no fallback path")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int32
    lib.te_default_options.restype = None
    lib.te_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.te_validate.restype = I
    lib.te_validate.argtypes = [I, P, I, P, P, I, P, P]
    lib.te_create.restype = I
    lib.te_create.argtypes = [I, P, I, P, P, I, P, P, I, ctypes.POINTER(P)]
    lib.te_update.restype = I
    lib.te_update.argtypes = [P, P, P]
    lib.te_solve.restype = I
    lib.te_solve.argtypes = [P, ctypes.POINTER(_Options), P, P, P, P, ctypes.POINTER(_Stats)]
    lib.te_grad.restype = I
    lib.te_grad.argtypes = [P, P, P, P, P]
    lib.te_create_batch.restype = I
    lib.te_create_batch.argtypes = [I, ctypes.POINTER(P), ctypes.POINTER(P)]
    lib.te_solve_batch.restype = I
    lib.te_solve_batch.argtypes = [P, ctypes.POINTER(_Options), P, P, P, P]
    lib.te_project.restype = I
    lib.te_project.argtypes = [P, P, P, P]
    lib.te_project_rates.restype = I
    lib.te_project_rates.argtypes = [P, P, P, ctypes.c_double, P, P]
    lib.te_project_rates_static.restype = I
    lib.te_project_rates_static.argtypes = [P, P, P, ctypes.c_double, P, P]
    lib.te_get_state.restype = I
    lib.te_get_state.argtypes = [P, P, P, P, P]
    lib.te_trace.restype = I
    lib.te_trace.argtypes = [P, P, I, P, ctypes.POINTER(I)]
    lib.te_kernel_times.restype = I
    lib.te_kernel_times.argtypes = [P, ctypes.POINTER(_Options), P, I, P]
    lib.te_destroy.restype = None
    lib.te_destroy.argtypes = [P]
    lib.te_destroy_batch.restype = None
    lib.te_destroy_batch.argtypes = [P]
    lib.te_info.restype = I
    lib.te_info.argtypes = [P, P]
    lib.te_last_error.restype = ctypes.c_char_p
    lib.te_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status):
    if status != TE_OK:
        raise TEError(status, library().te_last_error().decode())


@dataclass
class Options:
    alpha_target: float = math.inf
    gamma: float = 1e-3
    beta0: float = 1.0
    A: float = 10.0
    C: float = 2.0
    beta_min: float | None = None      # default 1e-3 * beta0
    beta_max: float | None = None      # default 1e3 * beta0
    max_iters: int = 20000
    alpha_max: int = 64
    fixed_iters: int = 0
    adapt_beta: bool = True
    beta_every: int = 1
    project: bool = True
    engine: int = ENGINE_AUTO
    record: bool = False
    ckpt_every: int = 16
    block_threads: int = 0             # workgroup engine: 256, 512, 1024; 0 = tuned on the first solve
    paths_per_lane: int = 0            # 1, 2, 4, 8; 0 = graph engine default, workgroup engine tuned
    warm: bool = False                 # continue from the handle's last graph-engine state
    trace: bool = False                # log (beta_k, alpha_k, r_k, s_k) per iteration (Problem.trace)
    link_sums: int = LINK_SUMS_AUTO    # graph engine: privatised (LDS rows; link lists or atomic adds) or CSC sums
    per_link: bool = False             # per-link adaptive penalties beta * w_e (graph engine, CSC sums)
    w_min: float = 0.25
    w_max: float = 4.0
    sched_beta: np.ndarray | None = None
    sched_alpha: np.ndarray | None = None

    def to_c(self):
        o = _Options()
        library().te_default_options(ctypes.byref(o))
        o.alpha_target = self.alpha_target
        o.gamma = self.gamma
        o.beta0 = self.beta0
        o.A = self.A
        o.C = self.C
        o.beta_min = self.beta0 * 1e-3 if self.beta_min is None else self.beta_min
        o.beta_max = self.beta0 * 1e3 if self.beta_max is None else self.beta_max
        o.max_iters = self.max_iters
        o.alpha_max = self.alpha_max
        o.fixed_iters = self.fixed_iters
        o.adapt_beta = int(self.adapt_beta)
        o.beta_every = self.beta_every
        o.project = int(self.project)
        o.engine = self.engine
        o.record = int(self.record)
        o.ckpt_every = self.ckpt_every
        o.block_threads = self.block_threads
        o.paths_per_lane = self.paths_per_lane
        o.warm = int(self.warm)
        o.trace = int(self.trace)
        o.link_sums = int(self.link_sums)
        o.per_link = int(self.per_link)
        o.w_min = float(self.w_min)
        o.w_max = float(self.w_max)
        keep = []
        if self.sched_beta is not None:
            sb = np.ascontiguousarray(self.sched_beta, np.float64)
            sa = np.ascontiguousarray(self.sched_alpha, np.float64)
            assert sb.shape == sa.shape
            o.sched_beta = sb.ctypes.data
            o.sched_alpha = sa.ctypes.data
            o.sched_len = sb.shape[0]
            keep = [sb, sa]
        return o, keep


def _arrays(inst):
    cap = np.ascontiguousarray(inst.capacity, np.float64)
    pptr = np.ascontiguousarray(inst.path_ptr, np.int64)
    plinks = np.ascontiguousarray(inst.path_links, np.int32)
    dptr = np.ascontiguousarray(inst.demand_path_ptr, np.int32)
    dem = np.ascontiguousarray(inst.demand, np.float64)
    return cap, pptr, plinks, dptr, dem


def validate(inst):
    """Host-only admissibility check (te_validate); raises TEError on an invalid instance."""
    cap, pptr, plinks, dptr, dem = _arrays(inst)
    _check(library().te_validate(cap.shape[0], cap.ctypes.data, pptr.shape[0] - 1, pptr.ctypes.data,
                                 plinks.ctypes.data, dem.shape[0], dptr.ctypes.data, dem.ctypes.data))


def _stream_ptr(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


class Problem:
    """A TE instance resident on one GPU (te_create)."""

    def __init__(self, inst, device: int = 0):
        lib = library()
        cap, pptr, plinks, dptr, dem = _arrays(inst)
        h = ctypes.c_void_p()
        _check(lib.te_create(cap.shape[0], cap.ctypes.data, pptr.shape[0] - 1, pptr.ctypes.data, plinks.ctypes.data,
                             dem.shape[0], dptr.ctypes.data, dem.ctypes.data, device, ctypes.byref(h)))
        self._h = h
        self.device = device
        self.n_links, self.n_paths, self.n_demands = cap.shape[0], pptr.shape[0] - 1, dem.shape[0]

    def info(self):
        sz = np.zeros(14, np.int64)
        _check(library().te_info(self._h, sz.ctypes.data))
        return dict(n_links=int(sz[0]), n_paths=int(sz[1]), n_demands=int(sz[2]), nnz=int(sz[3]),
                    max_paths=int(sz[4]), auto_engine=int(sz[5]), demand_workgroups=int(sz[6]),
                    link_workgroups=int(sz[7]), hop_slots=int(sz[8]), record_gen=int(sz[9]),
                    link_sums=int(sz[10]), scatter_workgroups=int(sz[11]), list_passes=int(sz[12]),
                    list_entries=int(sz[13]))

    def update(self, capacity=None, demand=None):
        c = None if capacity is None else np.ascontiguousarray(capacity, np.float64)
        d = None if demand is None else np.ascontiguousarray(demand, np.float64)
        _check(library().te_update(self._h, None if c is None else c.ctypes.data, None if d is None else d.ctypes.data))

    def solve(self, opts: Options | None = None, x0=None, x_out=None, S_out=None, stats: bool = True, stream=None):
        """Returns (x [n_paths] float32 cuda tensor, S [n_demands], stats dict or None)."""
        import torch
        dev = torch.device("cuda", self.device)
        opts = opts or Options()
        o, keep = opts.to_c()
        if x_out is None:
            x_out = torch.empty(self.n_paths, dtype=torch.float32, device=dev)
        if S_out is None:
            S_out = torch.empty(self.n_demands, dtype=torch.float32, device=dev)
        x0p = None
        if x0 is not None:
            assert x0.dtype == torch.float32 and x0.is_cuda and x0.numel() == self.n_paths
            x0p = x0.data_ptr()
        st = _Stats() if stats else None
        sp = _stream_ptr(dev) if stream is None else stream
        _check(library().te_solve(self._h, ctypes.byref(o), sp, x0p, x_out.data_ptr(), S_out.data_ptr(),
                                  ctypes.byref(st) if st is not None else None))
        del keep
        return x_out, S_out, (st.as_dict() if st is not None else None)

    def grad(self, dS, stream=None):
        """Vector-Jacobian product through the last solve run with record=True (te_grad):
        returns (dC [n_links], dD [n_demands]) float64 cuda tensors for the cotangent dS on the
        unprojected per-demand sums."""
        import torch
        dev = torch.device("cuda", self.device)
        dS = dS.to(device=dev, dtype=torch.float32).contiguous()
        dC = torch.empty(self.n_links, dtype=torch.float64, device=dev)
        dD = torch.empty(self.n_demands, dtype=torch.float64, device=dev)
        sp = _stream_ptr(dev) if stream is None else stream
        _check(library().te_grad(self._h, sp, dS.data_ptr(), dC.data_ptr(), dD.data_ptr()))
        return dC, dD

    def trace(self, cap: int, stream=None):
        """Per-iteration trace of the last solve run with trace=True or record=True (te_trace):
        returns a float64 array [n, 4] of (beta_k, alpha_k, r_k, s_k)."""
        import torch
        out = np.zeros((4, max(int(cap), 0)), np.float64)
        n = ctypes.c_int32(0)
        sp = _stream_ptr(torch.device("cuda", self.device)) if stream is None else stream
        _check(library().te_trace(self._h, sp, int(cap), out.ctypes.data, ctypes.byref(n)))
        return out[:, :n.value].T.copy()

    def project(self, x_out=None, S_out=None, stream=None):
        """Feasible allocation (Algorithm 2) from the state the last graph-engine solve left (te_project):
        returns (x [n_paths], S [n_demands]) float32 cuda tensors in caller units."""
        import torch
        dev = torch.device("cuda", self.device)
        if x_out is None:
            x_out = torch.empty(self.n_paths, dtype=torch.float32, device=dev)
        if S_out is None:
            S_out = torch.empty(self.n_demands, dtype=torch.float32, device=dev)
        sp = _stream_ptr(dev) if stream is None else stream
        _check(library().te_project(self._h, sp, x_out.data_ptr(), S_out.data_ptr()))
        return x_out, S_out

    def state(self, stream=None, with_w=False):
        """The FP64 rates and per-demand sums the last graph-engine solve left, before projection
        (te_get_state): returns (x [n_paths], S [n_demands]) float64 cuda tensors in caller units, and
        with with_w=True also the per-link penalty factors w [n_links]."""
        import torch
        dev = torch.device("cuda", self.device)
        x = torch.empty(self.n_paths, dtype=torch.float64, device=dev)
        S = torch.empty(self.n_demands, dtype=torch.float64, device=dev)
        w = torch.empty(self.n_links, dtype=torch.float64, device=dev) if with_w else None
        sp = _stream_ptr(dev) if stream is None else stream
        _check(library().te_get_state(self._h, sp, x.data_ptr(), S.data_ptr(), None if w is None else w.data_ptr()))
        return (x, S, w) if with_w else (x, S)

    def project_rates(self, x, alpha, x_out=None, S_out=None, stream=None, static_scratch=False):
        """Algorithm 2 applied to the given path rates x (caller units) under the handle's current
        capacities and demands, with trim scores at `alpha` (te_project_rates, or with
        static_scratch=True te_project_rates_static, whose working arrays live in the library's
        static device array): returns (x [n_paths], S [n_demands]) float32 cuda tensors in caller
        units."""
        import torch
        dev = torch.device("cuda", self.device)
        x = torch.as_tensor(x).to(device=dev, dtype=torch.float32).contiguous()
        if x.numel() != self.n_paths:
            raise ValueError(f"x has {x.numel()} entries, the instance has {self.n_paths} paths")
        if x_out is None:
            x_out = torch.empty(self.n_paths, dtype=torch.float32, device=dev)
        if S_out is None:
            S_out = torch.empty(self.n_demands, dtype=torch.float32, device=dev)
        sp = _stream_ptr(dev) if stream is None else stream
        fn = library().te_project_rates_static if static_scratch else library().te_project_rates
        _check(fn(self._h, sp, x.data_ptr(), float(alpha), x_out.data_ptr(), S_out.data_ptr()))
        return x_out, S_out

    def kernel_times(self, opts: Options | None = None, iters: int = 64, stream=None):
        """Mean device time (ms) of the graph engine's demand and link kernels over `iters` iterations."""
        import torch
        opts = opts or Options()
        o, keep = opts.to_c()
        out = np.zeros(2)
        sp = _stream_ptr(torch.device("cuda", self.device)) if stream is None else stream
        _check(library().te_kernel_times(self._h, ctypes.byref(o), sp, iters, out.ctypes.data))
        del keep
        return float(out[0]), float(out[1])

    def close(self):
        if getattr(self, "_h", None):
            library().te_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many instances solved in one launch of the workgroup engine (te_create_batch)."""

    def __init__(self, problems):
        lib = library()
        arr = (ctypes.c_void_p * len(problems))(*[p._h for p in problems])
        h = ctypes.c_void_p()
        _check(lib.te_create_batch(len(problems), arr, ctypes.byref(h)))
        self._h = h
        self.problems = list(problems)
        self.device = problems[0].device
        self.n_paths = [p.n_paths for p in problems]
        self.n_demands = [p.n_demands for p in problems]

    def solve(self, opts: Options | None = None, stats: bool = True, x_out=None, S_out=None, stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        opts = opts or Options()
        o, keep = opts.to_c()
        if x_out is None:
            x_out = torch.empty(sum(self.n_paths), dtype=torch.float32, device=dev)
        if S_out is None:
            S_out = torch.empty(sum(self.n_demands), dtype=torch.float32, device=dev)
        st = (_Stats * len(self.problems))() if stats else None
        sp = _stream_ptr(dev) if stream is None else stream
        _check(library().te_solve_batch(self._h, ctypes.byref(o), sp, x_out.data_ptr(), S_out.data_ptr(),
                                        ctypes.cast(st, ctypes.c_void_p) if st is not None else None))
        del keep
        return x_out, S_out, ([s.as_dict() for s in st] if st is not None else None)

    def close(self):
        if getattr(self, "_h", None):
            library().te_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_GATE_SOLVE = None


def _autograd_function():
    global _GATE_SOLVE
    if _GATE_SOLVE is not None:
        return _GATE_SOLVE
    import torch

    class GateSolve(torch.autograd.Function):
        """S^(K) = unprojected per-demand sums after K iterations, as a differentiable function of
        the capacities C [n_links] and demands D [n_demands] (float64 CPU tensors, caller units).
        Forward: te_update + te_solve(record, fixed_iters=K); backward: te_grad (adjoint kernels,
        checkpoints every opts.ckpt_every iterations).  The (beta, alpha) schedule of the forward solve
        and the unit scale are held fixed in the derivative."""

        @staticmethod
        def forward(ctx, problem, C, D, K, opts=None):
            o = opts or Options()
            o = Options(**{**o.__dict__, "fixed_iters": int(K), "record": True, "project": False})
            problem.update(C.detach().cpu().numpy(), D.detach().cpu().numpy())
            _, S, _ = problem.solve(o, stats=False)
            ctx.problem = problem
            ctx.gen = problem.info()["record_gen"]
            return S.clone()

        @staticmethod
        def backward(ctx, gS):
            if ctx.problem.info()["record_gen"] != ctx.gen:
                raise RuntimeError("GateSolve: the problem was solved again (or updated) after this forward; "
                                   "its recording no longer describes this output")
            dC, dD = ctx.problem.grad(gS)
            return None, dC.cpu(), dD.cpu(), None, None

    _GATE_SOLVE = GateSolve
    return GateSolve


def __getattr__(name):
    if name == "GateSolve":
        return _autograd_function()
    raise AttributeError(name)
