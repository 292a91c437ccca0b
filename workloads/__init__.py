"""Seeded synthetic traffic-engineering inputs.

This module builds the inputs of the TE problem of the paper (section "TE
Formulation"): a capacitated directed link set, a demand per ordered node pair
and, per demand, a set of precomputed paths.  It stands in for the paper's
topologies and traces (its "Experiment Setup" section: public topologies with
gravity-model demands, production WANs, k-shortest paths with k=4), none of
which is available here.  It holds none of the solver's arithmetic and is the
only code shared by the oracle-side tests and the GPU-side tests.

Recipes (all seeded through ``numpy.random.SeedSequence``):

* Waxman topology: nodes uniform in the unit square, an undirected edge (u, v)
  with probability beta_w * exp(-d(u, v) / (alpha_w * L)), L the largest
  pairwise distance.  beta_w is calibrated per draw so that the expected edge
  count equals the requested link count; draws are repeated until the graph is
  connected and the edge count is within 10% of the target.  Each undirected
  link becomes two arcs with the same capacity.
* Gravity demands: D_st proportional to w_s * w_t for all ordered pairs with at
  least one path, node weights w lognormal (or 1 + Pareto for the hierarchical
  graph).
* Paths: the first k simple paths in (cost, node sequence) order, cost = hop
  count or Euclidean length (Yen's algorithm, ``ksp.c``).
* Drift (``drift_path``): demands follow mean-preserving geometric Brownian motions calibrated to
  a 35 % mean absolute change per five minutes; link capacities change at Poisson times (200 per
  day over the network), each to U(0.25, 1) of its initial value.
* Scale: D = factor * lambda_star * D_gravity, where lambda_star is the largest
  lambda for which lambda * D_gravity is routable on the given paths (max
  concurrent flow, one LP).  The tightest path-restricted cut is then
  ``factor`` times oversubscribed.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LAMBDA_CACHE = os.path.join(_HERE, "lambda_star.json")


@dataclass
class Instance:
    """One TE instance in the layout the C ABI takes.

    link i is the arc link_src[i] -> link_dst[i] with capacity[i];
    paths of demand c are path ids demand_path_ptr[c] .. demand_path_ptr[c+1]-1;
    path r uses links path_links[path_ptr[r] : path_ptr[r+1]] in path order.
    """
    name: str
    n_nodes: int
    link_src: np.ndarray
    link_dst: np.ndarray
    capacity: np.ndarray
    demand_src: np.ndarray
    demand_dst: np.ndarray
    demand: np.ndarray
    path_ptr: np.ndarray
    path_links: np.ndarray
    demand_path_ptr: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_links(self) -> int:
        return int(self.capacity.shape[0])

    @property
    def n_demands(self) -> int:
        return int(self.demand.shape[0])

    @property
    def n_paths(self) -> int:
        return int(self.path_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.path_links.shape[0])

    def fingerprint(self) -> str:
        h = hashlib.sha256()
        for a in (self.link_src, self.link_dst, self.capacity, self.demand, self.path_ptr,
                  self.path_links, self.demand_path_ptr):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]

    def summary(self) -> str:
        return (f"{self.name}: nodes={self.n_nodes} links={self.n_links} demands={self.n_demands} "
                f"paths={self.n_paths} nnz={self.nnz}")


def make_instance(name, n_nodes, link_src, link_dst, capacity, demand_src, demand_dst, demand,
                  paths, meta=None) -> Instance:
    """paths: list (one entry per demand) of lists of link-id lists."""
    pp = [0]
    dp = [0]
    links = []
    for plist in paths:
        for p in plist:
            links.extend(int(e) for e in p)
            pp.append(len(links))
        dp.append(len(pp) - 1)
    return Instance(
        name=name, n_nodes=int(n_nodes),
        link_src=np.asarray(link_src, dtype=np.int32), link_dst=np.asarray(link_dst, dtype=np.int32),
        capacity=np.asarray(capacity, dtype=np.float64),
        demand_src=np.asarray(demand_src, dtype=np.int32), demand_dst=np.asarray(demand_dst, dtype=np.int32),
        demand=np.asarray(demand, dtype=np.float64),
        path_ptr=np.asarray(pp, dtype=np.int64), path_links=np.asarray(links, dtype=np.int32),
        demand_path_ptr=np.asarray(dp, dtype=np.int32), meta=dict(meta or {}))


# ----------------------------------------------------------------------------------------------
# k shortest paths (C helper)
# ----------------------------------------------------------------------------------------------
_ksp_lib = None


def _ksp():
    global _ksp_lib
    if _ksp_lib is None:
        path = os.path.join(_HERE, "libksp.so")
        if not os.path.exists(path):
            build_ksp()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.ksp_batch.restype = ctypes.c_int
        lib.ksp_batch.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int, P, P, P,
                                  ctypes.c_int, P, P, P]
        _ksp_lib = lib
    return _ksp_lib


def build_ksp() -> str:
    import subprocess
    out = os.path.join(_HERE, "libksp.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", os.path.join(_HERE, "ksp.c"),
                           "-o", out])
    return out


def k_shortest_paths_csr(n_nodes, arc_src, arc_dst, weight, pair_src, pair_dst, k, chunk=8192, progress=None):
    """Vectorised variant for large pair sets: returns (paths per pair [npairs], path_ptr [P+1] int64,
    path_links [nnz] int32), paths of a pair contiguous and in (cost, sequence) order.  progress, if
    given, is called with (pairs done, pairs total) after every chunk."""
    arc_src = np.ascontiguousarray(arc_src, dtype=np.int32)
    arc_dst = np.ascontiguousarray(arc_dst, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    m = arc_src.shape[0]
    n = int(n_nodes)
    out_arc = np.ascontiguousarray(np.lexsort((arc_dst, arc_src)), dtype=np.int32)
    out_ptr = np.cumsum(np.concatenate([[0], np.bincount(arc_src, minlength=n)])).astype(np.int32)
    in_arc = np.ascontiguousarray(np.lexsort((arc_src, arc_dst)), dtype=np.int32)
    in_ptr = np.cumsum(np.concatenate([[0], np.bincount(arc_dst, minlength=n)])).astype(np.int32)
    pair_src = np.ascontiguousarray(pair_src, dtype=np.int32)
    pair_dst = np.ascontiguousarray(pair_dst, dtype=np.int32)
    lib = _ksp()
    hop_cap = max(n - 1, 1)
    counts, hops_all, links_all = [], [], []
    for s0 in range(0, pair_src.shape[0], chunk):
        s1 = min(s0 + chunk, pair_src.shape[0])
        q = s1 - s0
        npaths = np.zeros(q, dtype=np.int32)
        hops = np.zeros(q * k, dtype=np.int32)
        arcs = np.zeros(q * k * hop_cap, dtype=np.int32)
        kp = np.full(q, k, dtype=np.int32)
        err = lib.ksp_batch(n, m, arc_src.ctypes.data, arc_dst.ctypes.data, weight.ctypes.data,
                            out_ptr.ctypes.data, out_arc.ctypes.data, in_ptr.ctypes.data, in_arc.ctypes.data,
                            q, np.ascontiguousarray(pair_src[s0:s1]).ctypes.data,
                            np.ascontiguousarray(pair_dst[s0:s1]).ctypes.data, kp.ctypes.data, k,
                            npaths.ctypes.data, hops.ctypes.data, arcs.ctypes.data)
        if err:
            raise RuntimeError("ksp_batch failed")
        valid = (np.arange(k)[None, :] < npaths[:, None]).ravel()
        h = hops[valid]
        slot = np.nonzero(valid)[0]
        # gather the hop lists of the valid slots
        starts = slot * hop_cap
        idx = np.repeat(starts - np.concatenate([[0], np.cumsum(h)[:-1]]), h) + np.arange(h.sum())
        counts.append(npaths)
        hops_all.append(h)
        links_all.append(arcs[idx])
        if progress is not None:
            progress(s1, pair_src.shape[0])
    counts = np.concatenate(counts)
    hops = np.concatenate(hops_all)
    path_ptr = np.concatenate([[0], np.cumsum(hops)]).astype(np.int64)
    return counts, path_ptr, np.concatenate(links_all).astype(np.int32)


def k_shortest_paths(n_nodes, arc_src, arc_dst, weight, pair_src, pair_dst, k_per, chunk=8192):
    """Returns, per pair, a list of paths, each a list of arc ids (first k in (cost, sequence) order)."""
    arc_src = np.ascontiguousarray(arc_src, dtype=np.int32)
    arc_dst = np.ascontiguousarray(arc_dst, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    m = arc_src.shape[0]
    n = int(n_nodes)
    order = np.lexsort((arc_dst, arc_src))
    out_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(out_ptr, arc_src + 1, 1)
    out_ptr = np.cumsum(out_ptr).astype(np.int32)
    out_arc = np.ascontiguousarray(order, dtype=np.int32)
    order_in = np.lexsort((arc_src, arc_dst))
    in_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(in_ptr, arc_dst + 1, 1)
    in_ptr = np.cumsum(in_ptr).astype(np.int32)
    in_arc = np.ascontiguousarray(order_in, dtype=np.int32)
    pair_src = np.ascontiguousarray(pair_src, dtype=np.int32)
    pair_dst = np.ascontiguousarray(pair_dst, dtype=np.int32)
    k_per = np.ascontiguousarray(np.broadcast_to(np.asarray(k_per, dtype=np.int32), pair_src.shape))
    kmax = int(k_per.max()) if k_per.size else 1
    lib = _ksp()
    res = []
    hop_cap = max(n - 1, 1)
    for s0 in range(0, pair_src.shape[0], chunk):
        s1 = min(s0 + chunk, pair_src.shape[0])
        q = s1 - s0
        npaths = np.zeros(q, dtype=np.int32)
        hops = np.zeros(q * kmax, dtype=np.int32)
        arcs = np.zeros(q * kmax * hop_cap, dtype=np.int32)
        ps = np.ascontiguousarray(pair_src[s0:s1])
        pt = np.ascontiguousarray(pair_dst[s0:s1])
        kp = np.ascontiguousarray(k_per[s0:s1])
        err = lib.ksp_batch(n, m, arc_src.ctypes.data, arc_dst.ctypes.data, weight.ctypes.data,
                            out_ptr.ctypes.data, out_arc.ctypes.data, in_ptr.ctypes.data, in_arc.ctypes.data,
                            q, ps.ctypes.data, pt.ctypes.data, kp.ctypes.data, kmax,
                            npaths.ctypes.data, hops.ctypes.data, arcs.ctypes.data)
        if err:
            raise RuntimeError("ksp_batch failed")
        for i in range(q):
            plist = []
            for j in range(npaths[i]):
                h = hops[i * kmax + j]
                base = (i * kmax + j) * hop_cap
                plist.append(arcs[base:base + h].tolist())
            res.append(plist)
    return res


# ----------------------------------------------------------------------------------------------
# topology and demand recipes
# ----------------------------------------------------------------------------------------------
def _connected(n, edges) -> bool:
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    seen = {0}
    stack = [0]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return len(seen) == n


def waxman(n, target_links, rng, alpha_w=0.4, tol=0.1, max_tries=1000, box=(0.0, 0.0, 1.0, 1.0)):
    """Undirected Waxman graph; returns (positions [n,2], edge list [(u, v) with u < v])."""
    for _ in range(max_tries):
        x0, y0, x1, y1 = box
        pos = np.column_stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)])
        iu, iv = np.triu_indices(n, 1)
        d = np.hypot(*(pos[iu] - pos[iv]).T)
        L = d.max()
        base = np.exp(-d / (alpha_w * L))
        beta_w = min(1.0, target_links / base.sum())
        keep = rng.uniform(size=base.shape) < beta_w * base
        edges = list(zip(iu[keep].tolist(), iv[keep].tolist()))
        if abs(len(edges) - target_links) <= tol * target_links and _connected(n, edges):
            return pos, edges
    raise RuntimeError("could not draw a connected Waxman graph")


def arcs_from_edges(edges, edge_cap, pos=None):
    """Each undirected edge (u, v) -> arcs u->v and v->u, same capacity; arc weights = Euclidean length."""
    src, dst, cap, w = [], [], [], []
    for (u, v), c in zip(edges, edge_cap):
        for a, b in ((u, v), (v, u)):
            src.append(a)
            dst.append(b)
            cap.append(float(c))
            w.append(float(np.hypot(*(pos[a] - pos[b]))) if pos is not None else 1.0)
    return (np.asarray(src, np.int32), np.asarray(dst, np.int32), np.asarray(cap, np.float64),
            np.asarray(w, np.float64))


def gravity(weights, pair_src, pair_dst):
    g = weights[pair_src] * weights[pair_dst]
    return g / g.sum()


def max_concurrent_flow(inst: Instance, base_demand: np.ndarray) -> float:
    """lambda_star = max lambda such that lambda * base_demand is routable on the instance's paths."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix
    P, D, E = inst.n_paths, inst.n_demands, inst.n_links
    path_of_inc = np.repeat(np.arange(P), np.diff(inst.path_ptr))
    dem_of_path = np.repeat(np.arange(D), np.diff(inst.demand_path_ptr))
    # rows 0..E-1: capacity; rows E..E+D-1: lambda*D_c - S_c <= 0
    rows = np.concatenate([inst.path_links, E + dem_of_path, E + np.arange(D)])
    cols = np.concatenate([path_of_inc, np.arange(P), np.full(D, P)])
    vals = np.concatenate([np.ones(inst.nnz), -np.ones(P), base_demand])
    A = coo_matrix((vals, (rows, cols)), shape=(E + D, P + 1)).tocsr()
    b = np.concatenate([inst.capacity, np.zeros(D)])
    c = np.zeros(P + 1)
    c[P] = -1.0
    res = linprog(c, A_ub=A, b_ub=b, bounds=[(0, None)] * (P + 1), method="highs")
    if res.status != 0:
        raise RuntimeError(f"lambda_star LP failed: {res.message}")
    return float(res.x[P])


def _lambda_cached(key: str, compute) -> float:
    cache = {}
    if os.path.exists(_LAMBDA_CACHE):
        with open(_LAMBDA_CACHE) as f:
            cache = json.load(f)
    if key in cache:
        return float(cache[key])
    val = compute()
    cache[key] = repr(val)
    try:
        with open(_LAMBDA_CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return val


def _assemble(name, n, src, dst, cap, pairs, base, paths, factor, meta):
    keep = [i for i, p in enumerate(paths) if len(p) > 0]
    ps = np.asarray([pairs[i][0] for i in keep], np.int32)
    pt = np.asarray([pairs[i][1] for i in keep], np.int32)
    base = np.asarray([base[i] for i in keep], np.float64)
    base = base / base.sum()
    kept_paths = [paths[i] for i in keep]
    inst = make_instance(name, n, src, dst, cap, ps, pt, base, kept_paths, meta)
    key = f"{name}:{inst.fingerprint()}"
    lam = _lambda_cached(key, lambda: max_concurrent_flow(inst, base))
    inst.demand = factor * lam * base
    inst.meta.update(lambda_star=lam, scale_factor=factor, dropped_pairs=len(pairs) - len(keep))
    return inst


def waxman20(seed: int = 0) -> Instance:
    """20-node Waxman, ~60 links, capacities {10,40,100}, all 380 pairs, lognormal(0,1) gravity,
    1.5x the path-restricted max concurrent flow, k=4 hop-shortest paths."""
    rng = np.random.default_rng(np.random.SeedSequence([1, seed]))
    n = 20
    pos, edges = waxman(n, 60, rng)
    ecap = rng.choice([10.0, 40.0, 100.0], size=len(edges))
    src, dst, cap, _ = arcs_from_edges(edges, ecap)
    w = rng.lognormal(0.0, 1.0, n)
    pairs = [(s, t) for s in range(n) for t in range(n) if s != t]
    base = gravity(w, np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]))
    paths = k_shortest_paths(n, src, dst, np.ones(len(src)), [p[0] for p in pairs], [p[1] for p in pairs], 4)
    return _assemble(f"waxman20/s{seed}", n, src, dst, cap, pairs, base, paths, 1.5,
                     dict(kind="waxman20", seed=seed, edges=len(edges)))


def waxman150(seed: int = 0) -> Instance:
    """150-node Waxman, ~600 links, capacities {100,400}, all 22,350 pairs, lognormal(0,1.5) gravity,
    1.3x the path-restricted max concurrent flow, k=8 Euclidean-latency-shortest paths."""
    rng = np.random.default_rng(np.random.SeedSequence([2, seed]))
    n = 150
    pos, edges = waxman(n, 600, rng)
    ecap = rng.choice([100.0, 400.0], size=len(edges))
    src, dst, cap, wgt = arcs_from_edges(edges, ecap, pos)
    w = rng.lognormal(0.0, 1.5, n)
    pairs = [(s, t) for s in range(n) for t in range(n) if s != t]
    base = gravity(w, np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]))
    paths = k_shortest_paths(n, src, dst, wgt, [p[0] for p in pairs], [p[1] for p in pairs], 8)
    return _assemble(f"waxman150/s{seed}", n, src, dst, cap, pairs, base, paths, 1.3,
                     dict(kind="waxman150", seed=seed, edges=len(edges)))


def two_level1000(seed: int = 0, regions: int = 50, region_nodes: int = 20, region_links: int = 80, gateways: int = 4,
            backbone_links: int = 1000, k: int = 4, factor: float = 1.3, cache_dir: str | None = None,
            progress=None) -> Instance:
    """Hierarchical WAN: `regions` Waxman regions of `region_nodes` nodes (~`region_links` links each,
    capacities {100, 400}) in their own unit sub-squares of a 10 x 5 layout, joined by a Waxman
    backbone over `gateways` gateway nodes per region (~`backbone_links` links, capacities
    {400, 1000}); all ordered pairs with gravity demands from 1 + Pareto(1.2) node weights; k
    latency-shortest paths.  Scale: factor x the uniform-split bound lambda_unif (the largest lambda
    for which lambda * D_gravity split evenly over each demand's paths fits every link), because the
    max-concurrent-flow LP over ~4M path variables is not tractable here.  Cached as .npz when
    cache_dir is given (the generation runs Yen's algorithm for ~1M pairs)."""
    if cache_dir:
        path = os.path.join(cache_dir, f"two_level1000_s{seed}.npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            return Instance(name=str(z["name"]), n_nodes=int(z["n_nodes"]), link_src=z["link_src"],
                            link_dst=z["link_dst"], capacity=z["capacity"], demand_src=z["demand_src"],
                            demand_dst=z["demand_dst"], demand=z["demand"], path_ptr=z["path_ptr"],
                            path_links=z["path_links"], demand_path_ptr=z["demand_path_ptr"],
                            meta=json.loads(str(z["meta"])))
    rng = np.random.default_rng(np.random.SeedSequence([3, seed]))
    n = regions * region_nodes
    pos = np.zeros((n, 2))
    edges, ecap = [], []
    gw = []
    cols = 10
    for g in range(regions):
        x0, y0 = (g % cols) * 1.0, (g // cols) * 1.0
        p, e = waxman(region_nodes, region_links, rng, box=(x0, y0, x0 + 1.0, y0 + 1.0))
        base = g * region_nodes
        pos[base:base + region_nodes] = p
        edges += [(u + base, v + base) for u, v in e]
        ecap += list(rng.choice([100.0, 400.0], size=len(e)))
        gw += list(base + rng.choice(region_nodes, size=gateways, replace=False))
    gw = np.array(sorted(gw))
    # backbone: Waxman over the gateway nodes at their actual positions, connected
    for _ in range(1000):
        iu, iv = np.triu_indices(len(gw), 1)
        d = np.hypot(*(pos[gw[iu]] - pos[gw[iv]]).T)
        base_p = np.exp(-d / (0.4 * d.max()))
        beta_w = min(1.0, backbone_links / base_p.sum())
        keep = rng.uniform(size=base_p.shape) < beta_w * base_p
        bb = [(int(gw[a]), int(gw[b])) for a, b in zip(iu[keep], iv[keep])]
        if _connected(n, edges + bb):
            break
    else:
        raise RuntimeError("could not draw a connected backbone")
    edges += bb
    ecap += list(rng.choice([400.0, 1000.0], size=len(bb)))
    src, dst, cap, wgt = arcs_from_edges(edges, ecap, pos)
    w = 1.0 + rng.pareto(1.2, n)
    ps, pt = np.nonzero(~np.eye(n, dtype=bool))
    ps = ps.astype(np.int32)
    pt = pt.astype(np.int32)
    counts, path_ptr, path_links = k_shortest_paths_csr(n, src, dst, wgt, ps, pt, k, progress=progress)
    keep = counts > 0
    ps, pt = ps[keep], pt[keep]
    base = gravity(w, ps, pt)
    dptr = np.concatenate([[0], np.cumsum(counts[keep])]).astype(np.int32)
    inst = Instance(name=f"two_level1000/s{seed}", n_nodes=n, link_src=src, link_dst=dst, capacity=cap,
                    demand_src=ps, demand_dst=pt, demand=base, path_ptr=path_ptr, path_links=path_links,
                    demand_path_ptr=dptr, meta=dict(kind="two_level1000", seed=seed, edges=len(edges),
                                                    backbone_edges=len(bb)))
    # uniform-split bound
    m = np.diff(inst.demand_path_ptr)
    path_of_inc = np.repeat(np.arange(inst.n_paths), np.diff(inst.path_ptr))
    dem_of_path = np.repeat(np.arange(inst.n_demands), m)
    per_path = base[dem_of_path] / m[dem_of_path]
    load = np.bincount(inst.path_links, weights=per_path[path_of_inc], minlength=inst.n_links)
    used = load > 0
    lam = float(np.min(inst.capacity[used] / load[used]))
    inst.demand = factor * lam * base
    inst.meta.update(lambda_unif=lam, scale_factor=factor, dropped_pairs=int((~keep).sum()))
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(os.path.join(cache_dir, f"two_level1000_s{seed}.npz"), name=inst.name, n_nodes=inst.n_nodes,
                 link_src=inst.link_src, link_dst=inst.link_dst, capacity=inst.capacity, demand_src=inst.demand_src,
                 demand_dst=inst.demand_dst, demand=inst.demand, path_ptr=inst.path_ptr, path_links=inst.path_links,
                 demand_path_ptr=inst.demand_path_ptr, meta=json.dumps(inst.meta))
    return inst


def failure_scenarios(seed: int = 0, n_scen: int = 512, base_seed: int = 0):
    """Failure scenarios on the 20-node topology: 1-3 undirected links cut, each demand times
    exp(N(0, 0.3)), paths recomputed with k_c ~ U{2..8} hop-shortest paths, disconnected pairs dropped."""
    base = waxman20(base_seed)
    n = base.n_nodes
    n_edges = base.n_links // 2
    ss = np.random.SeedSequence([4, seed]).spawn(n_scen)
    out = []
    for i, s in enumerate(ss):
        rng = np.random.default_rng(s)
        ncut = int(rng.integers(1, 4))
        cut = set(rng.choice(n_edges, size=ncut, replace=False).tolist())
        keep_arcs = [a for a in range(base.n_links) if (a // 2) not in cut]
        remap = {a: j for j, a in enumerate(keep_arcs)}
        src = base.link_src[keep_arcs]
        dst = base.link_dst[keep_arcs]
        cap = base.capacity[keep_arcs]
        dem = base.demand * np.exp(rng.normal(0.0, 0.3, base.n_demands))
        kper = rng.integers(2, 9, base.n_demands)
        paths = k_shortest_paths(n, src, dst, np.ones(len(src)), base.demand_src, base.demand_dst, kper)
        keep = [c for c in range(base.n_demands) if len(paths[c]) > 0]
        inst = make_instance(f"failures/s{seed}/{i}", n, src, dst, cap, base.demand_src[keep],
                             base.demand_dst[keep], dem[keep], [paths[c] for c in keep],
                             dict(kind="failures", seed=seed, scenario=i, cut=sorted(cut),
                                  dropped_pairs=base.n_demands - len(keep)))
        del remap
        out.append(inst)
    return out


# ----------------------------------------------------------------------------------------------
# synthetic drift of the network state over time (drift-adjusted optimality, section 4.1)
# ----------------------------------------------------------------------------------------------
SWING_5MIN = 0.35  # mean absolute relative demand change over five minutes (section 2, after prior work)
CAP_EVENTS_PER_DAY = 200.0  # link-capacity changes per day over the whole network (section 2: "O(100s)")


def swing_sigma(swing: float = SWING_5MIN) -> float:
    """Volatility per period of the mean-preserving lognormal ratio Y = exp(sigma Z - sigma^2 / 2)
    whose mean absolute change E|Y - 1| equals `swing`.  Since E[Y] = 1, E|Y - 1| = 2 E[(Y - 1)+]
    = 2 (2 Phi(sigma / 2) - 1), so sigma = 2 Phi^-1((1 + swing / 2) / 2)."""
    from scipy.stats import norm
    if not 0.0 <= swing < 2.0:
        raise ValueError("swing must be in [0, 2)")
    return float(2.0 * norm.ppf((1.0 + 0.5 * swing) / 2.0))


def drift_path(inst: Instance, times, seed: int = 0, swing: float = SWING_5MIN, period: float = 300.0,
               cap_events_per_day: float = CAP_EVENTS_PER_DAY, cap_low: float = 0.25):
    """Network states at `times` (seconds after T_0, sorted, >= 0) along ONE seeded sample path, as
    Instances with the topology and paths of `inst` and drifted capacities and demands.

    * Demands: independent geometric Brownian motions without drift in the mean,
      D_c(t) = D_c(0) exp(sigma W_c(t / period) - sigma^2 t / (2 period)), with sigma = swing_sigma(swing),
      so that the mean absolute change over one period is `swing` and E[D_c(t)] = D_c(0).
    * Capacities: capacity-change events arrive as a Poisson process of rate cap_events_per_day / 86400
      per second over the whole network, each on a uniformly drawn link with nonzero capacity, which
      is set to its T_0 capacity times U(cap_low, 1) (a degradation, or a partial recovery).
    States at later times extend the same path, so a state at T_K is the drift of the state at any
    earlier grid time."""
    times = np.asarray(times, dtype=np.float64)
    if times.ndim != 1 or np.any(times < 0.0) or np.any(np.diff(times) < 0.0):
        raise ValueError("times must be a sorted 1-D array of non-negative seconds")
    rng = np.random.default_rng(np.random.SeedSequence([11, seed]))
    sigma = swing_sigma(swing)
    D, E = inst.n_demands, inst.n_links
    t_end = float(times[-1]) if times.size else 0.0
    n_ev = int(rng.poisson(cap_events_per_day / 86400.0 * t_end)) if t_end > 0.0 else 0
    ev_t = np.sort(rng.uniform(0.0, t_end, n_ev)) if n_ev else np.zeros(0)
    live = np.flatnonzero(inst.capacity > 0.0)
    ev_link = rng.choice(live, size=n_ev) if n_ev else np.zeros(0, np.int64)
    ev_f = rng.uniform(cap_low, 1.0, n_ev)
    logw = np.zeros(D)
    t_prev = 0.0
    out = []
    for t in times:
        dt = (t - t_prev) / period
        if dt > 0.0:
            logw += np.sqrt(dt) * rng.standard_normal(D)
        t_prev = t
        demand = inst.demand * np.exp(sigma * logw - 0.5 * sigma * sigma * t / period)
        cap = inst.capacity.copy()
        for j in range(int(np.searchsorted(ev_t, t, side="right"))):
            cap[ev_link[j]] = inst.capacity[ev_link[j]] * ev_f[j]
        meta = dict(inst.meta, drift=dict(seed=seed, t=float(t), swing=swing, period=period,
                                          cap_events=int(np.searchsorted(ev_t, t, side="right"))))
        out.append(Instance(name=f"{inst.name}@{float(t):g}s", n_nodes=inst.n_nodes, link_src=inst.link_src,
                            link_dst=inst.link_dst, capacity=cap, demand_src=inst.demand_src,
                            demand_dst=inst.demand_dst, demand=demand, path_ptr=inst.path_ptr,
                            path_links=inst.path_links, demand_path_ptr=inst.demand_path_ptr, meta=meta))
    return out


# ----------------------------------------------------------------------------------------------
# small closed-form instances (for pins)
# ----------------------------------------------------------------------------------------------
def parking_lot(L: int, demand: float = 10.0, cap: float = 1.0) -> Instance:
    """Chain of L unit links; demand 0 uses all L links, demand i (1..L) uses link i-1 only."""
    src = np.arange(L, dtype=np.int32)
    dst = src + 1
    paths = [[list(range(L))]] + [[[i]] for i in range(L)]
    dsrc = [0] + list(range(L))
    ddst = [L] + list(range(1, L + 1))
    return make_instance(f"parking_lot{L}", L + 1, src, dst, np.full(L, cap), dsrc, ddst,
                         np.full(L + 1, demand), paths)


def shared_link(demands, cap: float = 1.0) -> Instance:
    """One link shared by single-path demands."""
    n = len(demands)
    return make_instance("shared_link", 2, [0], [1], [cap], [0] * n, [1] * n, demands, [[[0]] for _ in range(n)])


def parallel_paths(caps, demand) -> Instance:
    """One demand over disjoint single-link paths."""
    m = len(caps)
    return make_instance("parallel", 2, [0] * m, [1] * m, caps, [0], [1], [demand], [[[i] for i in range(m)]])


def single_paths(seed: int = 0, n_links: int = 17000, n_demands: int = 600000) -> Instance:
    """Edge-case instance for the privatised link sums' chunking (not a network): many demands of one
    path each, of 1 to 3 distinct links drawn uniformly, capacities in {1, 4, 10} x 100, demands
    log-uniform over two orders of magnitude.  Built without per-demand Python lists (vectorised)."""
    rng = np.random.default_rng(np.random.SeedSequence([11, seed]))
    hops = rng.integers(1, 4, size=n_demands)
    base = rng.integers(0, n_links, size=n_demands)
    off1 = rng.integers(1, n_links // 2, size=n_demands)
    off2 = off1 + rng.integers(1, n_links // 2, size=n_demands)  # 0 < off1 < off2 < n_links: distinct links
    cand = np.stack([base, (base + off1) % n_links, (base + off2) % n_links], axis=1)
    keep = np.arange(3)[None, :] < hops[:, None]
    links = cand[keep].astype(np.int32)  # row-major: each demand's first hops links, in order
    path_ptr = np.concatenate([[0], np.cumsum(hops)]).astype(np.int64)
    cap = 100.0 * rng.choice([1.0, 4.0, 10.0], size=n_links)
    demand = 10.0 ** rng.uniform(-1.0, 1.0, n_demands)
    src = np.arange(n_links, dtype=np.int32)
    return Instance(name=f"single_paths/s{seed}", n_nodes=n_links + 1, link_src=src, link_dst=src + 1,
                    capacity=cap, demand_src=np.zeros(n_demands, np.int32), demand_dst=np.ones(n_demands, np.int32),
                    demand=demand, path_ptr=path_ptr, path_links=links,
                    demand_path_ptr=np.arange(n_demands + 1, dtype=np.int32),
                    meta=dict(kind="single_paths", seed=seed))


def ragged(seed: int = 0, n_links: int = 48, n_demands: int = 40, max_hops: int = 12) -> Instance:
    """Edge-case instance for the kernels' boundaries (not a network): demands with 1, 2, 3, 5, 8, 17,
    33 and 64 paths (64 is the per-demand maximum), paths of 1 to max_hops links (12: beyond the 8-hop
    gather batch; above 16: beyond the fixed-width hop records, so the kernels read the CSR layout),
    one link on a large share of all paths, unused links with zero capacity, and demands spanning four
    orders of magnitude.  Path link sets are drawn without repeats inside a path."""
    rng = np.random.default_rng(np.random.SeedSequence([7, seed]))
    used = n_links - 4  # the last four links carry no path
    cap = np.concatenate([rng.choice([1.0, 4.0, 10.0], size=used), np.zeros(4)])
    counts = rng.choice([1, 2, 3, 5, 8, 17, 33, 64], size=n_demands)
    counts[0], counts[1] = 64, 1
    paths = []
    for c in range(n_demands):
        plist = []
        for _ in range(int(counts[c])):
            hops = int(rng.integers(1, max_hops + 1))
            links = rng.choice(used - 1, size=hops, replace=False) + 1
            if rng.uniform() < 0.4:
                links[0] = 0  # the hot link
            plist.append(sorted(set(int(e) for e in links)))
        paths.append(plist)
    demand = 10.0 ** rng.uniform(-2.0, 2.0, n_demands)
    src = np.arange(n_links, dtype=np.int32)
    return make_instance(f"ragged/s{seed}", n_links + 1, src, src + 1, cap, np.zeros(n_demands), np.ones(n_demands),
                         demand, paths, meta=dict(kind="ragged", seed=seed))
