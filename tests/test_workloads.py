"""Input generators: determinism, path order, instance shapes (no solver arithmetic here)."""
import numpy as np
import pytest

import workloads as W


def _all_simple_paths(n, arcs, w, s, t):
    adj = {u: [] for u in range(n)}
    for a, (u, v) in enumerate(arcs):
        adj[u].append((v, a))
    out = []

    def rec(u, nodes, used):
        if u == t:
            out.append((sum(w[a] for a in used), tuple(nodes), tuple(used)))
            return
        for v, a in adj[u]:
            if v not in nodes:
                rec(v, nodes + [v], used + [a])

    rec(s, [s], [])
    return out


@pytest.mark.parametrize("seed", range(6))
def test_yen_matches_brute_force_order(seed):
    rng = np.random.default_rng(seed)
    n = 7
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.uniform() < 0.5]
    arcs = [(u, v) for u, v in edges] + [(v, u) for u, v in edges]
    hop = seed % 2 == 0
    w = np.ones(len(arcs)) if hop else rng.uniform(0.5, 2.0, len(arcs))
    pairs = [(s, t) for s in range(n) for t in range(n) if s != t]
    k = 5
    res = W.k_shortest_paths(n, [a[0] for a in arcs], [a[1] for a in arcs], w, [p[0] for p in pairs],
                             [p[1] for p in pairs], k)
    for (s, t), got in zip(pairs, res):
        allp = _all_simple_paths(n, arcs, w, s, t)
        # (cost, node sequence) order; costs summed in path order like the generator
        allp.sort(key=lambda z: (z[0], z[1]))
        want = [list(z[2]) for z in allp[:k]]
        assert got == want, (s, t)


def test_waxman20_deterministic_and_shaped():
    a = W.waxman20(0)
    b = W.waxman20(0)
    assert a.fingerprint() == b.fingerprint()
    assert a.n_nodes == 20 and a.n_demands == 380
    assert 54 <= a.n_links // 2 <= 66
    assert set(np.unique(a.capacity)) <= {10.0, 40.0, 100.0}
    npaths = np.diff(a.demand_path_ptr)
    assert npaths.min() >= 1 and npaths.max() <= 4
    # every path is a simple chain of arcs from its demand's source to destination
    dem_of = np.repeat(np.arange(a.n_demands), npaths)
    for r in range(a.n_paths):
        links = a.path_links[a.path_ptr[r]:a.path_ptr[r + 1]]
        assert a.link_src[links[0]] == a.demand_src[dem_of[r]]
        assert a.link_dst[links[-1]] == a.demand_dst[dem_of[r]]
        assert np.all(a.link_dst[links[:-1]] == a.link_src[links[1:]])
        nodes = list(a.link_src[links]) + [a.link_dst[links[-1]]]
        assert len(set(nodes)) == len(nodes)
    assert W.waxman20(1).fingerprint() != a.fingerprint()


def test_lambda_star_scaling(waxman20):
    """D = 1.5 * lambda_star * D_gravity: the scaled-down demand 1/1.5 * D is exactly routable."""
    base = waxman20.demand / (1.5 * waxman20.meta["lambda_star"])
    lam = W.max_concurrent_flow(waxman20, base)
    assert lam == pytest.approx(waxman20.meta["lambda_star"], rel=1e-7)


def test_failure_scenarios_small():
    sc = W.failure_scenarios(0, n_scen=4)
    assert len(sc) == 4
    for inst in sc:
        npaths = np.diff(inst.demand_path_ptr)
        assert npaths.min() >= 1 and npaths.max() <= 8
        cut = inst.meta["cut"]
        assert 1 <= len(cut) <= 3
    assert sc[0].fingerprint() != sc[1].fingerprint()
    assert W.failure_scenarios(0, n_scen=2)[1].fingerprint() == sc[1].fingerprint()


def test_small_builders():
    pl = W.parking_lot(3)
    assert pl.n_demands == 4 and pl.n_paths == 4 and pl.nnz == 6
    sl = W.shared_link([0.1, 0.2])
    assert sl.n_links == 1 and sl.nnz == 2
    pp = W.parallel_paths([0.2, 0.3], 1.0)
    assert pp.n_paths == 2
