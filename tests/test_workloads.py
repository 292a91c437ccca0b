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


def test_swing_sigma_calibration():
    """The lognormal ratio exp(sigma Z - sigma^2 / 2) has mean 1 and mean absolute change `swing`
    (checked by quadrature of the normal density, independent of the closed form)."""
    from scipy import integrate
    for swing in (0.0, 0.1, 0.35, 1.0):
        s = W.swing_sigma(swing)
        dens = lambda z: np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)  # noqa: E731
        mean = integrate.quad(lambda z: np.exp(s * z - 0.5 * s * s) * dens(z), -40, 40)[0]
        mad = integrate.quad(lambda z: abs(np.exp(s * z - 0.5 * s * s) - 1.0) * dens(z), -40, 40, points=[s / 2])[0]
        assert abs(mean - 1.0) < 1e-9
        assert abs(mad - swing) < 1e-9
    with pytest.raises(ValueError):
        W.swing_sigma(2.5)


def test_drift_path_statistics(waxman20):
    """Demands: unchanged at t = 0, mean absolute change ~35 % after five minutes, log-variance
    growing linearly in time, mean preserved.  Capacities: only links with capacity change, each to
    a fraction in [0.25, 1] of its initial value; topology and paths untouched."""
    base = waxman20
    # many independent demands: replicate the instance's demand vector
    big = W.Instance(name="rep", n_nodes=base.n_nodes, link_src=base.link_src, link_dst=base.link_dst,
                     capacity=base.capacity, demand_src=np.zeros(40000, np.int32), demand_dst=np.ones(40000, np.int32),
                     demand=np.ones(40000), path_ptr=base.path_ptr, path_links=base.path_links,
                     demand_path_ptr=base.demand_path_ptr)
    st = W.drift_path(big, [0.0, 75.0, 300.0, 1200.0], seed=4, cap_events_per_day=86400 * 0.05)
    np.testing.assert_array_equal(st[0].demand, big.demand)
    np.testing.assert_array_equal(st[0].capacity, big.capacity)
    r300 = st[2].demand
    assert abs(np.mean(np.abs(r300 - 1.0)) - 0.35) < 0.01
    assert abs(np.mean(r300) - 1.0) < 0.01
    sig2 = W.swing_sigma() ** 2
    for s, t in zip(st[1:], (75.0, 300.0, 1200.0)):
        assert abs(np.var(np.log(s.demand)) / (sig2 * t / 300.0) - 1.0) < 0.05
        assert np.all(s.demand > 0) and np.all(np.isfinite(s.demand))
        ratio = s.capacity / big.capacity
        changed = ratio != 1.0
        assert np.all((ratio[changed] >= 0.25) & (ratio[changed] <= 1.0))
        assert s.path_links is big.path_links and s.demand_path_ptr is big.demand_path_ptr
    assert st[-1].meta["drift"]["cap_events"] > 0
    # the same call gives the same path
    again = W.drift_path(big, [0.0, 75.0, 300.0, 1200.0], seed=4, cap_events_per_day=86400 * 0.05)
    np.testing.assert_array_equal(again[3].demand, st[3].demand)
    np.testing.assert_array_equal(again[3].capacity, st[3].capacity)
    with pytest.raises(ValueError):
        W.drift_path(big, [1.0, 0.5])


def test_drift_path_keeps_unused_links_at_zero():
    inst = W.ragged(0)
    s = W.drift_path(inst, [3600.0], seed=1, cap_events_per_day=86400.0)[0]
    assert np.all(s.capacity[inst.capacity == 0.0] == 0.0)
    assert s.meta["drift"]["cap_events"] > 0


def test_single_paths_shape():
    inst = W.single_paths(1, n_links=500, n_demands=20000)
    assert inst.n_demands == 20000 and inst.n_paths == 20000
    np.testing.assert_array_equal(inst.demand_path_ptr, np.arange(20001))
    hops = np.diff(inst.path_ptr)
    assert hops.min() == 1 and hops.max() == 3 and inst.nnz == hops.sum()
    pl = inst.path_links
    assert pl.min() >= 0 and pl.max() < 500
    # the links of a path are distinct
    for h in (2, 3):
        rows = np.flatnonzero(hops == h)
        ids = pl[inst.path_ptr[rows][:, None] + np.arange(h)[None, :]]
        assert np.all(ids[:, 0] != ids[:, 1])
        if h == 3:
            assert np.all((ids[:, 2] != ids[:, 0]) & (ids[:, 2] != ids[:, 1]))
    again = W.single_paths(1, n_links=500, n_demands=20000)
    np.testing.assert_array_equal(again.path_links, pl)
    np.testing.assert_array_equal(again.demand, inst.demand)
