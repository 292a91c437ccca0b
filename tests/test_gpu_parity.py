"""GPU parity of the HIP path (through the C ABI) with the FP64 oracle.

Parity is taken at equal iteration counts with the oracle's (beta, alpha) schedule replayed on
the GPU, so that discrete decisions (beta steps, alpha increments) cannot flip between FP32 and
FP64.  The bar is on the per-demand sums S_c before projection:
    |S_gpu - S_oracle| <= 1e-4 * max(|S_oracle|, floor),  floor = 1e-2 * max_c D_c
i.e. 1e-4 relative for every demand above 1% of the largest one, and an absolute 1e-6 * max D
below it.  In normalised units (capacities <= 1) the iteration's terms are O(1) and FP32 spaces
them ~1e-7 apart; a small S_c is the difference of such terms, so below the floor only an
absolute bar of a few FP32 ulps of the unit scale is meaningful.  The projection (Algorithm 2) is checked for
feasibility and against the oracle's projection of the GPU's own unprojected rates.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def te(torch):
    import paper_2605_01748_amd as te_mod
    te_mod.library()
    return te_mod


@pytest.fixture(scope="module")
def c1():
    return W.waxman20(0)


@pytest.fixture(scope="module")
def c2():
    return W.waxman150(0)


def _oracle_run(inst, K, **kw):
    r = O.solve(inst, O.Options(fixed_iters=K, project=False, **kw), want_state=False)
    sb, sa = r.schedule
    return r, sb, sa


def _rel_err(S_gpu, S_orc, dem):
    floor = 1e-2 * dem.max()
    return np.abs(S_gpu - S_orc) / np.maximum(np.abs(S_orc), floor)


def _report(tag, S_gpu, S_orc, dem):
    err = _rel_err(S_gpu, S_orc, dem)
    big = np.abs(S_orc) >= 1e-2 * dem.max()
    pure = np.abs(S_gpu - S_orc)[big] / np.abs(S_orc)[big]
    absn = np.abs(S_gpu - S_orc).max() / dem.max()
    print(f"{tag}: max err {err.max():.3e} (p99 {np.quantile(err, 0.99):.3e}); pure relative on "
          f"S >= 1% max D: {pure.max() if pure.size else 0:.3e}; max |dS|/max D {absn:.3e}")
    return err


def _gpu_raw(te, prob, K, sb, sa, engine):
    opts = te.Options(fixed_iters=K, project=False, engine=engine, sched_beta=sb, sched_alpha=sa)
    x, S, st = prob.solve(opts)
    return x.cpu().numpy().astype(np.float64), S.cpu().numpy().astype(np.float64), st


@pytest.mark.parametrize("engine", ["block", "graph"])
@pytest.mark.parametrize("K", [1, 2, 16, 256])
def test_parity_waxman20(te, c1, engine, K):
    r, sb, sa = _oracle_run(c1, K)
    prob = te.Problem(c1)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    x, S, st = _gpu_raw(te, prob, K, sb, sa, eng)
    assert st["iters"] == K and st["engine"] == eng
    err = _report(f"waxman20 {engine} K={K}", S, r.S_raw * r.scale, c1.demand)
    assert err.max() <= REL


@pytest.mark.parametrize("K", [16, 256, 833])  # 833: the budget the benchmark times (first to reach 0.99)
def test_parity_waxman150_graph(te, c2, K):
    r, sb, sa = _oracle_run(c2, K)
    prob = te.Problem(c2)
    x, S, st = _gpu_raw(te, prob, K, sb, sa, te.ENGINE_GRAPH)
    assert st["iters"] == K
    err = _report(f"waxman150 graph K={K} ({st['ms']:.3f} ms)", S, r.S_raw * r.scale, c2.demand)
    assert err.max() <= REL


@pytest.fixture(scope="module")
def c3_small():
    # the two-level WAN generator at 6 regions (120 nodes, ~1,150 arcs, 14,280 pairs, k = 4):
    # same structure as the 1,000-node instance, at a size the oracle runs in a fraction of a second
    return W.two_level1000(1, regions=6, backbone_links=120)


@pytest.mark.slow
def test_parity_hierarchical_full_size(te):
    """The 1,000-node two-level instance (999,000 demands, ~4.0M paths, ~23.5M incidences) after 16
    iterations, every demand against the oracle."""
    inst = W.two_level1000(0)
    print(inst.summary(), flush=True)
    K = 16
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    # the link kernel's workgroups stay within the rows the control prefetch reads
    assert prob.info()["link_workgroups"] <= 512
    x, S, st = _gpu_raw(te, prob, K, sb, sa, te.ENGINE_GRAPH)
    assert st["iters"] == K
    assert st["paths_per_lane"] == 2  # the default for instances of this size
    err = _report(f"hierarchical 1000-node graph K={K} ({st['ms']:.3f} ms)", S, r.S_raw * r.scale, inst.demand)
    assert err.max() <= REL
    # Algorithm 2 at full size (links carrying up to ~10^5 paths go through the radix selection):
    # feasible, and the same per-demand sums as the oracle's Algorithm 2 on the GPU's own rates
    xp, Sp, stp = prob.solve(te.Options(fixed_iters=K, project=True, engine=te.ENGINE_GRAPH,
                                        sched_beta=sb, sched_alpha=sa))
    xp = xp.cpu().numpy().astype(np.float64)
    assert np.all(xp >= 0)
    assert np.all(O.link_loads(inst, xp) <= inst.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(inst, xp) <= inst.demand * (1 + 1e-7))
    ref = O.project(inst, x.astype(np.float64), stp["final_alpha"])
    d = np.abs(O.demand_sums(inst, xp) - O.demand_sums(inst, ref))
    print(f"hierarchical 1000-node projection: max |dS| {d.max():.3e} (max D {inst.demand.max():.3e})")
    np.testing.assert_allclose(O.demand_sums(inst, xp), O.demand_sums(inst, ref), rtol=1e-5,
                               atol=1e-6 * inst.capacity.max())


@pytest.mark.parametrize("K", [16, 128])
def test_parity_hierarchical_graph(te, c3_small, K):
    r, sb, sa = _oracle_run(c3_small, K)
    prob = te.Problem(c3_small)
    x, S, st = _gpu_raw(te, prob, K, sb, sa, te.ENGINE_GRAPH)
    assert st["iters"] == K
    err = _report(f"hierarchical graph K={K} ({st['ms']:.3f} ms)", S, r.S_raw * r.scale, c3_small.demand)
    assert err.max() <= REL


_EDGE = {
    "ragged0": lambda: W.ragged(0),
    "ragged1": lambda: W.ragged(1, n_links=20, n_demands=70),
    "one_link_one_demand": lambda: W.shared_link([5.0], cap=1.0),
    "shared_link": lambda: W.shared_link([0.1, 0.5, 2.0, 8.0], cap=1.0),
    "parallel_64": lambda: W.parallel_paths(np.linspace(0.5, 2.0, 64), 50.0),
}


@pytest.mark.parametrize("engine", ["block", "graph"])
@pytest.mark.parametrize("K", [1, 64])
@pytest.mark.parametrize("name", sorted(_EDGE))
def test_parity_edge_cases(te, name, engine, K):
    """Ragged path counts (1..64 per demand), paths longer than the gather batch, unused links,
    a single link and a single demand, and the widest demand (64 paths on one link each)."""
    inst = _EDGE[name]()
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    x, S, st = _gpu_raw(te, prob, K, sb, sa, eng)
    assert st["iters"] == K and st["engine"] == eng
    err = _report(f"{name} {engine} K={K}", S, r.S_raw * r.scale, inst.demand)
    assert err.max() <= REL
    # the projected output is feasible on every edge case
    xp, _, _ = prob.solve(te.Options(fixed_iters=K, engine=eng, sched_beta=sb, sched_alpha=sa))
    xp = xp.cpu().numpy().astype(np.float64)
    assert np.all(xp >= 0)
    assert np.all(O.link_loads(inst, xp) <= inst.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(inst, xp) <= inst.demand * (1 + 1e-7))


@pytest.mark.parametrize("engine", ["block", "graph"])
@pytest.mark.parametrize("alpha", [0.0, 1.0, 2.0])
def test_parity_finite_alpha_targets(te, c1, engine, alpha):
    """Max-flow (alpha = 0), proportional fairness (1) and alpha = 2 as fixed targets."""
    K = 400  # with gamma = 0.03 the schedule reaches alpha = 1 at sweep 151 and alpha = 2 at 331
    r, sb, sa = _oracle_run(c1, K, alpha_target=alpha, gamma=3e-2)
    assert np.max(sa) == alpha
    prob = te.Problem(c1)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    x, S, st = _gpu_raw(te, prob, K, sb, sa, eng)
    err = _report(f"waxman20 alpha={alpha} {engine}", S, r.S_raw * r.scale, c1.demand)
    assert err.max() <= REL


@pytest.mark.parametrize("engine", ["block", "graph"])
def test_adaptive_stop_proportional(te, c1, engine):
    """Adaptive mode (no replay) at alpha_target = 1: the GPU's own residual test stops the solve,
    near the oracle's stop and at nearly the oracle's allocation."""
    r = O.solve(c1, O.Options(alpha_target=1.0, gamma=1e-3, max_iters=20000, project=False), want_state=False)
    assert r.flags & O.CONVERGED
    prob = te.Problem(c1)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    x, S, st = prob.solve(te.Options(alpha_target=1.0, gamma=1e-3, max_iters=20000, project=False, engine=eng))
    S = S.cpu().numpy().astype(np.float64)
    print(f"adaptive alpha=1 {engine}: GPU {st['iters']} iterations, oracle {r.iters}; "
          f"max |dS|/max D {np.abs(S - r.S_raw * r.scale).max() / c1.demand.max():.2e}")
    assert st["flags"] & te.TE_CONVERGED and st["final_alpha"] == 1.0
    assert 0.8 * r.iters <= st["iters"] <= 1.25 * r.iters
    assert np.abs(S - r.S_raw * r.scale).max() <= 1e-2 * c1.demand.max()


@pytest.mark.parametrize("engine", ["block", "graph"])
def test_projection_waxman20(te, c1, engine):
    K = 300
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    prob = te.Problem(c1)
    r, sb, sa = _oracle_run(c1, K)
    opts = dict(fixed_iters=K, engine=eng, sched_beta=sb, sched_alpha=sa)
    xr, Sr, _ = prob.solve(te.Options(project=False, **opts))
    xp, Sp, st = prob.solve(te.Options(project=True, **opts))
    xr = xr.cpu().numpy().astype(np.float64)
    xp = xp.cpu().numpy().astype(np.float64)
    # feasibility of the FP32 output
    L = O.link_loads(c1, xp)
    assert np.all(xp >= 0)
    assert np.all(L <= c1.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(c1, xp) <= c1.demand * (1 + 1e-7))
    # same trims as the oracle's Algorithm 2 applied to the GPU's own unprojected rates
    ref = O.project(c1, xr, st["final_alpha"])
    np.testing.assert_allclose(xp, ref, rtol=2e-6, atol=1e-6 * c1.capacity.max())


def test_projection_waxman150_graph(te, c2):
    K = 64
    prob = te.Problem(c2)
    r, sb, sa = _oracle_run(c2, K)
    opts = dict(fixed_iters=K, engine=te.ENGINE_GRAPH, sched_beta=sb, sched_alpha=sa)
    xr, _, _ = prob.solve(te.Options(project=False, **opts))
    xp, Sp, st = prob.solve(te.Options(project=True, **opts))
    xr = xr.cpu().numpy().astype(np.float64)
    xp = xp.cpu().numpy().astype(np.float64)
    L = O.link_loads(c2, xp)
    assert np.all(xp >= 0)
    assert np.all(L <= c2.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(c2, xp) <= c2.demand * (1 + 1e-7))
    ref = O.project(c2, xr, st["final_alpha"])
    np.testing.assert_allclose(O.demand_sums(c2, xp), O.demand_sums(c2, ref), rtol=1e-5,
                               atol=1e-6 * c2.capacity.max())


def test_adaptive_solve_reaches_maxmin_waxman20(te, c1):
    gold = np.load(_golden("maxmin_waxman20_s0.npz"))["S"]
    prob = te.Problem(c1)
    x, S, st = prob.solve(te.Options(fixed_iters=600))
    S = S.cpu().numpy().astype(np.float64)
    opt = O.optimality(S, gold, 1e-9)
    print(f"waxman20 K=600 optimality {opt:.5f} alpha {st['final_alpha']} beta {st['beta']}")
    assert opt >= 0.99


@pytest.mark.parametrize("threads,ppl", [(256, 1), (512, 1), (1024, 1), (256, 8), (512, 2), (1024, 4)])
def test_batch_equals_individual(te, threads, ppl):
    """One launch over uneven instances gives each the same rates as its own workgroup-engine solve
    with the same workgroup size and paths per lane (bit for bit)."""
    scen = W.failure_scenarios(0, n_scen=24)
    probs = [te.Problem(s) for s in scen]
    batch = te.Batch(probs)
    opts = te.Options(fixed_iters=200, block_threads=threads, paths_per_lane=ppl)
    xb, Sb, stb = batch.solve(opts)
    xb = xb.cpu().numpy()
    off = 0
    for p, s, stt in zip(probs, scen, stb):
        x, S, st = p.solve(te.Options(fixed_iters=200, engine=te.ENGINE_BLOCK, block_threads=threads,
                                      paths_per_lane=ppl))
        np.testing.assert_array_equal(xb[off:off + s.n_paths], x.cpu().numpy())
        assert stt["iters"] == st["iters"] == 200
        assert stt["block_threads"] == st["block_threads"] == threads
        assert stt["paths_per_lane"] == st["paths_per_lane"] == ppl
        off += s.n_paths


@pytest.mark.parametrize("threads", [256, 512])
def test_parity_block_workgroup_sizes(te, c1, threads):
    """The workgroup engine at every workgroup size against the oracle (schedule replayed)."""
    K = 256
    r, sb, sa = _oracle_run(c1, K)
    prob = te.Problem(c1)
    opts = te.Options(fixed_iters=K, project=False, engine=te.ENGINE_BLOCK, block_threads=threads,
                      sched_beta=sb, sched_alpha=sa)
    x, S, st = prob.solve(opts)
    assert st["block_threads"] == threads
    err = _report(f"waxman20 block threads={threads}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                  c1.demand)
    assert err.max() <= REL


def test_batch_tuned_workgroup_size(te):
    """block_threads = paths_per_lane = 0 on a batch: the pair measured fastest on the first solve is
    kept, and the result equals the forced solve with that pair; fixing one member tunes the other."""
    scen = W.failure_scenarios(1, n_scen=64)
    batch = te.Batch([te.Problem(s) for s in scen])
    x1, _, st1 = batch.solve(te.Options(fixed_iters=64))
    t, q = st1[0]["block_threads"], st1[0]["paths_per_lane"]
    assert t in (256, 512, 1024) and q in (1, 2, 4, 8)
    assert all(s["block_threads"] == t and s["paths_per_lane"] == q for s in st1)
    x2, _, st2 = batch.solve(te.Options(fixed_iters=64))
    assert (st2[0]["block_threads"], st2[0]["paths_per_lane"]) == (t, q)
    x3, _, _ = batch.solve(te.Options(fixed_iters=64, block_threads=t, paths_per_lane=q))
    np.testing.assert_array_equal(x1.cpu().numpy(), x3.cpu().numpy())
    _, _, st4 = batch.solve(te.Options(fixed_iters=64, paths_per_lane=1))
    assert st4[0]["paths_per_lane"] == 1 and st4[0]["block_threads"] in (256, 512, 1024)
    _, _, st5 = batch.solve(te.Options(fixed_iters=64, block_threads=256))
    assert st5[0]["block_threads"] == 256 and st5[0]["paths_per_lane"] in (1, 2, 4, 8)
    print(f"tuned for 64 scenarios: {t} threads, {q} paths per lane")


@pytest.mark.parametrize("ppl", [2, 4, 8])
@pytest.mark.parametrize("name", ["waxman20", "ragged0"])
def test_parity_block_paths_per_lane(te, c1, ppl, name):
    """The workgroup engine with 2, 4 and 8 paths per lane against the oracle (schedule replayed),
    on the 20-node instance (8 path slots per demand) and the edge-case instance (1 to 64 paths)."""
    inst = c1 if name == "waxman20" else W.ragged(0)
    K = 256
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    opts = te.Options(fixed_iters=K, project=False, engine=te.ENGINE_BLOCK, block_threads=256, paths_per_lane=ppl,
                      sched_beta=sb, sched_alpha=sa)
    x, S, st = prob.solve(opts)
    assert st["paths_per_lane"] == ppl
    err = _report(f"{name} block ppl={ppl}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale, inst.demand)
    assert err.max() <= REL


def test_update_and_warm_start(te, c1, torch):
    prob = te.Problem(c1)
    x, S, st = prob.solve(te.Options(fixed_iters=300))
    dem2 = c1.demand * 1.1
    prob.update(demand=dem2)
    inst2 = W.make_instance("c1b", c1.n_nodes, c1.link_src, c1.link_dst, c1.capacity, c1.demand_src,
                            c1.demand_dst, dem2, [[c1.path_links[c1.path_ptr[r]:c1.path_ptr[r + 1]].tolist()
                                                   for r in range(c1.demand_path_ptr[c], c1.demand_path_ptr[c + 1])]
                                                  for c in range(c1.n_demands)])
    fresh = te.Problem(inst2)
    xa, _, _ = prob.solve(te.Options(fixed_iters=50))
    xb, _, _ = fresh.solve(te.Options(fixed_iters=50))
    np.testing.assert_array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    xw, Sw, stw = prob.solve(te.Options(fixed_iters=50), x0=x)
    assert np.all(np.isfinite(xw.cpu().numpy()))


def test_workgroup_engine_at_its_lds_limit(te):
    """The largest edge-case instance (1 to 64 paths per demand, 1 to 12 hops) that the automatic
    choice still runs inside one workgroup, i.e. within ~156 KB of LDS: parity with the oracle for
    several workgroup shapes, alone and in a batch with a small instance; one demand more and the
    workgroup engine refuses it (the automatic choice moves to the graph engine)."""
    big, over = None, None
    for nd in range(60, 400, 8):
        inst = W.ragged(3, n_links=300, n_demands=nd)
        if te.Problem(inst).info()["auto_engine"] == te.ENGINE_BLOCK:
            big = inst
        else:
            over = inst
            break
    assert big is not None and over is not None
    print(f"largest workgroup-engine instance: {big.summary()}")
    K = 64
    r, sb, sa = _oracle_run(big, K)
    want = r.S_raw * r.scale
    prob = te.Problem(big)
    for threads, ppl in ((256, 1), (256, 8), (512, 2), (1024, 4)):
        x, S, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=te.ENGINE_BLOCK, block_threads=threads,
                                         paths_per_lane=ppl, sched_beta=sb, sched_alpha=sa))
        err = _report(f"LDS-limit instance threads={threads} ppl={ppl}", S.cpu().numpy().astype(np.float64), want,
                      big.demand)
        assert err.max() <= REL
    small = W.ragged(0)
    batch = te.Batch([te.Problem(big), te.Problem(small), te.Problem(big)])
    xb, Sb, stb = batch.solve(te.Options(fixed_iters=K, project=False, block_threads=256, paths_per_lane=8,
                                         sched_beta=sb, sched_alpha=sa))
    Sb = Sb.cpu().numpy().astype(np.float64)
    for off in (0, big.n_demands + small.n_demands):
        assert _rel_err(Sb[off:off + big.n_demands], want, big.demand).max() <= REL
    with pytest.raises(te.TEError):
        te.Problem(over).solve(te.Options(fixed_iters=4, engine=te.ENGINE_BLOCK))
    _, S_over, st_over = te.Problem(over).solve(te.Options(fixed_iters=4))
    assert st_over["engine"] == te.ENGINE_GRAPH


@pytest.mark.parametrize("ppl", [2, 4, 8])
@pytest.mark.parametrize("name", ["waxman20", "ragged0", "waxman150"])
def test_parity_graph_paths_per_lane(te, c1, c2, ppl, name):
    """The graph engine's demand kernel with 2, 4 and 8 paths per lane (lane groups of
    max(1, G / ppl) lanes per demand) against the oracle, schedule replayed; the handle switches
    back to one path per lane afterwards and still matches."""
    inst = {"waxman20": c1, "waxman150": c2}.get(name) or W.ragged(0)
    K = 64 if name == "waxman150" else 256
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    for q in (ppl, 1):
        opts = te.Options(fixed_iters=K, project=False, engine=te.ENGINE_GRAPH, paths_per_lane=q,
                          sched_beta=sb, sched_alpha=sa)
        x, S, st = prob.solve(opts)
        assert st["paths_per_lane"] == q
        err = _report(f"{name} graph ppl={q}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale, inst.demand)
        assert err.max() <= REL


def test_invalid_options_rejected(te, c1):
    prob = te.Problem(c1)
    for bad in (dict(beta0=-1.0), dict(block_threads=128), dict(paths_per_lane=3)):
        with pytest.raises(te.TEError) as ex:
            prob.solve(te.Options(**bad))
        assert ex.value.status == te.TE_ERR_INVALID


def _golden(name):
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)


@pytest.mark.parametrize("which,K", [("tiny", 40), ("waxman20", 256)])
def test_grad_matches_oracle_reverse_pass(te, c1, which, K):
    """te_grad (adjoint kernels, checkpoints every 16 iterations) against the oracle's FP64 reverse
    pass with the same replayed schedule: total throughput (cotangent 1) and sum of logs (1/S)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import torch
    if which == "tiny":
        from test_oracle_pins import _tiny_random
        inst = _tiny_random(0)
    else:
        inst = c1
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    opts = te.Options(fixed_iters=K, project=False, record=True, engine=te.ENGINE_GRAPH, sched_beta=sb,
                      sched_alpha=sa)
    _, S, _ = prob.solve(opts)
    S = S.cpu().numpy().astype(np.float64)
    for wname in ("ones", "inv"):
        w = np.ones(inst.n_demands) if wname == "ones" else 1.0 / np.maximum(np.abs(S), 1e-12)
        dC, dD = prob.grad(torch.tensor(w, dtype=torch.float32))
        dC = dC.cpu().numpy()
        dD = dD.cpu().numpy()
        _, oC, oD = O.grad(inst, sb, sa, w.astype(np.float32).astype(np.float64))
        scale = max(np.abs(oC).max(), np.abs(oD).max())
        eC = np.abs(dC - oC).max() / scale
        eD = np.abs(dD - oD).max() / scale
        print(f"grad {which} K={K} {wname}: max |err| / max |grad|: dC {eC:.2e} dD {eD:.2e}")
        assert eC <= 1e-3 and eD <= 1e-3


def test_gatesolve_autograd(te, c1, torch):
    import torch as t
    GateSolve = te.GateSolve
    prob = te.Problem(c1)
    C = t.tensor(c1.capacity, dtype=t.float64, requires_grad=True)
    D = t.tensor(c1.demand, dtype=t.float64, requires_grad=True)
    S = GateSolve.apply(prob, C, D, 64)
    S.sum().backward()
    assert C.grad.shape == C.shape and D.grad.shape == D.shape
    assert t.isfinite(C.grad).all() and t.isfinite(D.grad).all()


_FIXED = dict(project=False, adapt_beta=False, alpha_target=0.0)


def test_warm_continuation_is_exact(te, c1):
    """Stopping after 30 iterations and continuing with warm = 1 for 50 more gives the rates of one
    uninterrupted 80-iteration run (beta fixed and alpha held at 0, so restarting the control record
    changes no arithmetic)."""
    prob = te.Problem(c1)
    x_ref, _, _ = prob.solve(te.Options(fixed_iters=80, engine=te.ENGINE_GRAPH, **_FIXED))
    prob.solve(te.Options(fixed_iters=30, engine=te.ENGINE_GRAPH, **_FIXED))
    x_w, _, st = prob.solve(te.Options(fixed_iters=50, warm=True, **_FIXED))
    assert st["iters"] == 50 and st["engine"] == te.ENGINE_GRAPH
    np.testing.assert_array_equal(x_w.cpu().numpy(), x_ref.cpu().numpy())


def test_warm_continuation_converts_units(te, c1):
    """te_update doubling every capacity doubles the unit scale; the warm restart converts the state
    to the new units (the same rates in caller units), so 20 further iterations start where the
    previous solve ended: their first-iteration rates stay close to the old ones, and a long warm
    continuation reaches the updated instance's solution."""
    opts = dict(engine=te.ENGINE_GRAPH, project=False, alpha_target=1.0)
    prob = te.Problem(c1)
    x_old, _, _ = prob.solve(te.Options(fixed_iters=20000, **opts))
    prob.update(capacity=2.0 * c1.capacity)
    x1, _, _ = prob.solve(te.Options(fixed_iters=1, warm=True, **opts))
    d1 = np.abs(x1.cpu().numpy() - x_old.cpu().numpy()).max() / c1.capacity.max()
    x_w, S_w, _ = prob.solve(te.Options(fixed_iters=20000, warm=True, **opts))
    ref = te.Problem(c1)
    ref.update(capacity=2.0 * c1.capacity)
    _, S_ref, _ = ref.solve(te.Options(fixed_iters=40000, **opts))
    e = np.abs(S_w.cpu().numpy() - S_ref.cpu().numpy()).max() / c1.demand.max()
    print(f"unit change: first warm iteration moves rates by {d1:.2e} of the capacity scale; "
          f"warm 1+20000 vs cold 40000: {e:.2e} of max D")
    assert d1 < 0.05 and e < 1e-3


def test_warm_restart_after_demand_drift(te, c1):
    """After demands drift by 5 % (lognormal), 100 iterations continued from the previous state land
    much closer to the new proportional-fair solution than 100 iterations from a cold start."""
    opts = dict(engine=te.ENGINE_GRAPH, project=False, alpha_target=1.0)
    prob = te.Problem(c1)
    prob.solve(te.Options(fixed_iters=20000, **opts))
    rng = np.random.default_rng(5)
    dem2 = c1.demand * np.exp(rng.normal(0.0, 0.05, c1.n_demands))
    prob.update(demand=dem2)
    ref = te.Problem(c1)
    ref.update(demand=dem2)
    _, S_ref, _ = ref.solve(te.Options(fixed_iters=60000, **opts))
    S_ref = S_ref.cpu().numpy().astype(np.float64)
    _, S_w, _ = prob.solve(te.Options(fixed_iters=100, warm=True, **opts))
    _, S_c, _ = ref.solve(te.Options(fixed_iters=100, **opts))
    e_w = np.abs(S_w.cpu().numpy() - S_ref).max() / dem2.max()
    e_c = np.abs(S_c.cpu().numpy() - S_ref).max() / dem2.max()
    print(f"demand drift 5%: after 100 iterations, warm {e_w:.3e}, cold {e_c:.3e} (max |dS| / max D)")
    assert e_w < 0.2 * e_c


def test_warm_needs_state(te, c1):
    prob = te.Problem(c1)
    with pytest.raises(te.TEError) as ex:
        prob.solve(te.Options(fixed_iters=10, warm=True))
    assert ex.value.status == te.TE_ERR_STATE
    prob.solve(te.Options(fixed_iters=10, engine=te.ENGINE_GRAPH))
    prob.kernel_times(te.Options(engine=te.ENGINE_GRAPH), iters=4)  # overwrites the state
    with pytest.raises(te.TEError) as ex:
        prob.solve(te.Options(fixed_iters=10, warm=True))
    assert ex.value.status == te.TE_ERR_STATE


def test_anytime_projection(te, c2):
    """te_project on the state a solve left equals the projection te_solve applies at the end, and
    interleaved with warm continuations gives a feasible allocation at every stop."""
    prob = te.Problem(c2)
    opts = dict(engine=te.ENGINE_GRAPH)
    xp, Sp, _ = prob.solve(te.Options(fixed_iters=64, **opts))
    prob.solve(te.Options(fixed_iters=64, project=False, **opts))
    xa, Sa = prob.project()
    np.testing.assert_array_equal(xa.cpu().numpy(), xp.cpu().numpy())
    gold = np.load(_golden("maxmin_waxman150_s0.npz"))["S"]
    scale = float(c2.capacity[np.unique(c2.path_links)].max())
    last = None
    for step in range(4):
        prob.solve(te.Options(fixed_iters=128, project=False, warm=True, **opts))
        x, S = prob.project()
        x = x.cpu().numpy().astype(np.float64)
        assert np.all(x >= 0)
        assert np.all(O.link_loads(c2, x) <= c2.capacity * (1 + 1e-7))
        assert np.all(O.demand_sums(c2, x) <= c2.demand * (1 + 1e-7))
        opt = O.optimality(S.cpu().numpy().astype(np.float64), gold, 1e-9 * scale)
        print(f"anytime: {64 + 128 * (step + 1)} iterations, optimality {opt:.4f}")
        last = opt
    assert last > 0.9


@pytest.mark.parametrize("engine", ["block", "graph"])
@pytest.mark.parametrize("K", [1, 2, 16, 256])
def test_parity_fixed_beta_fixed_alpha(te, c1, engine, K):
    """beta held at beta0 and alpha held at 0 (no adaptation at all): the plain iteration."""
    o = dict(fixed_iters=K, project=False, adapt_beta=False, alpha_target=0.0)
    r = O.solve(c1, O.Options(**o), want_state=False)
    sb, sa = r.schedule
    assert np.all(sb == 1.0) and np.all(sa == 0.0)
    prob = te.Problem(c1)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    x, S, st = prob.solve(te.Options(engine=eng, **o))
    err = _report(f"waxman20 fixed beta/alpha {engine} K={K}", S.cpu().numpy().astype(np.float64),
                  r.S_raw * r.scale, c1.demand)
    assert err.max() <= REL


def test_failure_scenarios_reach_maxmin(te):
    """The batched solve of the first 64 failure scenarios: every scenario within 1 % of its exact
    max-min allocation (progressive-filling LPs, tests/golden) after 1,000 iterations."""
    g = np.load(_golden("maxmin_failures_s0.npz"))
    scen = W.failure_scenarios(0, n_scen=64)
    batch = te.Batch([te.Problem(s) for s in scen])
    _, S, _ = batch.solve(te.Options(fixed_iters=1000))
    S = S.cpu().numpy().astype(np.float64)
    off = 0
    worst = 1.0
    for i, inst in enumerate(scen):
        assert str(g[f"fp{i}"]) == inst.fingerprint()
        opt = O.optimality(S[off:off + inst.n_demands], g[f"S{i}"], 1e-9 * 100.0)
        worst = min(worst, opt)
        off += inst.n_demands
    print(f"64 failure scenarios, 1000 iterations: worst optimality {worst:.5f}")
    assert worst >= 0.99


def test_gatesolve_matches_oracle_reverse_pass(te, c1, torch):
    """torch.autograd through GateSolve (te_update + recorded te_solve + te_grad) gives the FP64
    reverse pass of the oracle for a weighted sum of the sums, with the oracle's schedule replayed."""
    import torch as t
    K = 64
    r, sb, sa = _oracle_run(c1, K)
    prob = te.Problem(c1)
    C = t.tensor(c1.capacity, dtype=t.float64, requires_grad=True)
    D = t.tensor(c1.demand, dtype=t.float64, requires_grad=True)
    w = np.random.default_rng(4).uniform(0.5, 1.5, c1.n_demands)
    S = te.GateSolve.apply(prob, C, D, K, te.Options(engine=te.ENGINE_GRAPH, sched_beta=sb, sched_alpha=sa))
    (S.double().cpu() * t.tensor(w)).sum().backward()
    _, oC, oD = O.grad(c1, sb, sa, w.astype(np.float32).astype(np.float64))
    scale = max(np.abs(oC).max(), np.abs(oD).max())
    eC = np.abs(C.grad.numpy() - oC).max() / scale
    eD = np.abs(D.grad.numpy() - oD).max() / scale
    print(f"GateSolve K={K}: max |err| / max |grad|: dC {eC:.2e} dD {eD:.2e}")
    assert eC <= 1e-3 and eD <= 1e-3
