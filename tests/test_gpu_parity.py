"""GPU parity of the HIP path (through the C ABI) with the FP64 oracle.

Parity is taken at equal iteration counts with the oracle's (beta, alpha) schedule replayed on
the GPU (the adaptive control itself is compared with the oracle's trace separately).  The bar is
on the per-demand sums S_c before projection, relative for every demand:
    |S_gpu - S_oracle| <= 1e-4 * max(|S_oracle|, 1e-12 * max_c D_c)
(the floor only guards sums at FP64 noise level).  The GPU's output S is FP32, whose rounding
(6e-8 relative) is far inside the bar.  The projection (Algorithm 2) is checked for feasibility
and against the oracle's Algorithm 2 on the GPU's own unprojected rates, order-tolerant among
trim scores that FP32 does not resolve (tests/projcheck.py).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from projcheck import check_projection

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
    return np.abs(S_gpu - S_orc) / np.maximum(np.abs(S_orc), 1e-12 * dem.max())


def _report(tag, S_gpu, S_orc, dem):
    err = _rel_err(S_gpu, S_orc, dem)
    absn = np.abs(S_gpu - S_orc).max() / dem.max()
    print(f"{tag}: per-demand relative error max {err.max():.3e}, p99 {np.quantile(err, 0.99):.3e}, "
          f"median {np.median(err):.3e}, over 1e-5: {int((err > 1e-5).sum())} of {err.size}; "
          f"max |dS|/max D {absn:.3e}")
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
    x64 = prob.state()[0].cpu().numpy()  # the FP64 rates the projection started from
    xp = xp.cpu().numpy().astype(np.float64)
    assert np.all(xp >= 0)
    assert np.all(O.link_loads(inst, xp) <= inst.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(inst, xp) <= inst.demand * (1 + 1e-7))
    check_projection(inst, x64, xp, stp["final_alpha"], tag="hierarchical 1000-node", per_demand=True)


@pytest.mark.parametrize("K", [16, 128])
def test_parity_hierarchical_graph(te, c3_small, K):
    r, sb, sa = _oracle_run(c3_small, K)
    prob = te.Problem(c3_small)
    x, S, st = _gpu_raw(te, prob, K, sb, sa, te.ENGINE_GRAPH)
    assert st["iters"] == K
    err = _report(f"hierarchical graph K={K} ({st['ms']:.3f} ms)", S, r.S_raw * r.scale, c3_small.demand)
    assert err.max() <= REL


def _ragged_long():
    # paths of up to 24 links: beyond the fixed-width hop records, so every kernel reads the CSR layout
    return W.ragged(3, n_links=60, n_demands=50, max_hops=24)


_EDGE = {
    "ragged0": lambda: W.ragged(0),
    "ragged_long": _ragged_long,
    "ragged1": lambda: W.ragged(1, n_links=20, n_demands=70),
    "one_link_one_demand": lambda: W.shared_link([5.0], cap=1.0),
    "shared_link": lambda: W.shared_link([0.1, 0.5, 2.0, 8.0], cap=1.0),
    "parallel_64": lambda: W.parallel_paths(np.linspace(0.5, 2.0, 64), 50.0),
}


@pytest.mark.parametrize("engine", ["block", "graph"])
@pytest.mark.parametrize("K", [1, 64])
@pytest.mark.parametrize("name", sorted(_EDGE))
def test_parity_edge_cases(te, name, engine, K):
    """Ragged path counts (1..64 per demand), paths longer than the gather batch and than a hop
    record, unused links, a single link and a single demand, and the widest demand (64 paths on one
    link each)."""
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
    check_projection(c1, xr, xp, st["final_alpha"], tag=f"waxman20 {engine}")


def test_projection_waxman150_graph(te, c2):
    K = 64
    prob = te.Problem(c2)
    r, sb, sa = _oracle_run(c2, K)
    opts = dict(fixed_iters=K, engine=te.ENGINE_GRAPH, sched_beta=sb, sched_alpha=sa)
    xp, Sp, st = prob.solve(te.Options(project=True, **opts))
    xr = prob.state()[0].cpu().numpy()  # the FP64 rates the projection started from
    xp = xp.cpu().numpy().astype(np.float64)
    L = O.link_loads(c2, xp)
    assert np.all(xp >= 0)
    assert np.all(L <= c2.capacity * (1 + 1e-7))
    assert np.all(O.demand_sums(c2, xp) <= c2.demand * (1 + 1e-7))
    check_projection(c2, xr, xp, st["final_alpha"], tag="waxman150")


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


def test_single_solve_tuned_workgroup_size(te, c1):
    """A single workgroup-engine solve with block_threads = paths_per_lane = 0 tunes the pair on the
    handle's first such solve, keeps it, and equals the forced solve with that pair."""
    prob = te.Problem(c1)
    o = te.Options(fixed_iters=64, engine=te.ENGINE_BLOCK)
    x1, _, st1 = prob.solve(o)
    t, q = st1["block_threads"], st1["paths_per_lane"]
    assert t in (256, 512, 1024) and q in (1, 2, 4, 8) and st1["engine"] == te.ENGINE_BLOCK
    x2, _, st2 = prob.solve(o)
    assert (st2["block_threads"], st2["paths_per_lane"]) == (t, q)
    np.testing.assert_array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    x3, _, _ = prob.solve(te.Options(fixed_iters=64, engine=te.ENGINE_BLOCK, block_threads=t, paths_per_lane=q))
    np.testing.assert_array_equal(x1.cpu().numpy(), x3.cpu().numpy())
    _, _, st4 = prob.solve(te.Options(fixed_iters=64, engine=te.ENGINE_BLOCK, block_threads=256))
    assert st4["block_threads"] == 256 and st4["paths_per_lane"] in (1, 2, 4, 8)
    print(f"tuned for the 20-node instance: {t} threads, {q} paths per lane")


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
@pytest.mark.parametrize("name", ["waxman20", "ragged0", "ragged_long", "waxman150"])
def test_parity_graph_paths_per_lane(te, c1, c2, ppl, name):
    """The graph engine's demand kernel with 2, 4 and 8 paths per lane (lane groups of
    max(1, G / ppl) lanes per demand) against the oracle, schedule replayed; the handle switches
    back to one path per lane afterwards and still matches."""
    inst = {"waxman20": c1, "waxman150": c2, "ragged_long": None}.get(name) or (
        _ragged_long() if name == "ragged_long" else W.ragged(0))
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
    for bad in (dict(beta0=-1.0), dict(block_threads=128), dict(paths_per_lane=3), dict(link_sums=4)):
        with pytest.raises(te.TEError) as ex:
            prob.solve(te.Options(**bad))
        assert ex.value.status == te.TE_ERR_INVALID


def _grad_err(g, ref):
    """Per-component relative error of a gradient, floored at 1e-6 (caller units)."""
    return np.abs(np.asarray(g) - ref) / np.maximum(np.abs(ref), 1e-6)


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
        eC, eD = _grad_err(dC, oC), _grad_err(dD, oD)
        print(f"grad {which} K={K} {wname}: per-component relative error (floor 1e-6): dC {eC.max():.2e} "
              f"dD {eD.max():.2e}")
        assert eC.max() <= 1e-3 and eD.max() <= 1e-3


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
    eC, eD = _grad_err(C.grad.numpy(), oC), _grad_err(D.grad.numpy(), oD)
    print(f"GateSolve K={K}: per-component relative error (floor 1e-6): dC {eC.max():.2e} dD {eD.max():.2e}")
    assert eC.max() <= 1e-3 and eD.max() <= 1e-3


def _first_divergence(gb, ga, ob, oa):
    n = min(len(gb), len(ob))
    bad = np.nonzero((gb[:n] != ob[:n]) | (ga[:n] != oa[:n]))[0]
    return int(bad[0]) if bad.size else n


@pytest.mark.parametrize("name,engine,K", [("waxman20", "block", 833), ("waxman20", "graph", 833),
                                           ("waxman150", "graph", 833), ("parking2", "block", 400),
                                           ("parking2", "graph", 400), ("parking3", "graph", 400)])
def test_adaptive_control_matches_oracle_trace(te, c1, c2, name, engine, K):
    """The GPU's own control (no replay): its sequence of (beta_k, alpha_k) equals the oracle's, and its
    residuals r_k, s_k (section 3.4) agree with the oracle's to 1e-6 relative, over K iterations of
    the max-min solve.  The schedules may only part where the oracle's decision was a near-tie
    (r within 1e-6 of A s or s of A r, or a residual within 1e-6 of gamma).  On the parking lots the
    balancing rule reverses six times in 400 iterations, so its back-off is exercised."""
    inst = {"waxman20": c1, "waxman150": c2}.get(name) or W.parking_lot(int(name[-1]))
    r = O.solve(inst, O.Options(fixed_iters=K, project=False), want_state=False)
    ot = r.trace
    prob = te.Problem(inst)
    eng = te.ENGINE_BLOCK if engine == "block" else te.ENGINE_GRAPH
    _, S, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=eng, trace=True))
    gt = prob.trace(K)
    assert gt.shape == (K, 4) and st["iters"] == K
    n = _first_divergence(gt[:, 0], gt[:, 1], ot[:, 1], ot[:, 0])
    if n < K:
        k = n - 1  # the decision after iteration k set iteration n's (beta, alpha)
        rr, ss = ot[k, 2], ot[k, 3]
        margin = min(abs(rr - 10 * ss) / max(rr, 1e-300), abs(ss - 10 * rr) / max(ss, 1e-300),
                     abs(rr - 1e-3) / 1e-3, abs(ss - 1e-3) / 1e-3)
        print(f"{name} {engine}: schedules part at iteration {n} (decision margin {margin:.2e})")
        assert margin <= 1e-6
    er = np.abs(gt[:n, 2] - ot[:n, 2]) / np.maximum(np.abs(ot[:n, 2]), 1e-12)
    es = np.abs(gt[:n, 3] - ot[:n, 3]) / np.maximum(np.abs(ot[:n, 3]), 1e-12)
    changes = int((np.diff(ot[:n, 1]) != 0).sum())
    print(f"{name} {engine}: {n} iterations with equal schedules ({changes} beta changes, final alpha "
          f"{ot[n - 1, 0]:g}); residual relative error max r {er.max():.2e}, s {es.max():.2e}")
    assert er.max() <= 1e-6 and es.max() <= 1e-6
    if n == K:
        assert st["final_alpha"] == r.final_alpha and st["beta"] == r.beta
        _report(f"{name} {engine} adaptive K={K}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                inst.demand)


def _drifted(inst, seed, cap_mult=1.0):
    rng = np.random.default_rng(seed)
    return inst.capacity * cap_mult, inst.demand * np.exp(rng.normal(0.0, 0.05, inst.n_demands))


@pytest.mark.parametrize("case", ["same_beta", "other_beta", "unit_change"])
def test_warm_restart_matches_oracle(te, c1, case):
    """warm = 1 after te_update against the oracle continuing from its own iterate (Algorithm 1's
    optional inputs x^0 and beta, extended to every dual): 120 iterations, demands drifted by 5 %,
    then 80 more.  other_beta replays a second schedule starting at twice the penalty (both sides
    divide the scaled duals by 2); unit_change also doubles every capacity (new unit scale)."""
    K1, K2 = 120, 80
    r1 = O.solve(c1, O.Options(fixed_iters=K1, project=False, alpha_target=1.0))
    sb1, sa1 = r1.schedule
    cap2, dem2 = _drifted(c1, 7, 2.0 if case == "unit_change" else 1.0)
    inst2 = W.make_instance("c1w", c1.n_nodes, c1.link_src, c1.link_dst, cap2, c1.demand_src, c1.demand_dst, dem2,
                            [[c1.path_links[c1.path_ptr[q]:c1.path_ptr[q + 1]].tolist()
                              for q in range(c1.demand_path_ptr[c], c1.demand_path_ptr[c + 1])]
                             for c in range(c1.n_demands)])
    ws = r1.warm_state()
    if case == "other_beta":
        r2a = O.solve(inst2, O.Options(fixed_iters=K2, project=False, alpha_target=1.0), warm=ws,
                      want_state=False)
        sb2, sa2 = 2.0 * r2a.schedule[0], r2a.schedule[1]
        r2 = O.solve(inst2, O.Options(fixed_iters=K2, project=False, sched_beta=sb2, sched_alpha=sa2), warm=ws,
                     want_state=False)
    else:
        r2 = O.solve(inst2, O.Options(fixed_iters=K2, project=False, alpha_target=1.0), warm=ws, want_state=False)
        sb2, sa2 = r2.schedule
    prob = te.Problem(c1)
    _, S1, _ = prob.solve(te.Options(fixed_iters=K1, project=False, engine=te.ENGINE_GRAPH, sched_beta=sb1,
                                     sched_alpha=sa1))
    err1 = _report(f"warm {case}: first solve K={K1}", S1.cpu().numpy().astype(np.float64), r1.S_raw * r1.scale,
                   c1.demand)
    assert err1.max() <= REL
    prob.update(capacity=cap2, demand=dem2)
    _, S2, st2 = prob.solve(te.Options(fixed_iters=K2, project=False, warm=True, sched_beta=sb2, sched_alpha=sa2))
    assert st2["iters"] == K2
    err2 = _report(f"warm {case}: continuation K={K2}", S2.cpu().numpy().astype(np.float64), r2.S_raw * r2.scale,
                   dem2)
    assert err2.max() <= REL


def test_update_discards_recording(te, c1, torch):
    """te_update invalidates the recorded trajectory: te_grad then refuses, and the recording
    generation changes with every recorded solve and every update."""
    prob = te.Problem(c1)
    assert prob.info()["record_gen"] == 0
    prob.solve(te.Options(fixed_iters=32, record=True, project=False))
    g1 = prob.info()["record_gen"]
    assert g1 > 0
    prob.grad(torch.ones(c1.n_demands))
    prob.update(demand=c1.demand * 1.01)
    assert prob.info()["record_gen"] == 0
    with pytest.raises(te.TEError) as ex:
        prob.grad(torch.ones(c1.n_demands))
    assert ex.value.status == te.TE_ERR_STATE
    prob.solve(te.Options(fixed_iters=32, record=True, project=False))
    assert prob.info()["record_gen"] not in (0, g1)


def test_gatesolve_second_forward_invalidates_first(te, c1, torch):
    """Two GateSolve forwards on one Problem: the first output's backward refuses (the handle's
    recording is the second forward's), the second's backward works."""
    import torch as t
    prob = te.Problem(c1)
    C = t.tensor(c1.capacity, dtype=t.float64, requires_grad=True)
    D1 = t.tensor(c1.demand, dtype=t.float64, requires_grad=True)
    D2 = t.tensor(c1.demand * 1.1, dtype=t.float64, requires_grad=True)
    S1 = te.GateSolve.apply(prob, C, D1, 32)
    S2 = te.GateSolve.apply(prob, C, D2, 32)
    with pytest.raises(RuntimeError, match="solved again"):
        S1.sum().backward()
    S2.sum().backward()
    assert t.isfinite(D2.grad).all()


_LSUM_CASES = {
    "waxman20": lambda: W.waxman20(0),
    "ragged0": lambda: W.ragged(0),
    "ragged1": lambda: W.ragged(1, n_links=20, n_demands=70),
    "ragged_long": _ragged_long,
    "parallel_64": lambda: W.parallel_paths(np.linspace(0.5, 2.0, 64), 50.0),
    "waxman150": lambda: W.waxman150(0),
    "two_level_6": lambda: W.two_level1000(1, regions=6, backbone_links=120),
}


@pytest.mark.parametrize("ppl", [0, 2])
@pytest.mark.parametrize("lsum", ["private", "private_atomic", "csc"])
@pytest.mark.parametrize("name", sorted(_LSUM_CASES))
def test_parity_link_sum_variants(te, name, lsum, ppl):
    """The ways of forming the link loads (privatised LDS rows reduced per link, summed by link lists
    or by one atomic addition per incidence, or segmented sums over the link -> path list) against the
    oracle, schedule replayed, on instances with 1 to 64 paths per demand and hop-record or CSR path
    layouts; the handle switches between them; one and two paths per lane."""
    inst = _LSUM_CASES[name]()
    K = 64
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    want = {"private": te.LINK_SUMS_PRIVATE, "private_atomic": te.LINK_SUMS_PRIVATE_ATOMIC,
            "csc": te.LINK_SUMS_CSC}[lsum]
    other = te.LINK_SUMS_CSC if lsum != "csc" else te.LINK_SUMS_PRIVATE
    for ls in (want, other, want):
        x, S, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=te.ENGINE_GRAPH, link_sums=ls,
                                         paths_per_lane=ppl, sched_beta=sb, sched_alpha=sa))
        info = prob.info()
        assert info["link_sums"] == ls
        assert (info["hop_slots"] == 0) == (name == "ragged_long")
        assert (info["scatter_workgroups"] > 0) == (ls != te.LINK_SUMS_CSC)
        assert (info["list_passes"] > 0) == (ls == te.LINK_SUMS_PRIVATE)
        assert (info["list_entries"] >= inst.nnz) == (ls == te.LINK_SUMS_PRIVATE)
        err = _report(f"{name} link sums {ls} K={K}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                      inst.demand)
        assert err.max() <= REL


@pytest.mark.parametrize("ppl", [4, 8])
@pytest.mark.parametrize("lsum", ["private", "private_atomic"])
@pytest.mark.parametrize("name", ["ragged0", "parallel_64", "two_level_6"])
def test_parity_private_sums_many_paths_per_lane(te, name, lsum, ppl):
    """The privatised sums' kernels with four and eight paths per lane (link lists and atomic adds)
    against the oracle, schedule replayed."""
    inst = _LSUM_CASES[name]()
    K = 32
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    ls = te.LINK_SUMS_PRIVATE if lsum == "private" else te.LINK_SUMS_PRIVATE_ATOMIC
    x, S, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=te.ENGINE_GRAPH, link_sums=ls,
                                     paths_per_lane=ppl, sched_beta=sb, sched_alpha=sa))
    assert st["paths_per_lane"] == ppl
    assert (prob.info()["list_passes"] > 0) == (lsum == "private")
    err = _report(f"{name} link sums {ls} ppl {ppl} K={K}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                  inst.demand)
    assert err.max() <= REL


def test_link_sums_limit(te):
    """More links than one workgroup's LDS holds: the automatic choice is the CSC sums, and asking for
    privatised sums is refused."""
    inst = W.ragged(2, n_links=20000, n_demands=60)
    prob = te.Problem(inst)
    r, sb, sa = _oracle_run(inst, 16)
    x, S, st = prob.solve(te.Options(fixed_iters=16, project=False, engine=te.ENGINE_GRAPH, sched_beta=sb,
                                     sched_alpha=sa))
    assert prob.info()["link_sums"] == te.LINK_SUMS_CSC
    assert _rel_err(S.cpu().numpy().astype(np.float64), r.S_raw * r.scale, inst.demand).max() <= REL
    with pytest.raises(te.TEError) as ex:
        prob.solve(te.Options(fixed_iters=4, engine=te.ENGINE_GRAPH, link_sums=te.LINK_SUMS_PRIVATE))
    assert ex.value.status == te.TE_ERR_INVALID


@pytest.mark.parametrize("n_links,lists", [(17000, True), (19400, False)])
def test_link_lists_need_room_beside_the_loads(te, n_links, lists):
    """Privatised sums keep a chunk of rates in LDS beside the E loads: with 17,000 links a pass of
    rates still fits and the link lists are used; with 19,400 it does not, and the same option adds one
    incidence at a time. Both against the oracle, schedule replayed."""
    inst = W.ragged(3, n_links=n_links, n_demands=60)
    prob = te.Problem(inst)
    r, sb, sa = _oracle_run(inst, 16)
    x, S, st = prob.solve(te.Options(fixed_iters=16, project=False, engine=te.ENGINE_GRAPH,
                                     link_sums=te.LINK_SUMS_PRIVATE, sched_beta=sb, sched_alpha=sa))
    info = prob.info()
    assert info["link_sums"] == te.LINK_SUMS_PRIVATE and info["scatter_workgroups"] > 0
    assert (info["list_passes"] > 0) == lists
    err = _report(f"ragged E={n_links} private link sums", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                  inst.demand)
    assert err.max() <= REL


def test_link_lists_in_uneven_chunks(te, torch):
    """600,000 one-path demands over 17,000 links: passes of 1,024 demands, three a scatter workgroup
    (256 compute units), of which two fit beside the loads, so a workgroup sums its lists after passes
    2 and 3 (chunks of two and one) and the last workgroup has a single pass. Against the oracle,
    schedule replayed."""
    inst = W.single_paths(0)
    K = 8
    r, sb, sa = _oracle_run(inst, K)
    prob = te.Problem(inst)
    x, S, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=te.ENGINE_GRAPH,
                                     link_sums=te.LINK_SUMS_PRIVATE, sched_beta=sb, sched_alpha=sa))
    info = prob.info()
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    npass = -(-inst.n_demands // 1024)
    spw = -(-npass // ncu)
    print(f"compute units {ncu}, passes {npass}, {spw} a workgroup, {info['list_passes']} a chunk")
    assert info["scatter_workgroups"] == -(-npass // spw)
    assert 1 <= info["list_passes"] <= spw and info["list_entries"] >= inst.nnz
    if ncu == 256:
        assert spw == 3 and info["list_passes"] == 2
    err = _report("single paths private link sums", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale,
                  inst.demand)
    assert err.max() <= REL


def test_state_is_the_fp64_iterate(te, c1):
    """te_get_state returns the FP64 rates of the last graph-engine solve: their FP32 rounding is the
    unprojected output, and their per-demand sums are the output sums."""
    prob = te.Problem(c1)
    x, S, _ = prob.solve(te.Options(fixed_iters=40, project=False, engine=te.ENGINE_GRAPH))
    x64, S64 = prob.state()
    np.testing.assert_array_equal(x64.cpu().numpy().astype(np.float32), x.cpu().numpy())
    np.testing.assert_array_equal(S64.cpu().numpy().astype(np.float32), S.cpu().numpy())
    np.testing.assert_allclose(S64.cpu().numpy(), O.demand_sums(c1, x64.cpu().numpy()), rtol=1e-12)


@pytest.mark.parametrize("name,K", [("waxman20", 400), ("ragged0", 200), ("waxman150", 300)])
def test_per_link_penalties_match_oracle(te, name, K):
    """Per-link adaptive penalties (beta * w_e, w_e moved by the residual-balancing rule on link e's own
    residuals): the GPU's own control against the oracle's -- the same (beta_k, alpha_k) sequence, the
    same final per-link factors, and the per-demand sums to the parity bar."""
    inst = {"waxman20": lambda: W.waxman20(0), "ragged0": lambda: W.ragged(0),
            "waxman150": lambda: W.waxman150(0)}[name]()
    r = O.solve(inst, O.Options(fixed_iters=K, project=False, per_link=True))
    assert np.any(r.w != 1.0)
    prob = te.Problem(inst)
    _, S, st = prob.solve(te.Options(fixed_iters=K, project=False, per_link=True, trace=True))
    assert st["engine"] == te.ENGINE_GRAPH and prob.info()["link_sums"] == te.LINK_SUMS_CSC
    gt = prob.trace(K)
    n = _first_divergence(gt[:, 0], gt[:, 1], r.trace[:, 1], r.trace[:, 0])
    assert n == K, f"schedules part at iteration {n}"
    _, _, w = prob.state(with_w=True)
    w = w.cpu().numpy()
    print(f"{name} per-link K={K}: factors {dict(zip(*np.unique(w, return_counts=True)))}; "
          f"{int((w != r.w).sum())} of {w.size} differ from the oracle's")
    np.testing.assert_array_equal(w, r.w)
    err = _report(f"{name} per-link K={K}", S.cpu().numpy().astype(np.float64), r.S_raw * r.scale, inst.demand)
    assert err.max() <= REL


def test_per_link_refused_where_unsupported(te, c1):
    prob = te.Problem(c1)
    for bad in (dict(engine=te.ENGINE_BLOCK), dict(record=True, fixed_iters=8),
                dict(link_sums=te.LINK_SUMS_PRIVATE), dict(link_sums=te.LINK_SUMS_PRIVATE_ATOMIC),
                dict(w_min=2.0)):
        with pytest.raises(te.TEError) as ex:
            prob.solve(te.Options(per_link=True, **{"fixed_iters": 8, **bad}))
        assert ex.value.status == te.TE_ERR_INVALID


def test_mixed_batch_runs_as_union_on_graph_engine(te):
    """A batch of 20-node failure scenarios and the 150-node instance (too large for one workgroup):
    one graph-engine solve of the instances' disjoint union, each instance in its own units.  Each
    instance's sums equal the oracle's solve of the same union (per-demand bar), its projected rates
    are feasible, and the workgroup engine refuses the batch."""
    from test_oracle_union import union_normalised
    small = W.failure_scenarios(0, n_scen=5)
    insts = small[:2] + [W.waxman150(0)] + small[2:]
    batch = te.Batch([te.Problem(i) for i in insts])
    K = 200
    _, S, st = batch.solve(te.Options(fixed_iters=K, project=False))
    assert all(s["engine"] == te.ENGINE_GRAPH and s["iters"] == K for s in st)
    S = S.cpu().numpy().astype(np.float64)
    u, scales = union_normalised(insts)
    r = O.solve(u, O.Options(fixed_iters=K, project=False), want_state=False)
    off = 0
    for inst, s in zip(insts, scales):
        err = _report(f"union member {inst.name}", S[off:off + inst.n_demands],
                      r.S_raw[off:off + inst.n_demands] * s, inst.demand)
        assert err.max() <= REL
        off += inst.n_demands
    xp, Sp, _ = batch.solve(te.Options(fixed_iters=K))
    xp = xp.cpu().numpy().astype(np.float64)
    offP = 0
    for inst in insts:
        xi = xp[offP:offP + inst.n_paths]
        assert np.all(xi >= 0)
        assert np.all(O.link_loads(inst, xi) <= inst.capacity * (1 + 1e-7))
        assert np.all(O.demand_sums(inst, xi) <= inst.demand * (1 + 1e-7))
        offP += inst.n_paths
    with pytest.raises(te.TEError) as ex:
        batch.solve(te.Options(fixed_iters=8, engine=te.ENGINE_BLOCK))
    assert ex.value.status == te.TE_ERR_INVALID


def test_small_batch_on_graph_engine_reaches_maxmin(te):
    """The failure scenarios forced onto the graph engine's union: every scenario within 1 % of its own
    exact max-min allocation (tests/golden), like the workgroup engine's batch."""
    g = np.load(_golden("maxmin_failures_s0.npz"))
    scen = W.failure_scenarios(0, n_scen=32)
    batch = te.Batch([te.Problem(s) for s in scen])
    _, S, st = batch.solve(te.Options(fixed_iters=1000, engine=te.ENGINE_GRAPH))
    assert st[0]["engine"] == te.ENGINE_GRAPH
    S = S.cpu().numpy().astype(np.float64)
    off, worst = 0, 1.0
    for i, inst in enumerate(scen):
        assert str(g[f"fp{i}"]) == inst.fingerprint()
        worst = min(worst, O.optimality(S[off:off + inst.n_demands], g[f"S{i}"], 1e-9 * 100.0))
        off += inst.n_demands
    print(f"32 failure scenarios as one union, 1000 iterations: worst optimality {worst:.5f}")
    assert worst >= 0.99
