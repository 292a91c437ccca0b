"""The disjoint union of instances, each in its own normalised units, is what the batched graph
engine solves: under one (beta, alpha) schedule every instance iterates exactly as alone (they
share no link or demand), and the union's max-min optimum is the union of the instances' optima."""
import numpy as np

import oracle as O
import workloads as W


def union_normalised(insts):
    """(union instance, per-instance unit scales): capacities and demands of each instance divided by
    its own unit scale (the largest capacity of a used link), ids offset."""
    scales = [O.used_scale(i) for i in insts]
    cap, dem, pp, pl, dp, ls, ld, ds, dd = [], [], [0], [], [0], [], [], [], []
    offE = offP = offN = 0
    for inst, s in zip(insts, scales):
        cap.append(inst.capacity / s)
        dem.append(inst.demand / s)
        pp.extend((np.asarray(inst.path_ptr[1:]) + pp[-1]).tolist())
        pl.append(np.asarray(inst.path_links) + offE)
        dp.extend((np.asarray(inst.demand_path_ptr[1:]) + offP).tolist())
        ls.append(np.asarray(inst.link_src) + offN)
        ld.append(np.asarray(inst.link_dst) + offN)
        ds.append(np.asarray(inst.demand_src) + offN)
        dd.append(np.asarray(inst.demand_dst) + offN)
        offE += inst.n_links
        offP += inst.n_paths
        offN += inst.n_nodes
    u = W.Instance(name="union", n_nodes=offN, link_src=np.concatenate(ls).astype(np.int32),
                   link_dst=np.concatenate(ld).astype(np.int32), capacity=np.concatenate(cap),
                   demand_src=np.concatenate(ds).astype(np.int32), demand_dst=np.concatenate(dd).astype(np.int32),
                   demand=np.concatenate(dem), path_ptr=np.asarray(pp, np.int64),
                   path_links=np.concatenate(pl).astype(np.int32), demand_path_ptr=np.asarray(dp, np.int32),
                   meta={})
    return u, scales


def test_union_iterates_as_its_members():
    insts = W.failure_scenarios(0, n_scen=3) + [W.waxman20(0)]
    u, scales = union_normalised(insts)
    assert O.used_scale(u) == 1.0
    K = 150
    r = O.solve(u, O.Options(fixed_iters=K, project=False), want_state=False)
    sb, sa = r.schedule
    offD = 0
    for inst, s in zip(insts, scales):
        ri = O.solve(inst, O.Options(fixed_iters=K, project=False, sched_beta=sb, sched_alpha=sa), want_state=False)
        Su = r.S_raw[offD:offD + inst.n_demands] * s
        np.testing.assert_allclose(ri.S_raw * ri.scale, Su, rtol=1e-11, atol=1e-13 * s)
        offD += inst.n_demands


def test_union_maxmin_is_union_of_maxmins():
    insts = W.failure_scenarios(1, n_scen=2)
    u, scales = union_normalised(insts)
    opt_u, _ = O.maxmin_exact(u)
    offD = 0
    for inst, s in zip(insts, scales):
        opt_i, _ = O.maxmin_exact(inst)
        np.testing.assert_allclose(opt_u[offD:offD + inst.n_demands] * s, opt_i, rtol=1e-6, atol=1e-7 * s)
        offD += inst.n_demands
