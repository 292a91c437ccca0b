"""te_project_rates_static (the entry point that allocates nothing) against te_project_rates, through
the C ABI: two calls in a row on one GPU, the second on a smaller instance, so the second runs on
the static scratch the first left behind."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def te():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_01748_amd as te_mod
    te_mod.library()
    return te_mod


def _rates(te, inst, K):
    prob = te.Problem(inst)
    x, _, st = prob.solve(te.Options(fixed_iters=K, project=False, engine=te.ENGINE_GRAPH))
    # drifted demands and a degraded link: the projection has work to do on both phases
    cap = inst.capacity.copy()
    cap[np.argmax(O.link_loads(inst, x.cpu().numpy()))] *= 0.5
    prob.update(capacity=cap, demand=inst.demand * 0.9)
    return prob, x, st["final_alpha"]


def test_static_scratch_matches_handle_scratch(te):
    big, small = W.waxman150(0), W.waxman20(0)
    for inst, K in ((big, 64), (small, 40)):  # the second call is the smaller input
        prob, x, alpha = _rates(te, inst, K)
        xs, Ss = prob.project_rates(x, alpha, static_scratch=True)
        xh, Sh = prob.project_rates(x, alpha)
        np.testing.assert_array_equal(xs.cpu().numpy(), xh.cpu().numpy())
        np.testing.assert_array_equal(Ss.cpu().numpy(), Sh.cpu().numpy())
        xp = xs.cpu().numpy().astype(np.float64)
        assert np.all(xp >= 0)
        assert np.all(O.demand_sums(inst, xp) <= inst.demand * 0.9 * (1 + 1e-7))
        print(f"{inst.name}: static-scratch projection equals the handle's ({inst.n_paths} paths)")


def test_static_scratch_refuses_oversized_instance(te):
    """An instance whose projection needs more than the 32 MiB static array is refused, with nothing
    launched."""
    inst = W.shared_link(np.ones(1_100_000))  # 1.1M single-path demands on one link
    prob = te.Problem(inst)
    need = 24 * inst.n_paths + 8 * inst.n_demands + 8 * inst.n_links
    assert need > 32 << 20
    x = np.ones(inst.n_paths, np.float32)
    with pytest.raises(te.TEError) as ex:
        prob.project_rates(x, 1.0, static_scratch=True)
    assert ex.value.status == te.TE_ERR_INVALID and "static" in str(ex.value)
