"""The allocation-free entry point amf_solve_static against amf_solve + amf_combine of the same
plans bound to caller-owned workspaces: two calls in a row, the second with a smaller plan (the
static workspace keeps the first call's contents), FP64 and FP32, plus the size limit."""
import numpy as np
import pytest
import torch

from paper_2408_00559_amd import _lib as L
from paper_2408_00559_amd import inputs as I
from paper_2408_00559_amd.solver import Plan, StaticPlan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bound_prices(probs, grid, steps, precision, richardson=False):
    plan = Plan(probs, grid, steps, precision=precision, richardson=richardson, device=DEV)
    out = plan.price().cpu().numpy()
    del plan
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_static_solve_matches_bound_solve(precision, tol):
    big = (I.draw_instances(3, seed=201, d=4), I.combination(5, 1), 12, False)
    small = (I.draw_instances(1, seed=202, d=3), I.combination(4, 1), 8, True)
    outs = []
    for probs, grid, steps, rich in (big, small):
        sp = StaticPlan(probs, grid, steps, precision=precision, richardson=rich)
        out = torch.full((len(probs),), float("nan"), dtype=torch.float64, device=DEV)
        got = sp.price(out).cpu().numpy()
        ref = _bound_prices(probs, grid, steps, precision, rich)
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref) / np.abs(ref)) < tol, (got, ref)
        assert np.array_equal(got, ref)            # same kernels, same schedule: the same bits
        outs.append(got)
    # the first plan again, after the smaller one overwrote the front of the workspace
    probs, grid, steps, rich = big
    sp = StaticPlan(probs, grid, steps, precision=precision, richardson=rich)
    again = sp.price(torch.empty(len(probs), dtype=torch.float64, device=DEV)).cpu().numpy()
    assert np.array_equal(again, outs[0])


def test_static_solve_leaves_a_bound_plan_alone():
    probs, grid = I.draw_instances(2, seed=203, d=3), I.combination(4, 1)
    plan = Plan(probs, grid, 6, device=DEV)
    plan.solve()
    before = plan.state().cpu().numpy()
    out = torch.empty(2, dtype=torch.float64, device=DEV)
    L.check(L.lib().amf_solve_static(plan._h, out.data_ptr(), torch.cuda.current_stream().cuda_stream))
    assert np.array_equal(plan.state().cpu().numpy(), before)
    assert np.array_equal(out.cpu().numpy(), plan.combine().cpu().numpy())


def test_static_solve_rejects_plans_beyond_the_limit():
    w = I.workload_ct4()
    sp = StaticPlan(w["problems"], w["grid"], w["steps"])
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(L.AmfError) as ei:
        sp.price(out)
    assert ei.value.status == L.E_INVALID and "static" in str(ei.value)
