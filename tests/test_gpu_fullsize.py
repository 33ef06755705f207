"""GPU parity at the benchmark sizes, in the launch configurations the benchmark may time.

* d = 4, n = 7, psi = 3, 100 AMFR-W2 steps (295 component grids of 2^16..2^19 inner nodes): the
  combined price and every component grid's interpolated value against the FP64 oracle's values
  stored in tests/golden/ct4_n7_psi3_fp64.json (written by tests/golden/make_golden.py), for every
  admissible launch schedule, eager and graph-replayed; one full time step element by element on
  sampled component grids (the most elongated ones in each axis).
* 512 seeded d = 4 instances (n = 6, psi = 1): the first 16 prices against the oracle's stored
  values, FP64 and FP32, in the serving configuration (autotuned schedule, graph replay).
* d = 6, n = 8, psi = 1 with the Richardson pair (2,975 grids): u_l(x_eval) of sampled grids after
  the full 200 + 400 steps against the oracle's stored values
  (tests/golden/ct6_n8_psi1_sampled_fp64.json); and EVERY grid and the Richardson price over a
  shortened horizon at the workload's step sizes (8 + 16 steps of dt = T/200 and dt/2; the full
  horizon over all grids costs the oracle about 11 CPU-hours) against
  tests/golden/ct6_n8_psi1_short_all_fp64.json.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2408_00559_amd import autotune
from paper_2408_00559_amd import inputs as I
from paper_2408_00559_amd.solver import Plan

from _util import parallel, rel_maxerr, unit_slices

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
HERE = os.path.dirname(os.path.abspath(__file__))
CT4 = os.path.join(HERE, "golden", "ct4_n7_psi3_fp64.json")
BATCH4 = os.path.join(HERE, "golden", "batch4_first16_fp64.json")


def _golden(path):
    if not os.path.exists(path):
        pytest.skip("stored oracle values not present: %s" % os.path.basename(path))
    return json.load(open(path))


@pytest.fixture(scope="module")
def ct4():
    w = I.workload_ct4()
    return w, _golden(CT4)


def _check_units(plan, g, tol):
    vals = plan.unit_values().cpu().numpy().astype(np.float64)
    units = plan.units()
    assert len(units) == len(g["unit_levels"])
    scale = abs(g["price"])
    for u, v in zip(units, vals):
        k = g["unit_levels"].index(list(u["levels"]))
        assert abs(v - g["unit_values"][k]) / scale < tol, (u["levels"], v, g["unit_values"][k])


def test_ct4_full_size_fp64_every_schedule(ct4):
    w, g = ct4
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp64", device=DEV)
    cands = autotune.candidates(plan)
    assert cands
    for sc in cands:
        plan.set_schedule(**sc)
        price = float(plan.price().cpu().numpy()[0])
        assert abs(price - g["price"]) / abs(g["price"]) < 1e-10, (sc, price, g["price"])
        _check_units(plan, g, 1e-10)
    # graph replay of the tuned schedule (the benchmark's configuration)
    autotune.tune(plan, steps=1, reps=1, use_cache=False)
    plan.use_graph(True)
    for _ in range(2):
        price = float(plan.price().cpu().numpy()[0])
        assert abs(price - g["price"]) / abs(g["price"]) < 1e-10
    _check_units(plan, g, 1e-10)


def test_ct4_full_size_fp32(ct4):
    w, g = ct4
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp32", device=DEV)
    autotune.tune(plan, steps=1, reps=1, use_cache=False)
    plan.use_graph(True)
    price = float(plan.price().cpu().numpy()[0])
    assert abs(price - g["price"]) / abs(g["price"]) < 1e-5, (price, g["price"])
    _check_units(plan, g, 1e-5)


def test_ct4_full_size_one_step_sampled_grids():
    """One time step of the full workload; the component grids with the longest axis 0, axis 1,
    axis 2 and axis 3 (V) compared element by element with the oracle's step."""
    w = I.workload_ct4()
    p = w["problems"][0]
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp64", device=DEV)
    plan.init()
    plan.time_step(1)
    Y = plan.state().cpu().numpy()
    items = unit_slices(plan)
    picks = []
    for ax in range(p.d):
        best = max(items, key=lambda it: (it[0]["levels"][ax], -sum(it[0]["levels"])))
        if best not in picks:
            picks.append(best)

    def ref(item):
        lv = item[0]["levels"]
        Yf = oracle.initial_data(p, lv)
        oracle.advance(p, lv, Yf, p.T / w["steps"], 1)
        return oracle.inner_view(Yf, lv)

    for (u, sl), r in zip(picks, parallel(ref, picks)):
        assert rel_maxerr(Y[sl], r) < 1e-12, (u["levels"], rel_maxerr(Y[sl], r))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_batch4_serving_configuration(precision, tol):
    g = _golden(BATCH4)
    w = I.workload_batch4()
    plan = Plan(w["problems"], w["grid"], w["steps"], precision=precision, device=DEV)
    autotune.tune(plan, steps=1, reps=1, use_cache=False)
    plan.use_graph(True)
    prices = plan.price().cpu().numpy().astype(np.float64)
    ref = np.asarray(g["prices"])
    err = np.abs(prices[:len(ref)] - ref) / np.abs(ref)
    assert err.max() < tol, (err.max(), plan.schedule())
    assert np.all(np.isfinite(prices))


CT6 = os.path.join(HERE, "golden", "ct6_n8_psi1_sampled_fp64.json")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_ct6_full_size_sampled_grids(precision, tol):
    """d = 6, n = 8, psi = 1 (2,975 grids) with the Richardson pair, in the benchmark's configuration
    (autotuned schedule, graph replay): after the solve, u_l(x_eval) of the fine run on sampled grids
    (longest axis 1, 3 and V, a balanced grid, two of the coarsest layer) against the oracle's stored
    values."""
    g = _golden(CT6)
    w = I.workload_ct6()
    plan = Plan(w["problems"], w["grid"], w["steps"], precision=precision, richardson=True, device=DEV)
    autotune.tune(plan, steps=1, reps=1, use_cache=False)
    plan.use_graph(True)
    plan.solve()
    vals = plan.unit_values().cpu().numpy()
    index = {tuple(u["levels"]): i for i, u in enumerate(plan.units())}
    scale = max(abs(v) for v in g["unit_values"])
    for lv, ref in zip(g["unit_levels"], g["unit_values"]):
        got = vals[index[tuple(lv)]]
        assert abs(got - ref) / scale < tol, (lv, got, ref)


CT6ALL = os.path.join(HERE, "golden", "ct6_n8_psi1_short_all_fp64.json")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_ct6_every_grid_short_horizon(precision, tol):
    """Every one of the 2,975 d = 6 grids and the Richardson-extrapolated price, in the benchmark's
    configuration (autotuned schedule, graph replay), with the workload's problem, grids and step
    sizes over 8 coarse + 16 fine steps."""
    g = _golden(CT6ALL)
    w = I.workload_ct6()
    p = w["problems"][0]
    p.T = p.T * g["steps"] / w["steps"]
    assert abs(p.T - g["maturity"]) < 1e-15
    plan = Plan([p], w["grid"], g["steps"], precision=precision, richardson=True, device=DEV)
    autotune.tune(plan, steps=1, reps=1, use_cache=False)
    plan.use_graph(True)
    plan.solve()
    price = plan.combine().item()
    assert abs(price - g["price"]) / abs(g["price"]) < tol, (price, g["price"], plan.schedule())
    vals = plan.unit_values().cpu().numpy()
    units = plan.units()
    assert len(units) == len(g["unit_levels"]) == 2975
    index = {tuple(lv): k for k, lv in enumerate(g["unit_levels"])}
    ref = np.array([g["unit_values_fine"][index[tuple(u["levels"])]] for u in units])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(vals - ref)) / scale < tol, np.max(np.abs(vals - ref)) / scale
