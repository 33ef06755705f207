"""Write oracle-computed expected values for the large workloads into tests/golden/.

Calls only the CPU oracle (oracle/) and the input definitions (paper_2408_00559_amd/inputs.py).
Usage:  python tests/golden/make_golden.py ct4 [threads]      (d=4, n=7, psi=3, 100 steps, FP64)
        python tests/golden/make_golden.py batch4 [threads]   (first 16 of the 512 seeded instances)
        python tests/golden/make_golden.py ct6 [threads]      (d=6, n=8, psi=1: sampled grids, 400 steps)
        python tests/golden/make_golden.py fg2d                (d=2 full grid 65x65, 50 steps, FP64)
        python tests/golden/make_golden.py ct6all [threads]   (d=6, n=8, psi=1: every grid, both
                                                               Richardson runs, 8 + 16 steps at the
                                                               workload's dt)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2408_00559_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _dump(obj, name):
    """One key per line, lists on one line (values are written with repr precision)."""
    lines = ["{"]
    items = list(obj.items())
    for i, (k, v) in enumerate(items):
        lines.append(" %s: %s%s" % (json.dumps(k), json.dumps(v), "," if i + 1 < len(items) else ""))
    lines.append("}")
    with open(os.path.join(HERE, name), "w") as f:
        f.write("\n".join(lines) + "\n")


def run_ct4(threads):
    w = I.workload_ct4()
    p = w["problems"][0]
    t = time.time()
    price, units = oracle.price(p, w["grid"], w["steps"], nthreads=threads, return_units=True)
    lv, cf = oracle.ct_grids(p.d, w["grid"].n, w["grid"].psi)
    out = dict(workload=w["name"], steps=w["steps"], price=price,
               unit_levels=lv.tolist(), unit_coef=cf.tolist(), unit_values=list(map(float, units)),
               oracle_seconds=time.time() - t, threads=threads,
               note="FP64 CPU oracle, all component grids, written by tests/golden/make_golden.py")
    _dump(out, "ct4_n7_psi3_fp64.json")


def run_batch4(threads, count=16):
    w = I.workload_batch4()
    t = time.time()
    prices = []
    for p in w["problems"][:count]:
        prices.append(oracle.price(p, w["grid"], w["steps"], nthreads=threads))
    out = dict(workload=w["name"], steps=w["steps"], count=count, prices=prices,
               oracle_seconds=time.time() - t, threads=threads,
               note="FP64 CPU oracle, first %d seeded instances, written by tests/golden/make_golden.py" % count)
    _dump(out, "batch4_first16_fp64.json")


CT6_SAMPLE = [[9, 1, 1, 1, 1, 1], [1, 1, 1, 1, 1, 9], [1, 1, 9, 1, 1, 1], [3, 3, 2, 2, 2, 2],
              [4, 1, 1, 1, 1, 1], [1, 1, 1, 2, 2, 2]]


def run_ct6(threads):
    """Sampled component grids of the d = 6 workload: u_l(x_eval) after the fine run of the
    Richardson pair (2 * 200 steps), one oracle solve per grid."""
    from concurrent.futures import ThreadPoolExecutor
    w = I.workload_ct6()
    p = w["problems"][0]
    lv, _ = oracle.ct_grids(p.d, w["grid"].n, w["grid"].psi)
    listed = set(tuple(int(v) for v in row) for row in lv)
    assert all(tuple(s) in listed for s in CT6_SAMPLE)
    steps = 2 * w["steps"]
    t = time.time()

    def one(levels):
        return float(oracle.interpolate(p, levels, oracle.solve_grid(p, levels, steps)))

    with ThreadPoolExecutor(max_workers=max(1, threads or len(CT6_SAMPLE))) as ex:
        vals = list(ex.map(one, CT6_SAMPLE))
    out = dict(workload=w["name"], steps=steps, unit_levels=CT6_SAMPLE, unit_values=vals,
               oracle_seconds=time.time() - t,
               note="FP64 CPU oracle, sampled component grids after the fine Richardson run, "
                    "written by tests/golden/make_golden.py")
    _dump(out, "ct6_n8_psi1_sampled_fp64.json")


def run_fg2d(threads):
    w = I.workload_fg2d()
    p = w["problems"][0]
    t = time.time()
    price = oracle.price(p, w["grid"], w["steps"], nthreads=1)
    out = dict(workload=w["name"], steps=w["steps"], levels=w["grid"].levels, price=price,
               oracle_seconds=time.time() - t, threads=1,
               note="FP64 CPU oracle, written by tests/golden/make_golden.py")
    _dump(out, "fg2d_65x65_fp64.json")


CT6_SHORT_STEPS = 8


def ct6_short_workload():
    """The d = 6 workload over a shortened horizon: the same problem, grids and step sizes
    (coarse dt = T / 200, fine dt / 2), but T' = 8 dt, so the coarse run takes 8 steps and the fine
    run 16.  (The full 200 + 400 steps over all 2,975 grids take about 11 CPU-hours in the oracle.)"""
    w = I.workload_ct6()
    p = w["problems"][0]
    p.T = p.T * CT6_SHORT_STEPS / w["steps"]
    return dict(w, problems=[p], steps=CT6_SHORT_STEPS, name=w["name"] + "_short")


def run_ct6all(threads):
    w = ct6_short_workload()
    p = w["problems"][0]
    t = time.time()
    price, (uc, uf) = oracle.price(p, w["grid"], w["steps"], nthreads=threads, richardson=True,
                                   return_units=True)
    lv, cf = oracle.ct_grids(p.d, w["grid"].n, w["grid"].psi)
    out = dict(workload=w["name"], maturity=p.T, steps=w["steps"], price=price,
               unit_levels=lv.tolist(), unit_coef=cf.tolist(),
               unit_values_coarse=list(map(float, uc)), unit_values_fine=list(map(float, uf)),
               oracle_seconds=time.time() - t, threads=threads,
               note="FP64 CPU oracle, every component grid, Richardson pair, written by "
                    "tests/golden/make_golden.py")
    _dump(out, "ct6_n8_psi1_short_all_fp64.json")


def reformat(name):
    """Rewrite an existing file in the layout above (values unchanged)."""
    _dump(json.load(open(os.path.join(HERE, name))), name)


if __name__ == "__main__":
    which = sys.argv[1]
    if which == "reformat":
        reformat(sys.argv[2])
        sys.exit(0)
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    {"ct4": run_ct4, "batch4": run_batch4, "ct6": run_ct6, "ct6all": run_ct6all, "fg2d": run_fg2d}[which](threads)
