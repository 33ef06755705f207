"""Write oracle-computed expected values for the large workloads into tests/golden/.

Calls only the CPU oracle (oracle/) and the input definitions (paper_2408_00559_amd/inputs.py).
Usage:  python tests/golden/make_golden.py ct4 [threads]      (d=4, n=7, psi=3, 100 steps, FP64)
        python tests/golden/make_golden.py batch4 [threads]   (first 16 of the 512 seeded instances)
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
    json.dump(out, open(os.path.join(HERE, "ct4_n7_psi3_fp64.json"), "w"), indent=1)


def run_batch4(threads, count=16):
    w = I.workload_batch4()
    t = time.time()
    prices = []
    for p in w["problems"][:count]:
        prices.append(oracle.price(p, w["grid"], w["steps"], nthreads=threads))
    out = dict(workload=w["name"], steps=w["steps"], count=count, prices=prices,
               oracle_seconds=time.time() - t, threads=threads,
               note="FP64 CPU oracle, first %d seeded instances, written by tests/golden/make_golden.py" % count)
    json.dump(out, open(os.path.join(HERE, "batch4_first16_fp64.json"), "w"), indent=1)


if __name__ == "__main__":
    which = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    {"ct4": run_ct4, "batch4": run_batch4}[which](threads)
