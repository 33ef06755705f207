"""Benchmark: grid-point stage-updates/s of the AMFR-W2 + modified-combination solver on one MI355X.

One benchmark step = one whole solve of the d = 4 workload (3 forward rates + V, modified
combination technique n = 7, psi = 3: 295 component grids, 94.6 M inner points, 100 AMFR-W2 steps)
followed by the FP64 combination into its price.  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("grid-point stage-updates/s and prices/s at 1e-5 rel err, plain FP64 vs batched "
          "FP32/surrogate")
HBM_PEAK_GBPS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_2408_00559_amd", "csrc", f)
              for f in ("amfrw_kernels.hip", "amfrw_march.h", "amfrw_internal.h", "amfrw_consts.h")]
GOLDEN = os.path.join(ROOT, "tests", "golden", "ct4_n7_psi3_fp64.json")


def kernel_hash() -> str:
    """Hash of the device code's sources (kernels and the headers they include)."""
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


COPY_BYTES = 2 << 30


def kernel_class_of(name: str):
    """Map a rocprofv3 kernel name to the library's kernel class (None for other kernels)."""
    from paper_2408_00559_amd import _lib as L
    for sym, lg in (("k_sweep_strided_long<", True), ("k_sweep_strided<", False)):
        if sym in name:
            args = [a.strip() for a in name.split(sym, 1)[1].split(">", 1)[0].split(",")]   # <T, EPI[, V]>
            up = args[1] in ("1", "EPI_UPDATE", "amf::EPI_UPDATE")
            return ("sweep_update" if up else "sweep_strided") + ("_long" if lg else "")
    if "k_sweep_contig<" in name:
        return "sweep_contig_long" if "true>" in name else "sweep_contig"
    if "k_march<" in name:    # template arguments <T, D, OP>
        op = name.split("k_march<", 1)[1].split(">", 1)[0].split(",")[2].strip()
        return {"2": "stage1", "3": "stage2", "4": "refine"}[op]
    for sym in ("k_stencil_vec<", "k_stencil<"):
        if sym in name:       # template arguments <T, D, OP[, R]>
            op = name.split(sym, 1)[1].split(">", 1)[0].split(",")[2].strip()
            return {"0": "operator", "1": "operator", "2": "stage1", "3": "stage2", "4": "refine"}[op]
    for k in ("k_node", "k_unit_values", "k_combine", "k_resident", "k_lincomb", "k_lower"):
        if k in name:
            return {"k_node": "init", "k_unit_values": "unit_values", "k_combine": "combine",
                    "k_resident": "resident", "k_lincomb": "lincomb", "k_lower": "lower"}[k]
    assert L.K_NAMES
    return None


def summarize_pmc(fetch_dir: str, write_dir: str, precision: str, out_path: str, command: str):
    """Per kernel class: median FETCH_SIZE and WRITE_SIZE per dispatch (KiB, from two rocprofv3 --pmc
    runs), scaled by what the same counters read for the 2 GiB device-to-device copy."""
    import csv
    import glob

    def load(d, counter):
        per, copies = {}, []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                name = r["Kernel_Name"]
                if "copyBuffer" in name:
                    copies.append(v)
                k = kernel_class_of(name)
                if k is not None:
                    per.setdefault(k, []).append(v)
        big = sorted(c for c in copies if c * 1024 > COPY_BYTES / 2)
        scale = (COPY_BYTES / 1024.0) / big[len(big) // 2] if big else None
        # median per class: the timed solves dominate the dispatch count, so the median is the
        # tuned schedule's launch even when a few launches of other schedules precede them
        return {k: sorted(v)[len(v) // 2] for k, v in per.items()}, scale, len(big)

    fetch, fs, nf = load(fetch_dir, "FETCH_SIZE")
    write, ws, nw = load(write_dir, "WRITE_SIZE")
    rec = {}
    for k in sorted(set(fetch) | set(write)):
        if k in fetch and k in write and fs and ws:
            rec[k] = {"fetch_KiB": fetch[k], "write_KiB": write[k],
                      "bytes_per_launch": (fetch[k] * fs + write[k] * ws) * 1024.0}
    old = json.load(open(out_path)) if os.path.exists(out_path) else {}
    per_launch = old.get("per_launch", {}) if old.get("kernel_source_sha256_16") == kernel_hash() else {}
    per_launch[precision] = rec
    out = {"kernel_source_sha256_16": kernel_hash(), "copy_calibration": {
        "bytes": COPY_BYTES, "fetch_scale": fs, "write_scale": ws, "copies_seen": [nf, nw]},
        "command": command, "per_launch": per_launch}
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps(out))


def traffic_for(kernel: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_ct4.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    rec = d.get("per_launch", {}).get(precision, {}).get(kernel)
    return None if rec is None else rec.get("bytes_per_launch")


def copy_bandwidth(torch, nbytes=2 << 30, reps=10):
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_form(torch, Plan, w, precision, steps, warmup, tune=True, prof_solves=2):
    """Time `steps` whole solves (+ combine) of workload w as hipGraph replays with per-kernel
    profiling off; then, in a separate pass of `prof_solves` eager solves, take per-kernel HIP-event
    times (recorded by the library around each launch on the plan's stream) for the roofline."""
    from paper_2408_00559_amd import autotune
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    plan = Plan(w["problems"], w["grid"], w["steps"], precision=precision, device="cuda:0")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    tuned = autotune.tune(plan, steps=2, reps=1) if tune else None
    prices = torch.empty(len(w["problems"]), dtype=torch.float64, device="cuda:0")
    plan.use_graph(True)
    for _ in range(max(1, warmup)):
        plan.solve()
        plan.combine(prices)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve()
        plan.combine(prices)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / steps
    price = float(prices[0].item())
    # per-kernel pass (eager launches bracketed by events)
    plan.use_graph(False)
    plan.profile_begin()
    tp0 = time.perf_counter()
    for _ in range(prof_solves):
        plan.solve()
        plan.combine(prices)
    torch.cuda.synchronize()
    sec_eager = (time.perf_counter() - tp0) / prof_solves
    kstats = plan.profile_end()
    su = plan.stage_updates
    hot = [k for k in kstats if k not in ("init", "operator", "unit_values", "combine")]
    dom = max(hot, key=lambda k: kstats[k]["ms"])
    ks = kstats[dom]
    achieved = ks["algo_bytes"] / (ks["ms"] * 1e-3) / 1e9 if ks["ms"] > 0 else 0.0
    launches = max(ks["launches"], 1)
    from paper_2408_00559_amd import _lib as L
    sym = L.K_SYMBOLS[dom]
    if plan.schedule()["march"] and dom in ("stage1", "stage2", "refine"):   # the plane-tiled operator ran
        sym = "k_march<%s>" % {"stage1": "OP_STAGE1", "stage2": "OP_STAGE2", "refine": "OP_REFINE"}[dom]
    roof = {"kernel": dom, "kernel_symbol": sym, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_for(dom, precision),
            "algo_bytes_per_launch": ks["algo_bytes"] / launches,
            "avg_launch_us": ks["ms"] * 1e3 / launches, "launches_per_solve": ks["launches"] / prof_solves,
            "measured_in": "separate eager pass of %d solves, HIP events on the plan's stream" % prof_solves}
    per_kernel = {k: {"launches_per_solve": v["launches"] / prof_solves, "ms_per_solve": v["ms"] / prof_solves,
                      "GBps": (v["algo_bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
                  for k, v in kstats.items() if v["launches"]}
    out = dict(value=su / sec, sec_per_solve=sec, sec_per_solve_eager_profiled=sec_eager, price=price,
               stage_updates=su, roofline=roof, plan_setup_s=t_setup,
               kernels=per_kernel, units=plan.n_units, inner_points=plan.inner_points,
               schedule=plan.schedule(), autotune=(None if tuned is None else
                                                   {"trials": tuned.get("trials"), "cached": tuned.get("cached")}))
    del plan
    torch.cuda.empty_cache()
    return out


def run_serving(torch, Plan, batches=200):
    """Batched serving: 512 seeded parameter sets (d = 4, modified combination n = 6, psi = 1,
    100 steps), FP32 stencil and sweeps with FP64 combination, the whole solve replayed as one
    hipGraph.  Latency per price = submit-to-host-result time of its batch."""
    import numpy as np

    from paper_2408_00559_amd import autotune
    from paper_2408_00559_amd import inputs as I

    w = I.workload_batch4()
    n = len(w["problems"])
    ref64 = Plan(w["problems"], w["grid"], w["steps"], precision="fp64", device="cuda:0")
    autotune.tune(ref64, steps=1, reps=1)
    p64 = ref64.price().cpu().numpy()
    del ref64
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp32", device="cuda:0")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tuned = autotune.tune(plan, steps=1, reps=1)
    plan.use_graph(True)
    prices = torch.empty(n, dtype=torch.float64, device="cuda:0")
    plan.solve()
    plan.combine(prices)
    torch.cuda.synchronize()
    lat = []
    host = None
    tb = time.perf_counter()
    for _ in range(batches):
        t0 = time.perf_counter()
        plan.solve()
        plan.combine(prices)
        host = prices.cpu().numpy()
        lat.append(time.perf_counter() - t0)
    wall = time.perf_counter() - tb
    lat = np.array(lat)
    rel = np.abs(host - p64) / np.abs(p64)
    golden = os.path.join(ROOT, "tests", "golden", "batch4_first16_fp64.json")
    rel_oracle = None
    if os.path.exists(golden):
        g = json.load(open(golden))
        k = g["count"]
        rel_oracle = float(np.max(np.abs(host[:k] - np.array(g["prices"])) / np.abs(np.array(g["prices"]))))
    out = {"workload": w["name"], "instances": n, "component_grids": plan.n_units,
           "inner_points": plan.inner_points, "dtype": "f32 (FP64 combine)", "graph": True,
           "batches": batches, "prices_per_s": n * batches / wall,
           "stage_updates_per_s": plan.stage_updates * batches / wall,
           "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                         "min": float(lat.min()), "max": float(lat.max())},
           "max_rel_err_vs_fp64": float(rel.max()), "max_rel_err_vs_oracle_first16": rel_oracle,
           "plan_setup_s": setup_s,
           "schedule": plan.schedule(), "autotune_cached": tuned.get("cached")}
    del plan
    torch.cuda.empty_cache()
    return out


def run_fg2d(torch, Plan, reps=200):
    """The d = 2 full grid 65 x 65 (FP64, 50 AMFR-W2 steps, one caplet): the whole solve replayed as
    a hipGraph; a 32 KiB state, so the time is launch latency, not bandwidth.  The error is against
    the oracle's stored price (tests/golden/fg2d_65x65_fp64.json)."""
    import numpy as np

    from paper_2408_00559_amd import autotune
    from paper_2408_00559_amd import inputs as I

    w = I.workload_fg2d()
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp64", device="cuda:0")
    tuned = autotune.tune(plan, steps=2, reps=1)
    plan.use_graph(True)
    pr = torch.empty(1, dtype=torch.float64, device="cuda:0")
    plan.solve()
    plan.combine(pr)
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.solve()
        plan.combine(pr)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat)
    price = float(pr.item())
    golden = os.path.join(ROOT, "tests", "golden", "fg2d_65x65_fp64.json")
    ref = json.load(open(golden))["price"] if os.path.exists(golden) else None
    out = {"workload": w["name"], "time_steps": w["steps"], "inner_points": plan.inner_points,
           "sec_per_solve_p50": float(np.median(lat)), "sec_per_solve_min": float(lat.min()),
           "stage_updates_per_s": plan.stage_updates / float(np.median(lat)), "price": price,
           "oracle_price": ref, "rel_err_vs_oracle": abs(price - ref) / abs(ref) if ref else None,
           "schedule": plan.schedule(), "autotune_cached": tuned.get("cached")}
    del plan
    return out


def run_paper_tables(torch, Plan):
    """The paper's own Section 6 runs on this GPU in FP64 (the paper's precision), against the
    prices and times it prints (tests/golden/paper_tables.json; the paper's times are from its own
    CPU runs and are context, not a target): Table sg_d4 (standard technique, 8 steps, levels
    12-17), Table d4:level (psi = 1, 2, levels 9-13, 16 steps) and Table d1:Level (caplet, psi = 1,
    2, levels 7-14, 256 steps).  Then two comparisons the method motivates at d = 4, psi = 1,
    16 steps: Neumann against Dirichlet rate faces (eq. (bound1) vs eq. (bound1_0)), and the cost
    per step of AMFR-W2 against the theta-method with one Gauss-Seidel sweep (W = P, Section 4.2).
    Each solve is timed on its second call (the first builds and caches the launch graph)."""
    import numpy as np

    from paper_2408_00559_amd import inputs as I
    from paper_2408_00559_amd import solver as S

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))

    def solve(problem, grid, steps, scheme=None):
        plan = Plan([problem], grid, steps, precision="fp64", scheme=scheme, device="cuda:0")
        plan.set_schedule(march=1 if plan.schedule()["march_available"] else 0, xcd_remap=1, fuse_axis0=0)
        plan.use_graph(True)
        pr = torch.empty(1, dtype=torch.float64, device="cuda:0")
        plan.solve()
        plan.combine(pr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve()
        plan.combine(pr)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out = (float(pr.item()) * 1e4, sec, plan.inner_points)
        del plan
        return out

    def table(name, problem_of, rows, keep=lambda r: True):
        res = []
        for r in rows:
            if not keep(r):
                continue
            psi, n, steps, ref, paper_s = r[0], r[1], r[2], r[3], r[4]
            v, sec, pts = solve(problem_of(), I.combination(n, psi), steps)
            res.append({"psi": psi, "n": n, "steps": steps, "price_bps": v, "paper_bps": ref,
                        "rel_diff": abs(v - ref) / abs(ref), "gpu_s": sec, "paper_s": paper_s,
                        "inner_points": pts})
        torch.cuda.empty_cache()
        return {"table": name, "rows": res, "max_rel_diff": max(x["rel_diff"] for x in res)}

    out = {
        "sg_d4": table("sg_d4", lambda: I.paper_swaption(3), gold["sg_d4"]["rows"], lambda r: r[2] == 8),
        "d4_level": table("d4:level", lambda: I.paper_swaption(3), gold["d4_level_all"]["rows"]),
        "d1_level": table("d1:Level", I.paper_caplet, gold["d1_level_all"]["rows"]),
    }
    # boundary kinds at d = 4 (no printed Dirichlet values: the two series side by side)
    bc = []
    for n in (9, 10, 11, 12):
        neu = solve(I.paper_swaption(3), I.combination(n, 1), 16)[0]
        q = I.paper_swaption(3)
        q.boundary = I.DIRICHLET
        dir_ = solve(q, I.combination(n, 1), 16)[0]
        bc.append({"n": n, "neumann_bps": neu, "dirichlet_bps": dir_})
    out["boundary_d4_psi1"] = bc
    # cost per step: AMFR-W2 (two stages, AMF W) and Crank-Nicolson with s Gauss-Seidel sweeps
    # (theta = 1/2, W = P; order 2 for s >= 2)
    steps = 16
    w2 = solve(I.paper_swaption(3), I.combination(9, 1), steps)
    cost = {"steps": steps, "paper_bps_d4_level_n9": gold["d4_level_all"]["rows"][0][3],
            "amfrw2": {"price_bps": w2[0], "ms_per_step": w2[1] * 1e3 / steps}}
    for st in (2, 4):
        gs = solve(I.paper_swaption(3), I.combination(9, 1), steps, scheme=S.scheme_theta_gs(0.5, st))
        cost["theta_half_gauss_seidel_s%d" % st] = {"price_bps": gs[0], "ms_per_step": gs[1] * 1e3 / steps}
    out["scheme_cost_d4_psi1_n9"] = cost
    torch.cuda.empty_cache()
    return out


def run_ct6(torch, Plan):
    """d = 6 (5 rates + V), modified combination n = 8, psi = 1 (2975 component grids): FP32
    stencil and sweeps with FP64 combination, fourth order in time by Richardson extrapolation of
    AMFR-W2 over 200 and 400 steps; error per price against the FP64 run of the same scheme."""
    from paper_2408_00559_amd import autotune
    from paper_2408_00559_amd import inputs as I

    w = I.workload_ct6()
    res = {}
    for prec in ("fp32", "fp64"):
        plan = Plan(w["problems"], w["grid"], w["steps"], precision=prec, richardson=True, device="cuda:0")
        autotune.tune(plan, steps=2, reps=1)
        plan.use_graph(True)
        pr = torch.empty(1, dtype=torch.float64, device="cuda:0")
        plan.solve()
        plan.combine(pr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve()
        plan.combine(pr)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        res[prec] = {"price": float(pr.item()), "sec_per_solve": sec,
                     "stage_updates_per_s": plan.stage_updates / sec, "schedule": plan.schedule()}
        units, pts, su = plan.n_units, plan.inner_points, plan.stage_updates
        del plan
        torch.cuda.empty_cache()
    res["rel_err_fp32_vs_fp64"] = abs(res["fp32"]["price"] - res["fp64"]["price"]) / abs(res["fp64"]["price"])
    res.update({"workload": w["name"], "component_grids": units, "inner_points": pts,
                "stage_updates_per_solve": su, "time_steps": "200 + 400 (Richardson)"})
    return res


def run_surrogate(torch, Plan):
    """Form (4) next to the solver on the surrogate's label discretisation (d = 6, n = 5, psi = 1,
    100 steps, FP32 with FP64 combine): solver prices/s on 512 seeded requests, the BF16-MFMA
    network's inference prices/s (amf_mlp_infer) on 50,000 and on 2^21 requests (throughput does not
    depend on the weights), and the
    held-out accuracy and fallback rates of the trained network as recorded in
    profiles/surrogate_d6_n5.json by train_surrogate."""
    from paper_2408_00559_amd import autotune
    from paper_2408_00559_amd import inputs as I
    from paper_2408_00559_amd import surrogate as S

    w = I.workload_surrogate_labels(512, 6)
    plan = Plan(w["problems"], w["grid"], w["steps"], precision="fp32", device="cuda:0")
    autotune.tune(plan, steps=1, reps=1)
    plan.use_graph(True)
    plan.price()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.price()
    torch.cuda.synchronize()
    solver_rate = len(w["problems"]) / (time.perf_counter() - t0)
    del plan
    torch.cuda.empty_cache()
    net = S.Mlp(n_in=8, width=256, depth=3, max_batch=50000, seed=1)
    x = torch.randn(50000, 8, dtype=torch.float32, device="cuda:0")
    net.set_normalization([0.0] * 8, [1.0] * 8, 0.02, 0.01)
    net.infer(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net.infer(x)
    torch.cuda.synchronize()
    net_rate = 10 * 50000 / (time.perf_counter() - t0)
    xl = torch.randn(1 << 21, 8, dtype=torch.float32, device="cuda:0")   # a large batch: MFMA-bound
    net.infer(xl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        net.infer(xl)
    torch.cuda.synchronize()
    net_rate_large = 5 * xl.shape[0] / (time.perf_counter() - t0)
    del xl
    res = {"workload": "surrogate labels d6 n5 psi1 100 steps", "solver_prices_per_s": solver_rate,
           "network_prices_per_s": net_rate, "network_prices_per_s_2M_batch": net_rate_large,
           "network_flop_per_price": 2 * (8 * 256 + 2 * 256 * 256 + 256 * 2),
           "network_padded_mfma_tflops_2M_batch": net_rate_large * 2 * (32 * 256 + 2 * 256 * 256 + 256 * 32) / 1e12}
    rep_path = os.path.join(ROOT, "profiles", "surrogate_d6_n5.json")
    if os.path.exists(rep_path):
        rep = json.load(open(rep_path))
        res["trained"] = {"labels": rep.get("labels", {}).get("counts"),
                          "held_out_rel_err": rep.get("held_out", {}).get("rel_err"),
                          "fallback": [{k: r.get(k) for k in ("tol", "served_fraction", "served_rel_err_p95",
                                                              "prices_per_s_with_fallback")}
                                       for r in rep.get("fallback", [])],
                          "source": "profiles/surrogate_d6_n5.json"}
    return res


def cpu_baseline(w, target_seconds=12.0):
    """The FP64 oracle on a bounded sample of the same workload: the smallest combination layer
    (35 component grids of 65,536 inner points) for as many of the 100 time steps, at the workload's
    dt, as take about `target_seconds` on all host cores (a 6-step run sizes it)."""
    import ctypes as C

    import numpy as np

    import oracle

    p = w["problems"][0]
    lv, cf = oracle.ct_grids(p.d, w["grid"].n, w["grid"].psi)
    sums = lv.sum(axis=1)
    sel = lv[sums == sums.min()]
    threads = oracle.max_threads()
    sc = oracle.scheme_amfrw2()
    L = oracle.lib()
    lvc = np.ascontiguousarray(sel, dtype=np.int32)
    coef = np.ones(len(sel))
    units = np.empty(len(sel))
    out = np.zeros(1)

    def run(steps, ngrids=len(sel), nthreads=threads):
        # orc_price_grids solves to the problem's maturity with `steps` steps: scale the maturity
        # so that dt stays the workload's T / steps
        ps = oracle.problem_struct(p)
        ps.T = p.T * steps / w["steps"]
        t0 = time.perf_counter()
        rc = L.orc_price_grids(C.byref(ps), lvc.ctypes.data_as(C.POINTER(C.c_int32)),
                               coef.ctypes.data_as(C.POINTER(C.c_double)), ngrids, C.byref(sc), steps,
                               nthreads, units.ctypes.data_as(C.POINTER(C.c_double)),
                               out.ctypes.data_as(C.POINTER(C.c_double)))
        assert rc == 0
        return time.perf_counter() - t0

    t6 = run(6)
    steps = int(min(w["steps"], max(6, round(6 * target_seconds / max(t6, 1e-3)))))
    dt = run(steps)
    su = float(sum(1 << int(s) for s in sel.sum(axis=1))) * 2 * steps
    # the same grids on one thread: 2 grids, steps sized to about a quarter of the target
    g1 = min(2, len(sel))
    t1 = run(2, g1, 1)
    steps1 = int(min(w["steps"], max(2, round(2 * target_seconds / 4 / max(t1, 1e-3)))))
    dt1 = run(steps1, g1, 1)
    su1 = float(g1 * (1 << int(sums.min()))) * 2 * steps1
    return {"value": su / dt, "unit": "stage-updates/s", "cores": threads, "kind": "oracle",
            "seconds": dt,
            "sample": "%d of %d component grids (smallest layer, %d inner points each), %d of %d time "
                      "steps at the workload's dt, FP64 CPU oracle" % (len(sel), len(lv),
                                                                      1 << int(sums.min()), steps,
                                                                      w["steps"]),
            "single_thread": {"value": su1 / dt1, "unit": "stage-updates/s", "cores": 1,
                              "seconds": dt1,
                              "sample": "%d grids of the same layer, %d time steps" % (g1, steps1)},
            "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-ct6", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-fg2d", action="store_true")
    ap.add_argument("--serving-batches", type=int, default=200, help="timed batches of the serving section")
    ap.add_argument("--only", choices=["serving", "ct6", "surrogate", "fg2d", "paper"], default=None,
                    help="run one secondary section alone and print its JSON (profiling runs)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/hbm_traffic_ct4.json from two rocprofv3 --pmc runs")
    ap.add_argument("--pmc-precision", default="fp64")
    ap.add_argument("--pmc-command", default="")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.pmc_precision,
                      os.path.join(ROOT, "profiles", "hbm_traffic_ct4.json"), args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the component grids are independent until the final "
              "FP64 combination, so a multi-GPU run would shard them and add one small reduction; "
              "only the one-GPU share is measured here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2408_00559_amd import inputs as I
    from paper_2408_00559_amd.solver import Plan

    if args.only:
        run = {"serving": lambda t, p: run_serving(t, p, args.serving_batches), "ct6": run_ct6,
               "surrogate": run_surrogate, "fg2d": run_fg2d, "paper": run_paper_tables}[args.only]
        print(json.dumps({args.only: run(torch, Plan)}), flush=True)
        return
    w = I.workload_ct4()
    copy_gbps = copy_bandwidth(torch)
    f64 = None if args.no_fp64 else run_form(torch, Plan, w, "fp64", args.steps, args.warmup)
    f32 = None if args.no_fp32 else run_form(torch, Plan, w, "fp32", args.steps, args.warmup)
    if f64 is None:            # profiling runs of the FP32 form alone
        print(json.dumps({"fp32": f32}), flush=True)
        return
    golden = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else None
    ref = golden["price"] if golden else None
    res = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "stage-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["sec_per_solve"] * 1e3,           # one bench step = one whole solve
        "ms_per_solve": f64["sec_per_solve"] * 1e3,
        "ms_per_time_step": f64["sec_per_solve"] * 1e3 / w["steps"],
        "timing": "hipGraph replays of whole solves, per-kernel profiling off",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "d": 4, "grid": "modified combination n=7 psi=3",
                   "component_grids": f64["units"], "inner_points": f64["inner_points"],
                   "time_steps": w["steps"], "scheme": "AMFR-W2 (nu = theta)",
                   "stage_updates_per_solve": f64["stage_updates"]},
        "prices_per_s": 1.0 / f64["sec_per_solve"],
        "price": f64["price"],
        "oracle_price": ref,
        "rel_err_vs_oracle": (abs(f64["price"] - ref) / abs(ref)) if ref else None,
        "roofline": f64["roofline"],
        "kernels": f64["kernels"],
        "schedule": f64["schedule"],
        "autotune": f64["autotune"],
        "plan_setup_s": f64["plan_setup_s"],
        "copy_GBps": copy_gbps,
    }
    if f32 is not None:
        base = ref if ref else f64["price"]
        res["fp32"] = {"value": f32["value"], "unit": "stage-updates/s", "dtype": "f32",
                       "ms_per_solve": f32["sec_per_solve"] * 1e3,
                       "ms_per_time_step": f32["sec_per_solve"] * 1e3 / w["steps"],
                       "prices_per_s": 1.0 / f32["sec_per_solve"],
                       "price": f32["price"], "rel_err": abs(f32["price"] - base) / abs(base),
                       "rel_err_against": "oracle" if ref else "fp64 GPU",
                       "roofline": f32["roofline"], "kernels": f32["kernels"],
                       "schedule": f32["schedule"], "autotune": f32["autotune"]}
    if not args.no_fg2d:
        res["fg2d_65x65"] = run_fg2d(torch, Plan)
    if not args.no_serving:
        res["serving_batch4"] = run_serving(torch, Plan, args.serving_batches)
    if not args.no_ct6:
        res["ct6_fp32_richardson"] = run_ct6(torch, Plan)
    if not args.no_surrogate:
        res["surrogate"] = run_surrogate(torch, Plan)
    if not args.no_paper:
        res["paper_tables"] = run_paper_tables(torch, Plan)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
