"""Launch-schedule autotuner: times each admissible schedule of a bound plan on its own data (a
few AMFR-W steps from the initial data, HIP events on the plan's stream) and keeps the fastest.
Schedules within TIE of the fastest count as equal, and among those the XCD-grouped block order
(xcd_remap 1) is kept: it reads each operator halo plane into one XCD's L2 only, so it moves the
least data through HBM for the same time.  Results are cached in a JSON file keyed by the plan's
shape, so each workload is tuned once.

Cache file: $AMF_AUTOTUNE_CACHE, else ~/.cache/amfrw/autotune.json.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

TIE = 0.015          # relative step-time difference below which two schedules count as equal


def cache_path() -> str:
    return os.environ.get("AMF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "amfrw", "autotune.json"))


def signature(plan) -> str:
    i = plan.info
    dev = torch.cuda.get_device_name(plan.device)
    return "d%d|%s|units%d|pts%d|probs%d|%s" % (i.d, plan.precision, i.n_units, i.inner_points,
                                                i.n_problems, dev)


def candidates(plan):
    sc = plan.schedule()
    nodes = [r for r in (1, 2, 4, 8) if r <= sc["max_stencil_nodes"]]
    out = [dict(stencil_nodes=r, xcd_remap=x, resident=0, fuse_axis0=0, march=0)
           for r, x in itertools.product(nodes, (0, 1, 2))]
    out += [dict(stencil_nodes=r, xcd_remap=x, resident=0, fuse_axis0=1, march=0)
            for r, x in itertools.product(nodes, (0, 1)) if plan.fuse_allowed(r)]
    if sc["march_available"]:
        out += [dict(stencil_nodes=sc["stencil_nodes"], xcd_remap=x, resident=0, fuse_axis0=0, march=1)
                for x in (0, 1, 2)]
        if sc["fuse_max_axis0"] <= 1024:
            out += [dict(stencil_nodes=sc["stencil_nodes"], xcd_remap=x, resident=0, fuse_axis0=1, march=1)
                    for x in (0, 1)]
    if sc["resident_available"]:
        out.append(dict(stencil_nodes=sc["stencil_nodes"], xcd_remap=0, resident=1, fuse_axis0=0, march=0))
    return out


def _time(plan, steps: int, reps: int) -> float:
    best = float("inf")
    for _ in range(reps):
        plan.init()
        plan.time_step(1)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.time_step(steps)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / steps)
    return best


def tune(plan, steps: int = 2, reps: int = 2, use_cache: bool = True, verbose: bool = False) -> dict:
    """Pick and set the fastest schedule for `plan`; returns {schedule, ms_per_step, trials}."""
    key = signature(plan)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except ValueError:
            cache = {}
    if use_cache and key in cache:
        sc = cache[key]["schedule"]
        try:
            plan.set_schedule(**sc)
            return dict(cache[key], cached=True)
        except Exception:
            pass
    trials = []
    for sc in candidates(plan):
        plan.set_schedule(**sc)
        ms = _time(plan, steps, reps)
        trials.append(dict(schedule=sc, ms_per_step=ms))
        if verbose:
            print("autotune", sc, "%.3f ms/step" % ms, flush=True)
    fastest = min(t["ms_per_step"] for t in trials)
    near = [t for t in trials if t["ms_per_step"] <= (1.0 + TIE) * fastest]
    best = min(near, key=lambda t: (t["schedule"]["xcd_remap"] != 1, t["ms_per_step"]))
    plan.set_schedule(**best["schedule"])
    rec = dict(schedule=best["schedule"], ms_per_step=best["ms_per_step"], trials=trials)
    if use_cache:
        cache[key] = rec
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, path)
    return dict(rec, cached=False)
