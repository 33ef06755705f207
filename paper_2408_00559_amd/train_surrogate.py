"""Generate solver labels, train the pricing surrogate, calibrate its error estimate and measure
what it gains over the solver on held-out requests.

    python -m paper_2408_00559_amd.train_surrogate --out <dir> [--train 16384 --cal 4096 --held 8192]

Labels: d = 6 (5 rates + V) modified combination technique (psi = 1, level --n), --steps AMFR-W2
steps, FP32 solver with FP64 combination, instances drawn by inputs.surrogate_instances (seeds 5,
7 and 6 for training, calibration and held-out sets).  Writes <dir>/surrogate_report.json and
<dir>/surrogate_weights.pt.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import inputs as I
from . import surrogate as S


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=8192)
    ap.add_argument("--cal", type=int, default=2048)
    ap.add_argument("--held", type=int, default=4096)
    ap.add_argument("--n", type=int, default=5)
    ap.add_argument("--psi", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    log = lambda m: print(m, flush=True)
    grid = I.combination(a.n, a.psi)
    sets = {}
    rep = {"labels": {"d": 6, "n": a.n, "psi": a.psi, "steps": a.steps, "precision": "fp32 (FP64 combine)",
                      "domain": "4x evaluation point"}}
    for name, count, seed in (("train", a.train, 5), ("cal", a.cal, 7), ("held", a.held, 6)):
        probs = I.surrogate_instances(count, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = S.solver_prices(probs, grid, a.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sets[name] = (probs, S.features(probs), y)
        rep["labels"][name] = {"count": count, "seconds": dt, "solver_prices_per_s": count / dt}
        log("labels %s: %d in %.1f s (%.0f prices/s)" % (name, count, dt, count / dt))
    _, xtr, ytr = sets["train"]
    t0 = time.perf_counter()
    sur = S.Surrogate.train(xtr, ytr, grid, a.steps, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    torch.cuda.synchronize()
    rep["training"] = {"seconds": time.perf_counter() - t0, "epochs": a.epochs, "batch": a.batch, "lr": a.lr,
                       "network": "8 -> 256 -> 256 -> 256 -> 2, SiLU, BF16 weights/activations, FP32 accumulate"}
    _, xc, yc = sets["cal"]
    rep["calibration"] = {"factor": sur.calibrate(xc, yc), "quantile": 0.95}
    hp, xh, yh = sets["held"]
    # network throughput alone (batched forward, device-resident inputs)
    xt = torch.tensor(xh, dtype=torch.float32, device="cuda:0")
    sur.mlp.forward(xt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        out = sur.mlp.forward(xt)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / reps
    p, err = out[:, 0].double().cpu().numpy(), out[:, 1].double().cpu().numpy()
    rel = np.abs(p - yh) / np.abs(yh)
    rep["held_out"] = {"count": len(yh), "network_prices_per_s": len(yh) / t_net,
                       "network_seconds": t_net,
                       "rel_err": {"median": float(np.median(rel)), "p90": float(np.quantile(rel, 0.9)),
                                   "p99": float(np.quantile(rel, 0.99)), "max": float(rel.max())},
                       "solver_prices_per_s": rep["labels"]["held"]["solver_prices_per_s"]}
    rows = []
    for tol in (1e-4, 1e-3, 1e-2, 3e-2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp, used, tn, tf = sur.price(hp, tol=tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = np.abs(pp - yh) / np.abs(yh)
        served = ~used
        rows.append({"tol": tol, "served_fraction": float(served.mean()),
                     "served_rel_err_max": float(r[served].max()) if served.any() else None,
                     "served_rel_err_p95": float(np.quantile(r[served], 0.95)) if served.any() else None,
                     "within_tol_fraction_of_served": float(np.mean(r[served] <= tol)) if served.any() else None,
                     "prices_per_s_with_fallback": len(hp) / dt, "seconds": dt})
        log("tol %.0e: served %.1f%% p95 %s, %.0f prices/s" % (tol, 100 * served.mean(),
            rows[-1]["served_rel_err_p95"], len(hp) / dt))
    rep["fallback"] = rows
    torch.save({"params": sur.mlp.params().cpu(), "norm": sur.mlp.norm, "calib": sur.calib,
                "box_lo": sur.box_lo, "box_hi": sur.box_hi, "layout": sur.mlp.layout(),
                "grid": {"n": a.n, "psi": a.psi}, "steps": a.steps}, os.path.join(a.out, "surrogate_weights.pt"))
    json.dump(rep, open(os.path.join(a.out, "surrogate_report.json"), "w"), indent=1)
    log(json.dumps(rep))
    return 0


if __name__ == "__main__":
    sys.exit(main())
