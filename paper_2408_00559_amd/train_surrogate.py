"""Generate solver labels, train the pricing surrogate, calibrate its error estimate and measure
what it gains over the solver on held-out requests.

    # labels (resumable: each set is written chunk by chunk and a rerun continues where it stopped)
    python -m paper_2408_00559_amd.train_surrogate labels --dir D [--train 200000 --cal 20000 --held 50000]
                                                         [--max-seconds S]
    # training, calibration and evaluation from the stored labels
    python -m paper_2408_00559_amd.train_surrogate train --dir D --out O
    # discretisation error of the labels: the same held-out requests at levels n .. n+3 and at
    # twice the steps on the finest level
    python -m paper_2408_00559_amd.train_surrogate label-accuracy --dir D --out O [--count 128]

Labels: d = 6 (5 rates + V) modified combination technique (psi = 1, level --n), --steps AMFR-W2
steps, FP32 solver (autotuned schedule) with FP64 combination, instances drawn by
inputs.surrogate_instances with seeds 5, 7 and 6 for the training, calibration and held-out sets.
Only the prices are stored (D/<set>_seed<seed>.npy, float64, NaN = not yet computed): the features
are re-drawn from the seeds.  `train` writes O/surrogate_report.json and O/surrogate_weights.pt.
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

SETS = (("train", 5), ("cal", 7), ("held", 6))


def _label_path(d, name, seed):
    return os.path.join(d, "%s_seed%d.npy" % (name, seed))


def labels(a, log):
    os.makedirs(a.dir, exist_ok=True)
    grid = I.combination(a.n, a.psi)
    counts = {"train": a.train, "cal": a.cal, "held": a.held}
    t_start = time.perf_counter()
    meta_path = os.path.join(a.dir, "labels_meta.json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    meta.update({"d": 6, "n": a.n, "psi": a.psi, "steps": a.steps, "chunk": a.chunk,
                 "precision": "fp32 (FP64 combine)", "domain": "4x evaluation point"})
    for name, seed in SETS:
        count = counts[name]
        path = _label_path(a.dir, name, seed)
        y = np.load(path) if os.path.exists(path) else np.full(count, np.nan)
        if len(y) < count:
            y = np.concatenate([y, np.full(count - len(y), np.nan)])
        probs = I.surrogate_instances(count, seed)
        todo = [s for s in range(0, count, a.chunk) if np.isnan(y[s:s + a.chunk]).any()]
        done_before = int(np.sum(~np.isnan(y)))
        t0 = time.perf_counter()
        for s in todo:
            if a.max_seconds and time.perf_counter() - t_start > a.max_seconds:
                log("time budget reached; %s has %d of %d labels" % (name, int(np.sum(~np.isnan(y))), count))
                np.save(path, y)
                json.dump(meta, open(meta_path, "w"), indent=1)
                return 3
            e = min(count, s + a.chunk)
            y[s:e] = S.solver_prices(probs[s:e], grid, a.steps, chunk=a.chunk, tune=True)
            np.save(path, y)
            log("labels %s: %d / %d (%.0f prices/s)" % (name, e, count,
                (int(np.sum(~np.isnan(y))) - done_before) / max(time.perf_counter() - t0, 1e-9)))
        if todo:
            meta.setdefault("rates", {})[name] = (int(np.sum(~np.isnan(y))) - done_before) / (time.perf_counter() - t0)
        json.dump(meta, open(meta_path, "w"), indent=1)
    return 0


def train(a, log):
    os.makedirs(a.out, exist_ok=True)
    meta = json.load(open(os.path.join(a.dir, "labels_meta.json")))
    grid = I.combination(meta["n"], meta["psi"])
    steps = meta["steps"]
    sets = {}
    for name, seed in SETS:
        y = np.load(_label_path(a.dir, name, seed))
        if np.isnan(y).any():
            raise RuntimeError("labels of %s are incomplete" % name)
        probs = I.surrogate_instances(len(y), seed)
        sets[name] = (probs, S.features(probs), y)
    rep = {"labels": dict(meta, counts={k: len(v[2]) for k, v in sets.items()})}
    _, xtr, ytr = sets["train"]
    t0 = time.perf_counter()
    sur = S.Surrogate.train(xtr, ytr, grid, steps, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    torch.cuda.synchronize()
    rep["training"] = {"seconds": time.perf_counter() - t0, "epochs": a.epochs, "batch": a.batch, "lr": a.lr,
                       "target": "log price" if sur.mlp.norm[4] else "price",
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
    p = out[:, 0].double().cpu().numpy()
    rel = np.abs(p - yh) / np.abs(yh)
    solver_rate = meta.get("rates", {}).get("held")
    ab = np.abs(p - yh)
    rep["held_out"] = {"count": len(yh), "network_prices_per_s": len(yh) / t_net, "network_seconds": t_net,
                       "rel_err": {"median": float(np.median(rel)), "p90": float(np.quantile(rel, 0.9)),
                                   "p99": float(np.quantile(rel, 0.99)), "max": float(rel.max())},
                       "abs_err": {"median": float(np.median(ab)), "p90": float(np.quantile(ab, 0.9)),
                                   "p99": float(np.quantile(ab, 0.99)), "max": float(ab.max())},
                       "label_price": {"median": float(np.median(yh)), "min": float(yh.min()),
                                       "max": float(yh.max()), "nonpositive": int(np.sum(yh <= 0))},
                       "solver_prices_per_s": solver_rate}
    # serving with fallback on a held-out sample (the solver prices every routed request again)
    ns = min(len(hp), a.serve_sample)
    rows = []
    for tol in (1e-4, 1e-3, 1e-2, 3e-2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp, used, _ = sur.price(hp[:ns], tol=tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = np.abs(pp - yh[:ns]) / np.abs(yh[:ns])
        served = ~used
        rows.append({"tol": tol, "requests": ns, "served_fraction": float(served.mean()),
                     "served_rel_err_max": float(r[served].max()) if served.any() else None,
                     "served_rel_err_p95": float(np.quantile(r[served], 0.95)) if served.any() else None,
                     "within_tol_fraction_of_served": float(np.mean(r[served] <= tol)) if served.any() else None,
                     "prices_per_s_with_fallback": ns / dt, "seconds": dt,
                     "speedup_vs_solver": (ns / dt) / solver_rate if solver_rate else None})
        log("tol %.0e: served %.1f%% p95 %s, %.0f prices/s" % (tol, 100 * served.mean(),
            rows[-1]["served_rel_err_p95"], ns / dt))
    rep["fallback"] = rows
    torch.save({"params": sur.mlp.params().cpu(), "norm": sur.mlp.norm, "calib": sur.calib,
                "box_lo": sur.box_lo, "box_hi": sur.box_hi, "layout": sur.mlp.layout(),
                "grid": {"n": meta["n"], "psi": meta["psi"]}, "steps": steps},
               os.path.join(a.out, "surrogate_weights.pt"))
    json.dump(rep, open(os.path.join(a.out, "surrogate_report.json"), "w"), indent=1)
    log(json.dumps(rep))
    return 0


def label_accuracy(a, log):
    """Prices of `count` held-out requests (seed 6) at levels n .. n+3 of the same combination and
    steps, and at the finest level with twice the steps; the label level's difference from the
    finest is its discretisation error as far as these levels resolve it.  Plans hold 32 requests
    (under 1e9 inner points at level n + 3 = 8)."""
    os.makedirs(a.out, exist_ok=True)
    probs = I.surrogate_instances(a.count, 6)
    runs = [(n, a.steps) for n in range(a.n, a.n + 4)] + [(a.n + 3, 2 * a.steps)]
    prices = {}
    for n, steps in runs:
        t0 = time.perf_counter()
        prices[(n, steps)] = np.asarray(S.solver_prices(probs, I.combination(n, a.psi), steps,
                                                        chunk=32, tune=False), dtype=np.float64)
        log("level %d, %d steps: %.1f s" % (n, steps, time.perf_counter() - t0))
    ref = prices[(a.n + 3, 2 * a.steps)]
    scale = np.abs(ref)
    rep = {"d": 6, "psi": a.psi, "requests": a.count, "seed": 6, "precision": "fp32 (FP64 combine)",
           "reference": {"n": a.n + 3, "steps": 2 * a.steps}, "levels": []}
    for (n, steps), v in prices.items():
        rel = np.abs(v - ref) / scale
        rep["levels"].append({"n": n, "steps": steps, "non_positive": int(np.sum(v <= 0)),
                              "rel_diff_median": float(np.median(rel)),
                              "rel_diff_p90": float(np.quantile(rel, 0.9)),
                              "rel_diff_max": float(np.max(rel)),
                              "abs_diff_median": float(np.median(np.abs(v - ref)))})
    rep["reference_non_positive"] = int(np.sum(ref <= 0))
    rep["reference_price_median"] = float(np.median(ref))
    json.dump(rep, open(os.path.join(a.out, "label_accuracy.json"), "w"), indent=1)
    log(json.dumps(rep))
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["labels", "train", "label-accuracy"])
    ap.add_argument("--dir", required=True, help="label directory")
    ap.add_argument("--out", default=None)
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--cal", type=int, default=20000)
    ap.add_argument("--held", type=int, default=50000)
    ap.add_argument("--n", type=int, default=5)
    ap.add_argument("--psi", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--max-seconds", type=float, default=0.0)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--serve-sample", type=int, default=4096)
    ap.add_argument("--count", type=int, default=128, help="requests of the label-accuracy study")
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if a.mode == "labels":
        return labels(a, log)
    if not a.out:
        ap.error("%s needs --out" % a.mode)
    if a.mode == "label-accuracy":
        return label_accuracy(a, log)
    return train(a, log)


if __name__ == "__main__":
    sys.exit(main())
