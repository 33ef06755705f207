"""Learned pricing surrogate on top of the solver.

A small network maps the eight instance parameters (beta, sigma, phi, F0, V0, K, T, lambda) to a
price and an estimate of its own error; it is trained on prices the solver computes, and requests
whose estimated relative error exceeds the caller's tolerance, or that fall outside the training
box, are priced by the solver instead.  The network runs in libamfrw (BF16 MFMA kernels, FP32
accumulation); this module marshals arguments and orchestrates training and fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from typing import List, Sequence

import numpy as np
import torch

from . import _lib as L
from . import inputs as I
from .solver import Plan, _stream


def _mlp_lib():
    lib = L.lib()
    if not getattr(lib, "_mlp_ready", False):
        vp, st = C.c_void_p, C.c_int32
        lib.amf_mlp_last_error.restype = C.c_char_p
        lib.amf_mlp_create.restype = st
        lib.amf_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                       C.POINTER(vp)]
        lib.amf_mlp_info_get.restype = st
        lib.amf_mlp_info_get.argtypes = [vp, C.POINTER(MlpInfo)]
        lib.amf_mlp_bind.restype = st
        lib.amf_mlp_bind.argtypes = [vp, vp, C.c_uint64, vp]
        lib.amf_mlp_set_normalization.restype = st
        fp = C.POINTER(C.c_float)
        lib.amf_mlp_set_normalization.argtypes = [vp, fp, fp, fp, fp, C.c_int32, vp]
        lib.amf_mlp_params.restype = st
        lib.amf_mlp_params.argtypes = [vp, vp, C.c_int32, vp]
        lib.amf_mlp_grads.restype = st
        lib.amf_mlp_grads.argtypes = [vp, vp, vp]
        lib.amf_mlp_forward.restype = st
        lib.amf_mlp_forward.argtypes = [vp, vp, C.c_int32, vp, vp]
        lib.amf_mlp_infer.restype = st
        lib.amf_mlp_infer.argtypes = [vp, vp, C.c_int32, vp, vp]
        lib.amf_mlp_backward.restype = st
        lib.amf_mlp_backward.argtypes = [vp, vp, C.c_int32, vp]
        lib.amf_mlp_train_step.restype = st
        lib.amf_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, C.c_float, vp, vp]
        lib.amf_mlp_destroy.restype = None
        lib.amf_mlp_destroy.argtypes = [vp]
        lib.amf_mlp_set_router.restype = st
        lib.amf_mlp_set_router.argtypes = [vp, fp, fp, C.c_float]
        lib.amf_price_or_fallback.restype = st
        lib.amf_price_or_fallback.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp, vp, vp]
        lib._mlp_ready = True
    return lib


class MlpInfo(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("workspace_bytes", C.c_uint64), ("n_in", C.c_int32),
                ("width", C.c_int32), ("depth", C.c_int32), ("n_out", C.c_int32), ("max_batch", C.c_int32),
                ("layers", C.c_int32), ("layer_rows", C.c_int32 * 8), ("layer_cols", C.c_int32 * 8),
                ("layer_w_offset", C.c_int64 * 8), ("layer_b_offset", C.c_int64 * 8)]


def _check(st):
    if st != L.OK:
        raise L.AmfError(st, _mlp_lib().amf_mlp_last_error().decode())


FEATURES = ["beta", "sigma", "phi", "F0", "V0", "K", "T", "lambda"]


class Mlp:
    """The network: n_in -> width x depth (SiLU) -> (price, log error), on `device`."""

    def __init__(self, n_in=8, width=256, depth=3, max_batch=8192, seed=1, device="cuda:0"):
        lib = _mlp_lib()
        h = C.c_void_p()
        _check(lib.amf_mlp_create(n_in, width, depth, 2, max_batch, seed, C.byref(h)))
        self._h = h
        self.info = MlpInfo()
        _check(lib.amf_mlp_info_get(h, C.byref(self.info)))
        self.device = torch.device(device)
        self.ws = torch.empty(int(self.info.workspace_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        _check(lib.amf_mlp_bind(h, C.c_void_p(base + off), int(self.info.workspace_bytes), _stream()))
        self.n_in = n_in
        self.max_batch = max_batch
        self.norm = None

    def layout(self):
        i = self.info
        n = i.layers
        return ([i.layer_rows[l] for l in range(n)], [i.layer_cols[l] for l in range(n)],
                [i.layer_w_offset[l] for l in range(n)], [i.layer_b_offset[l] for l in range(n)])

    def set_normalization(self, in_mean, in_std, out_mean, out_std, out_log: bool = False):
        f = lambda a: (C.c_float * len(a))(*[float(v) for v in a])
        self.norm = (np.asarray(in_mean, np.float32), np.asarray(in_std, np.float32), float(out_mean),
                     float(out_std), bool(out_log))
        _check(_mlp_lib().amf_mlp_set_normalization(self._h, f(in_mean), f(in_std), f([out_mean]), f([out_std]),
                                                    1 if out_log else 0, _stream()))

    def set_router(self, box_lo, box_hi, calib: float):
        """Training box and calibration factor used by price_or_fallback."""
        f = lambda a: (C.c_float * self.n_in)(*[float(v) for v in a])
        _check(_mlp_lib().amf_mlp_set_router(self._h, f(box_lo), f(box_hi), float(calib)))

    def price_or_fallback(self, plan: Plan, x: torch.Tensor, tol: float, abs_floor: float = 0.0):
        """Prices of the plan's problems (FP64) and the 0/1 solver-routing flags, decided and computed
        in the library: the network where it is trusted, the plan's solver elsewhere."""
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        n = len(plan.problems)
        assert x.shape == (n, self.n_in)
        prices = torch.empty(n, dtype=torch.float64, device=self.device)
        used = torch.empty(n, dtype=torch.int32, device=self.device)
        st = _mlp_lib().amf_price_or_fallback(self._h, plan._h, C.c_void_p(x.data_ptr()), float(tol),
                                              float(abs_floor), C.c_void_p(prices.data_ptr()),
                                              C.c_void_p(used.data_ptr()), _stream())
        L.check(st)
        return prices, used

    def params(self) -> torch.Tensor:
        out = torch.empty(int(self.info.n_params), dtype=torch.float32, device=self.device)
        _check(_mlp_lib().amf_mlp_params(self._h, C.c_void_p(out.data_ptr()), 0, _stream()))
        return out

    def load_params(self, p: torch.Tensor):
        p = p.to(device=self.device, dtype=torch.float32).contiguous()
        _check(_mlp_lib().amf_mlp_params(self._h, C.c_void_p(p.data_ptr()), 1, _stream()))

    def grads(self) -> torch.Tensor:
        out = torch.empty(int(self.info.n_params), dtype=torch.float32, device=self.device)
        _check(_mlp_lib().amf_mlp_grads(self._h, C.c_void_p(out.data_ptr()), _stream()))
        return out

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: [B, n_in] FP32 raw features -> [B, 2] (price, estimated relative error)."""
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        B = x.shape[0]
        out = torch.empty(B, 2, dtype=torch.float32, device=self.device)
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            _check(_mlp_lib().amf_mlp_forward(self._h, C.c_void_p(x[s:e].data_ptr()), e - s,
                                              C.c_void_p(out[s:e].data_ptr()), _stream()))
        return out

    def infer(self, x: torch.Tensor) -> torch.Tensor:
        """Inference only (amf_mlp_infer): the outputs of forward, nothing kept for backward."""
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        out = torch.empty(x.shape[0], 2, dtype=torch.float32, device=self.device)
        _check(_mlp_lib().amf_mlp_infer(self._h, C.c_void_p(x.data_ptr()), x.shape[0], C.c_void_p(out.data_ptr()),
                                        _stream()))
        return out

    def backward(self, dy: torch.Tensor):
        dy = dy.to(device=self.device, dtype=torch.float32).contiguous()
        _check(_mlp_lib().amf_mlp_backward(self._h, C.c_void_p(dy.data_ptr()), dy.shape[0], _stream()))

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float, err_weight: float = 0.1,
                   loss: torch.Tensor | None = None):
        _check(_mlp_lib().amf_mlp_train_step(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                             x.shape[0], float(lr), float(err_weight),
                                             C.c_void_p(loss.data_ptr()) if loss is not None else None,
                                             _stream()))

    def close(self):
        if getattr(self, "_h", None):
            _mlp_lib().amf_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------------------------
def solver_prices(problems: Sequence[I.Problem], grid, steps: int, precision: str = "fp32",
                  chunk: int = 512, device: str = "cuda:0", tune: bool = True) -> np.ndarray:
    """Prices of `problems` by the solver: batched plans of `chunk` instances, each run with the
    autotuned schedule (cached per plan shape) and the FP64 combination."""
    from . import autotune
    out = []
    for s in range(0, len(problems), chunk):
        plan = Plan(problems[s:s + chunk], grid, steps, precision=precision, device=device)
        if tune:
            autotune.tune(plan, steps=1, reps=1)
        out.append(plan.price().cpu().numpy())
        del plan
    return np.concatenate(out) if out else np.zeros(0)


def features(problems: Sequence[I.Problem]) -> np.ndarray:
    return np.asarray([I.surrogate_features(p) for p in problems], dtype=np.float32)


class Surrogate:
    """Trained network plus the box it was trained on; `price` serves requests with fallback."""

    def __init__(self, mlp: Mlp, box_lo: np.ndarray, box_hi: np.ndarray, grid, steps: int, calib: float = 1.0):
        self.mlp, self.box_lo, self.box_hi, self.grid, self.steps = mlp, box_lo, box_hi, grid, steps
        self.calib = calib

    def calibrate(self, x: np.ndarray, y: np.ndarray, q: float = 0.95) -> float:
        """Scale the error estimate so that a fraction q of the calibration residuals (data not
        used for training) lie below it: calib = q-quantile of |actual rel. error| / estimate."""
        p, err = self.predict(x)
        ratio = (np.abs(p - y) / np.abs(y)) / np.maximum(err, 1e-30)
        self.calib = float(np.quantile(ratio, q))
        self.mlp.set_router(self.box_lo, self.box_hi, self.calib)
        return self.calib

    @staticmethod
    def train(x: np.ndarray, y: np.ndarray, grid, steps: int, epochs: int = 300, batch: int = 1024,
              lr: float = 2e-3, seed: int = 1, width: int = 256, depth: int = 3, err_weight: float = 0.1,
              device: str = "cuda:0", log=None) -> "Surrogate":
        mlp = Mlp(n_in=x.shape[1], width=width, depth=depth, max_batch=max(batch, 8192), seed=seed,
                  device=device)
        out_log = bool(np.all(y > 0))          # model log-prices: the residual is a relative error
        yt_ = np.log(y) if out_log else y
        mlp.set_normalization(x.mean(axis=0), x.std(axis=0) + 1e-12, float(yt_.mean()), float(yt_.std()),
                              out_log)
        xt = torch.tensor(x, dtype=torch.float32, device=device)
        yt = torch.tensor(y, dtype=torch.float32, device=device)
        n = x.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        loss = torch.zeros(1, dtype=torch.float32, device=device)
        steps_total = epochs * max(1, n // batch)
        k = 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(device)
            for s in range(0, n - batch + 1, batch):
                idx = perm[s:s + batch]
                xb = xt[idx].contiguous()
                yb = yt[idx].contiguous()
                # cosine decay of the learning rate
                cur = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps_total))
                mlp.train_step(xb, yb, max(cur, lr * 1e-3), err_weight, loss)
                k += 1
            if log is not None and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log("epoch %d loss %.3e" % (ep, loss.item() / batch))
        sur = Surrogate(mlp, x.min(axis=0), x.max(axis=0), grid, steps)
        mlp.set_router(sur.box_lo, sur.box_hi, sur.calib)
        return sur

    def predict(self, x: np.ndarray):
        """(price, estimated relative error before calibration) from the network."""
        out = self.mlp.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
        return out[:, 0].astype(np.float64), out[:, 1].astype(np.float64)

    def price(self, problems: Sequence[I.Problem], tol: float = 1e-4, precision: str = "fp32",
              abs_floor: float = 0.0, plan: Plan | None = None):
        """Prices with fallback, decided and computed in the library (amf_price_or_fallback): the
        network's price where the request lies inside the training box and its calibrated error
        estimate is within `tol` (relative) or `abs_floor` (absolute), else the solver's.  `plan`
        (built here when not given) holds the requests' problems and is the solver.  Returns
        (prices, used_solver mask, seconds)."""
        from . import autotune
        if plan is None:
            plan = Plan(problems, self.grid, self.steps, precision=precision, device=str(self.mlp.device))
            autotune.tune(plan, steps=1, reps=1)
        x = torch.tensor(features(problems), dtype=torch.float32, device=self.mlp.device)
        t0 = time.perf_counter()
        prices, used = self.mlp.price_or_fallback(plan, x, tol, abs_floor)
        dt = time.perf_counter() - t0
        return prices.cpu().numpy(), used.cpu().numpy().astype(bool), dt
