"""FP64 CPU reference of the pricing surrogate's network (TEST INFRASTRUCTURE ONLY).

A plain fully connected network: inputs normalised by (x - mean)/std, hidden layers
z = W a + b, a = silu(z) = z / (1 + exp(-z)), and a linear output layer with two outputs (price in
normalised units, log of the estimated error).  Parameters use the library's padded layout (given
by layer shapes and offsets), so the same FP32 master vector can be evaluated on both sides.

With bf16=True the inputs, weights, hidden activations and output gradients are rounded to BF16
(round to nearest even) at the points where the GPU stores them in BF16; arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Layout:
    def __init__(self, rows, cols, w_off, b_off):
        self.rows, self.cols, self.w_off, self.b_off = list(rows), list(cols), list(w_off), list(b_off)

    @property
    def layers(self):
        return len(self.rows)

    def unpack(self, p):
        out = []
        for l in range(self.layers):
            r, c = self.rows[l], self.cols[l]
            W = np.asarray(p[self.w_off[l]:self.w_off[l] + r * c], dtype=np.float64).reshape(r, c)
            b = np.asarray(p[self.b_off[l]:self.b_off[l] + r], dtype=np.float64)
            out.append((W, b))
        return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(layout, p, x, in_mean, in_std, bf16=False):
    """Returns the raw outputs y [B, rows_last] and the cache for backward."""
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    B, nin = x.shape
    a = np.zeros((B, layout.cols[0]))
    xn = (np.asarray(x, dtype=np.float32) - np.asarray(in_mean, dtype=np.float32)) / np.asarray(in_std, dtype=np.float32)
    a[:, :nin] = xn
    a = rnd(a)
    params = layout.unpack(p)
    cache = []
    for l, (W, b) in enumerate(params):
        Wr = rnd(W)
        z = a @ Wr.T + b
        cache.append((a, Wr, z))
        if l + 1 < layout.layers:
            a = rnd(silu(z))
        else:
            a = z
    return a, cache


def backward(layout, cache, dy, bf16=False):
    """Gradient of sum(dy * y) with respect to the padded parameter vector (FP64)."""
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    g = np.zeros(layout.b_off[-1] + layout.rows[-1])
    B = dy.shape[0]
    dz = np.zeros((B, layout.rows[-1]))
    dz[:, :dy.shape[1]] = dy
    dz = rnd(dz)
    for l in range(layout.layers - 1, -1, -1):
        a, Wr, z = cache[l]
        dW = dz.T @ a
        db = dz.sum(axis=0)
        r, c = layout.rows[l], layout.cols[l]
        g[layout.w_off[l]:layout.w_off[l] + r * c] = dW.reshape(-1)
        g[layout.b_off[l]:layout.b_off[l] + r] = db
        if l == 0:
            break
        da = dz @ Wr
        zprev = cache[l - 1][2]
        dz = rnd(da * dsilu(zprev))
    return g
