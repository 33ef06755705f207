"""Pins of the FP64 surrogate-network reference (oracle/mlp.py): its backward pass against central
finite differences, and its BF16 rounding against torch's own float32 -> bfloat16 conversion."""
import numpy as np
import torch

from oracle import mlp as M


def _layout():
    rows, cols = [32, 32, 32], [32, 32, 32]
    w, b, o = [], [], 0
    for r, c in zip(rows, cols):
        w.append(o)
        o += r * c
        b.append(o)
        o += r
    return M.Layout(rows, cols, w, b), o


def test_backward_matches_finite_differences():
    lay, n = _layout()
    rng = np.random.default_rng(0)
    p = rng.normal(scale=0.3, size=n)
    x = rng.normal(size=(5, 8))
    dy = rng.normal(size=(5, 2))
    mean, std = np.zeros(8), np.ones(8)

    def f(pp):
        y, _ = M.forward(lay, pp, x, mean, std)
        return float(np.sum(dy * y[:, :2]))

    y, cache = M.forward(lay, p, x, mean, std)
    g = M.backward(lay, cache, dy)
    idx = rng.choice(n, 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = eps
        fd = (f(p + e) - f(p - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=5000) * 10 ** rng.uniform(-8, 8, 5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e-39])])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.to_bf16(x), ref)
