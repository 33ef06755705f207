"""Shared helpers of the GPU parity tests: map between the library's inner-node unit vectors and the
oracle's full vectors, and run the oracle on a list of units in parallel threads."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def unit_slices(plan):
    out = []
    for u in plan.units():
        n = 1 << int(sum(u["levels"]))
        out.append((u, slice(u["offset"], u["offset"] + n)))
    return out


def rel_maxerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def parallel(fn, items, workers=8):
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def isolate_axis(p, ax):
    """A copy of problem p whose operator F reduces to the directional term of axis ax: the other
    volatilities switched off, so no mixed or advection terms remain."""
    from paper_2408_00559_amd import inputs as I
    q = I.Problem(**{k: (list(v) if isinstance(v, list) else v) for k, v in p.__dict__.items()})
    q.rho = [list(r) for r in p.rho]
    if ax != p.d - 1:
        q.sigma = 0.0
    q.alpha = [a if i == ax else 0.0 for i, a in enumerate(p.alpha)]
    q.tau = [0.0] * len(p.tau)
    return q


def axis_backward_error(oracle, p, levels, ax, nudt, x, g):
    """Normwise backward error of inner-node vector x as a solution of the directional system
    (I - nudt A_ax) x = g of Lemma lema:ls, with A_ax applied by the oracle:
    ||r||_inf / (|| |I - nudt A_ax| ||_inf ||x||_inf + ||g||_inf).  The three diagonals of A_ax (for
    the matrix norm) come from the oracle's operator applied to comb vectors (nodes whose axis-ax
    index is k mod 3)."""
    q = isolate_axis(p, ax)
    shp = oracle.grid_shape(levels)
    dim = len(shp) - 1 - ax
    j = np.indices(shp)[dim].reshape(-1)
    cols = [oracle.eval_F(q, levels, (j % 3 == k).astype(np.float64)) for k in range(3)]
    ad = np.choose(j % 3, cols)
    al = np.choose((j - 1) % 3, cols)
    au = np.choose((j + 1) % 3, cols)
    rows = oracle.inner_view(np.abs(1.0 - nudt * ad) + nudt * (np.abs(al) + np.abs(au)), levels)
    Xf = oracle.full_from_inner(x, levels)
    g = np.asarray(g, dtype=np.float64)
    r = oracle.inner_view(Xf - nudt * oracle.eval_F(q, levels, Xf), levels) - g
    x = np.asarray(x, dtype=np.float64)
    return float(np.max(np.abs(r)) / (np.max(rows) * np.max(np.abs(x)) + np.max(np.abs(g))))
