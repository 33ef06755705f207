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
