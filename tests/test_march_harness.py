"""Host emulation of the plane-tiled operator on real plans (tests/march_harness.cpp): every global
and table access inside its unit, every LDS access inside the slot ring and free of races between
barriers, and every inner node written exactly once.  CPU only; the plans come from the library's
own host code (amf_plan_create needs no GPU).

The d = 4 benchmark plans (295 grids, 94.6M nodes) are walked in full when AMF_MARCH_FULL=1 (a few
minutes); by default every 13th block of them, and every block of the smaller plans."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2408_00559_amd import _lib as L
from paper_2408_00559_amd import inputs as I
from paper_2408_00559_amd import solver as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "march_harness.cpp")
OUT = os.path.join(ROOT, "_build", "libmarch_harness.so")
OPS = {"stage1": 2, "stage2": 3, "refine": 4}


@pytest.fixture(scope="module")
def harness():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I",
                           os.path.join(ROOT, "paper_2408_00559_amd", "csrc"), SRC, "-o", tmp])
    os.replace(tmp, OUT)
    lib = C.CDLL(OUT)
    lib.march_check.restype = C.c_int
    lib.march_check.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                C.c_int, C.c_int, C.c_int64, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.c_void_p, C.c_char_p, C.c_int]
    return lib


def _plan_units(probs, grid, precision):
    lib = L.lib()
    arr = (L.AmfProblem * len(probs))(*[S.problem_struct(p) for p in probs])
    gs = S.grid_struct(grid)
    sc = S.scheme_amfrw2()
    h = C.c_void_p()
    L.check(lib.amf_plan_create(arr, len(probs), C.byref(gs), C.byref(sc), L.FP64 if precision == "fp64" else L.FP32,
                                10, 0, C.byref(h)))
    info = L.AmfPlanInfo()
    L.check(lib.amf_plan_info_get(h, C.byref(info)))
    d = probs[0].d
    n = int(info.n_units)
    lv = np.zeros((n, 6), dtype=np.int8)
    off = np.zeros(n, dtype=np.int64)
    prob = C.c_int32()
    lvs = (C.c_int32 * 8)()
    cf = C.c_double()
    o = C.c_int64()
    for u in range(n):
        L.check(lib.amf_unit_info(h, u, C.byref(prob), lvs, C.byref(cf), C.byref(o)))
        lv[u, :d] = [lvs[i] for i in range(d)]
        off[u] = o.value
    elem = 8 if precision == "fp64" else 4
    total = int(info.vector_bytes) // elem
    lib.amf_plan_destroy(h)
    return d, lv, off, total, elem


def _walk(harness, probs, grid, precision, op, stride, xorder=0, fuse=0):
    d, lv, off, total, elem = _plan_units(probs, grid, precision)
    writes = np.zeros(total, dtype=np.int32)
    nb, reads = C.c_int64(), C.c_int64()
    err = C.create_string_buffer(512)
    rc = harness.march_check(d, OPS[op], len(off), lv.ctypes.data, off.ctypes.data, total, elem, xorder, fuse, 0,
                             stride, C.byref(nb), C.byref(reads), writes.ctypes.data, err, 512)
    assert rc == 0, err.value.decode()
    inner = np.zeros(total, dtype=bool)
    for u in range(len(off)):
        inner[off[u]:off[u] + (1 << int(lv[u].sum()))] = True
    assert np.all(writes[~inner] == 0)                 # padding is never written
    if stride == 1:
        assert np.all(writes[inner] == 1)              # every node exactly once
    else:
        assert np.all(writes[inner] <= 1)
    return nb.value, reads.value


SMALL = {
    "fg2d": (I.workload_fg2d()["problems"], I.full_grid([6, 6])),
    "d2_long_axis0": (I.workload_fg2d()["problems"], I.full_grid([10, 3])),
    "d2_long_v": (I.workload_fg2d()["problems"], I.full_grid([2, 13])),
    "d2_standard_ct": ([I.paper_caplet()], I.combination(6, 0)),
    "d3_ct": (I.draw_instances(2, seed=31, d=3), I.combination(5, 1)),
    "d3_ragged": (I.draw_instances(1, seed=33, d=3), I.full_grid([7, 0, 8])),
    "d4_ct": (I.draw_instances(3, seed=41, d=4), I.combination(4, 1)),
    "d4_levels_0": (I.draw_instances(1, seed=42, d=4), I.combination(3, 0)),
}


@pytest.mark.parametrize("op", list(OPS))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_march_small_plans_every_block(harness, name, precision, op):
    """The unit-by-unit table and the XCD-grouped one, with and without the fused axis-1 solve."""
    probs, grid = SMALL[name]
    for fuse in (0, 1):
        _walk(harness, probs, grid, precision, op, 1, 0, fuse)
        _walk(harness, probs, grid, precision, op, 1, 1, fuse)


@pytest.mark.parametrize("xorder,fuse", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("op", ["stage1", "stage2", "refine"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_march_benchmark_plan(harness, precision, op, xorder, fuse):
    """The d = 4, n = 7, psi = 3 workload (295 grids, 94.6M nodes), in the benchmark's XCD order
    with and without the fused axis-1 solve."""
    w = I.workload_ct4()
    stride = 1 if os.environ.get("AMF_MARCH_FULL") == "1" else 13
    nb, reads = _walk(harness, w["problems"], w["grid"], precision, op, stride, xorder, fuse)
    assert nb > 10000


def test_march_batch_plan_sample(harness):
    """A 16-instance slice of the 512-instance batch (d = 4, n = 6, psi = 1: grids down to 2 points
    per axis, tiles smaller than a block)."""
    w = I.workload_batch4(count=16)
    _walk(harness, w["problems"], w["grid"], "fp32", "stage2", 1)
    _walk(harness, w["problems"], w["grid"], "fp32", "refine", 1, 1, 1)
