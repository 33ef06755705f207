"""Host-side checks of libamfrw that need no GPU: the library loads, exports every symbol the
header declares, validates descriptors, and enumerates the combination technique's grids exactly as
the paper's formula (cross-checked against the oracle's independent enumeration)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2408_00559_amd import _lib as L
from paper_2408_00559_amd import inputs as I
from paper_2408_00559_amd import solver as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "amfrw.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amf_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)
    assert lib.amf_abi_version() == 2 == L.ABI_VERSION


def _create(probs, grid, steps=10, prec=L.FP64, rich=0, scheme=None):
    lib = L.lib()
    arr = (L.AmfProblem * len(probs))(*[S.problem_struct(p) for p in probs])
    gs = S.grid_struct(grid)
    sc = scheme or S.scheme_amfrw2()
    h = C.c_void_p()
    st = lib.amf_plan_create(arr, len(probs), C.byref(gs), C.byref(sc), prec, steps, rich, C.byref(h))
    return st, h


def test_scheme_coefficients():
    s = S.scheme_amfrw2()
    assert s.stages == 2
    assert s.a[1 * 6 + 0] == 2.0 / 3.0 and s.q[1 * 6 + 0] == -4.0 / 3.0
    assert (s.b[0], s.b[1]) == (1.25, 0.75)
    assert abs(s.theta - (3 + math.sqrt(3)) / 6) < 1e-16 and s.nu == s.theta
    assert s.w_matrix == L.W_AMF and s.struct_size == C.sizeof(L.AmfScheme)


@pytest.mark.parametrize("stages", [1, 2, 3, 6])
def test_theta_gauss_seidel_scheme(stages):
    """Section 4.2: W = P, a_rj = theta, q_rj = -1, b_r = 1."""
    s = S.scheme_theta_gs(0.5, stages)
    assert s.stages == stages and s.w_matrix == L.W_LOWER and s.theta == 0.5
    for r in range(stages):
        assert s.b[r] == 1.0
        for j in range(6):
            assert s.a[r * 6 + j] == (0.5 if j < r else 0.0)
            assert s.q[r * 6 + j] == (-1.0 if j < r else 0.0)
    bad = L.AmfScheme()
    assert L.lib().amf_scheme_theta_gs(0.0, 2, C.byref(bad)) == L.E_INVALID
    assert L.lib().amf_scheme_theta_gs(0.5, 7, C.byref(bad)) == L.E_INVALID


@pytest.mark.parametrize("mutate,status", [
    (lambda p: setattr(p, "beta", 1.5), L.E_INVALID),
    (lambda p: setattr(p, "sigma", -0.1), L.E_INVALID),
    (lambda p: setattr(p, "T", 0.0), L.E_INVALID),
    (lambda p: p.xeval.__setitem__(0, 0.5), L.E_INVALID),
    (lambda p: p.phi.__setitem__(0, 1.5), L.E_INVALID),
    (lambda p: p.rho[0].__setitem__(1, 0.3), L.E_INVALID),     # asymmetric
    (lambda p: p.xmax.__setitem__(1, 0.0), L.E_INVALID),
])
def test_invalid_problems_rejected(mutate, status):
    p = I.draw_instances(1, seed=1, d=3)[0]
    mutate(p)
    st, h = _create([p], I.combination(4, 1))
    assert st == status, L.lib().amf_last_error()
    assert not h.value
    assert len(L.lib().amf_last_error()) > 0


def test_invalid_grid_and_scheme():
    p = I.draw_instances(1, seed=1, d=4)[0]
    assert _create([p], I.combination(2, 1))[0] == L.E_INVALID          # n < d - 1
    assert _create([p], I.combination(5, -1))[0] == L.E_INVALID
    assert _create([p], I.full_grid([21, 1, 1, 1]))[0] == L.E_INVALID
    assert _create([p], I.combination(5, 1), steps=0)[0] == L.E_INVALID
    sc = S.scheme_amfrw2()
    sc.stages = 7
    assert _create([p], I.combination(5, 1), scheme=sc)[0] == L.E_INVALID
    sc = S.scheme_amfrw2()
    sc.w_matrix = 2
    assert _create([p], I.combination(5, 1), scheme=sc)[0] == L.E_INVALID
    sc = S.scheme_amfrw2()
    sc.nu = 0.0
    assert _create([p], I.combination(5, 1), scheme=sc)[0] == L.E_INVALID
    for st in (1, 3, 6):                                                 # generic stage counts
        sc = S.scheme_theta_gs(0.5, st)
        sc.w_matrix = L.W_AMF
        code, h = _create([p], I.combination(5, 1), scheme=sc)
        assert code == L.OK
        L.lib().amf_plan_destroy(h)
    arr = (L.AmfProblem * 1)(S.problem_struct(I.draw_instances(1, seed=1, d=4)[0]))
    arr[0].boundary = 5
    gs = S.grid_struct(I.combination(5, 1))
    sc = S.scheme_amfrw2()
    h = C.c_void_p()
    assert L.lib().amf_plan_create(arr, 1, C.byref(gs), C.byref(sc), L.FP64, 10, 0, C.byref(h)) == L.E_INVALID
    q = I.draw_instances(1, seed=1, d=3)[0]
    assert _create([p, q], I.combination(5, 1))[0] == L.E_INVALID      # mixed d
    p7 = I.draw_instances(1, seed=1, d=7)[0]
    assert _create([p7], I.combination(7, 1))[0] == L.E_INVALID


@pytest.mark.parametrize("d,n,psi", [(2, 6, 0), (3, 8, 1), (4, 7, 3), (6, 8, 1), (4, 6, 1)])
def test_units_match_combination_formula(orc, d, n, psi):
    probs = I.draw_instances(2, seed=3, d=d)
    plan_st, h = _create(probs, I.combination(n, psi))
    assert plan_st == L.OK
    lib = L.lib()
    info = L.AmfPlanInfo()
    L.check(lib.amf_plan_info_get(h, C.byref(info)))
    olv, ocf = orc.ct_grids(d, n, psi)
    assert info.n_units == 2 * len(ocf)
    total = 0
    inner = 0
    for u in range(info.n_units):
        prob = C.c_int32()
        lv = (C.c_int32 * 8)()
        cf = C.c_double()
        off = C.c_int64()
        L.check(lib.amf_unit_info(h, u, C.byref(prob), lv, C.byref(cf), C.byref(off)))
        g = u % len(ocf)
        assert prob.value == u // len(ocf)
        assert [lv[i] for i in range(d)] == list(olv[g])
        assert cf.value == ocf[g]
        assert off.value % 64 == 0 and off.value >= total
        total = off.value + (1 << int(sum(olv[g])))
        inner += 1 << int(sum(olv[g]))
    assert info.inner_points == inner
    assert info.stage_updates_per_solve == inner * 2 * 10
    assert info.vector_bytes >= 8 * total
    lib.amf_plan_destroy(h)


def test_workload_sizes():
    """Inner-point counts of the benchmark workloads (d=4 n=7 psi=3; d=6 n=8 psi=1)."""
    st, h = _create(I.workload_ct4()["problems"], I.workload_ct4()["grid"], steps=100)
    info = L.AmfPlanInfo()
    L.check(L.lib().amf_plan_info_get(h, C.byref(info)))
    assert (info.n_units, info.inner_points) == (295, 94568448)
    L.lib().amf_plan_destroy(h)
    w = I.workload_ct6()
    st, h = _create(w["problems"], w["grid"], steps=200, prec=L.FP32, rich=1)
    L.check(L.lib().amf_plan_info_get(h, C.byref(info)))
    assert (info.n_units, info.inner_points) == (2975, 30140416)
    assert info.stage_updates_per_solve == 30140416 * 2 * 200 * 3
    L.lib().amf_plan_destroy(h)


def test_state_calls_need_bound_workspace():
    p = I.draw_instances(1, seed=1, d=3)[0]
    st, h = _create([p], I.combination(4, 1))
    assert st == L.OK
    assert L.lib().amf_init(h, None) == L.E_STATE
    assert L.lib().amf_time_step(h, 1, None) == L.E_STATE
    L.lib().amf_plan_destroy(h)
    L.lib().amf_plan_destroy(None)


def _sched(h):
    sc = L.AmfSchedule()
    sc.struct_size = C.sizeof(L.AmfSchedule)
    L.check(L.lib().amf_schedule_get(h, C.byref(sc)))
    return sc


def _set(h, **kw):
    sc = _sched(h)
    for k, v in kw.items():
        setattr(sc, k, v)
    return L.lib().amf_schedule_set(h, C.byref(sc))


def test_schedule_validation():
    """Launch knobs are checked on the host: node counts, XCD modes, the fused axis-0 solve's
    block-size condition (256 * stencil_nodes >= the longest axis-0 line) and the resident limit."""
    w = I.workload_ct4()
    st, h = _create(w["problems"], w["grid"], steps=w["steps"])
    assert st == L.OK
    sc = _sched(h)
    assert (sc.max_stencil_nodes, sc.fuse_max_axis0, sc.resident_available) == (8, 1024, 0)
    assert _set(h, stencil_nodes=3) == L.E_INVALID
    assert _set(h, stencil_nodes=16) == L.E_INVALID
    assert _set(h, xcd_remap=3) == L.E_INVALID
    assert _set(h, resident=1) == L.E_INVALID               # grids of 2^16..2^19 points
    assert _set(h, stencil_nodes=2, fuse_axis0=1) == L.E_INVALID   # 512 < 1024-node lines
    assert _set(h, stencil_nodes=4, fuse_axis0=1) == L.OK
    assert _set(h, stencil_nodes=8, fuse_axis0=1, xcd_remap=2) == L.OK
    assert _sched(h).fuse_axis0 == 1
    assert _set(h, stencil_nodes=1, fuse_axis0=1) == L.E_INVALID
    assert _sched(h).march_available == 1
    assert _set(h, stencil_nodes=4, fuse_axis0=1, march=1) == L.OK   # short axis-1 lines in the operator
    assert _set(h, stencil_nodes=1, fuse_axis0=1, march=1) == L.OK   # stencil_nodes does not bind march
    assert _set(h, stencil_nodes=4, fuse_axis0=0, march=2) == L.E_INVALID
    assert _set(h, stencil_nodes=4, fuse_axis0=0, march=1) == L.OK
    assert _sched(h).march == 1
    L.lib().amf_plan_destroy(h)
    # the marching operator is built for d <= 4 only
    p6 = I.draw_instances(1, seed=9, d=6)[0]
    st, h = _create([p6], I.combination(5, 1))
    assert _sched(h).march_available == 0
    assert _set(h, stencil_nodes=1, march=1) == L.E_INVALID
    L.lib().amf_plan_destroy(h)
    # a plan whose smallest axis-0 line has 2 nodes: every unit runs at min(stencil_nodes, M_1),
    # but the fused solve needs stencil_nodes <= 2
    p = I.draw_instances(1, seed=9, d=3)[0]
    st, h = _create([p], I.combination(4, 1))
    sc = _sched(h)
    assert sc.max_stencil_nodes == 8 and sc.resident_available == 1
    assert _set(h, stencil_nodes=8) == L.OK
    assert _set(h, stencil_nodes=4, fuse_axis0=1) == L.E_INVALID
    assert _set(h, stencil_nodes=2, fuse_axis0=1) == L.OK
    assert _set(h, stencil_nodes=2, fuse_axis0=0, resident=1) == L.OK
    L.lib().amf_plan_destroy(h)


def test_long_axis0_lines():
    """Axis-0 levels up to 16 build (the paper's standard-technique levels); the W = P solve and the
    fused axis-0 schedules (with or without the marching operator) keep their 2^10 limit and say so."""
    p = I.paper_swaption(3)
    for grid in (I.combination(13, 1), I.combination(12, 0), I.full_grid([16, 0, 0, 0])):
        st, h = _create([p], grid, steps=16)
        assert st == L.OK
        sc = _sched(h)
        assert sc.fuse_max_axis0 > 1024
        assert _set(h, stencil_nodes=8, fuse_axis0=1) == L.E_INVALID
        assert _set(h, stencil_nodes=1, fuse_axis0=1, march=1) == L.E_INVALID   # axis-1 lines > 1024
        assert _set(h, stencil_nodes=1, fuse_axis0=0, march=1) == L.OK
        L.lib().amf_plan_destroy(h)
    gs = S.scheme_theta_gs(1.0, 1)
    assert _create([p], I.combination(13, 1), scheme=gs)[0] == L.E_UNSUPPORTED
    code, h = _create([p], I.combination(9, 1), scheme=gs)
    assert code == L.OK
    L.lib().amf_plan_destroy(h)


@pytest.mark.parametrize("d,n,psi,count", [(4, 7, 3, 1), (4, 6, 1, 3), (3, 5, 0, 2), (6, 5, 1, 1)])
def test_unit_offsets_keep_axis0_lines_inside_operator_blocks(d, n, psi, count):
    """Unit offsets are multiples of 64 elements and of min(M_0, 1024), and units do not overlap:
    a node block of 256 R >= M_0 nodes then never splits an axis-0 line (the fused axis-0 solve
    relies on it)."""
    probs = I.draw_instances(count, seed=3, d=d)
    st, h = _create(probs, I.combination(n, psi))
    assert st == L.OK
    info = L.AmfPlanInfo()
    L.check(L.lib().amf_plan_info_get(h, C.byref(info)))
    prob = C.c_int32()
    lv = (C.c_int32 * L.MAX_D)()
    cf = C.c_double()
    off = C.c_int64()
    end = 0
    for u in range(info.n_units):
        L.check(L.lib().amf_unit_info(h, u, C.byref(prob), lv, C.byref(cf), C.byref(off)))
        m0 = 1 << lv[0]
        assert off.value % 64 == 0 and off.value % min(m0, 1024) == 0, (u, off.value, m0)
        assert off.value >= end
        end = off.value + (1 << sum(lv[i] for i in range(d)))
    assert end * (8 if info.precision == L.FP64 else 4) <= info.vector_bytes
    L.lib().amf_plan_destroy(h)


def test_empty_and_null_arguments():
    """No problems, null descriptors and null outputs are rejected with AMF_E_INVALID; destroying a
    null plan is a no-op; a zero-level axis (M = 1) is a valid, degenerate grid."""
    lib = L.lib()
    p = I.draw_instances(1, seed=2, d=3)[0]
    gs = S.grid_struct(I.combination(4, 1))
    sc = S.scheme_amfrw2()
    h = C.c_void_p()
    arr = (L.AmfProblem * 1)(S.problem_struct(p))
    assert lib.amf_plan_create(arr, 0, C.byref(gs), C.byref(sc), L.FP64, 4, 0, C.byref(h)) == L.E_INVALID
    assert lib.amf_plan_create(None, 1, C.byref(gs), C.byref(sc), L.FP64, 4, 0, C.byref(h)) == L.E_INVALID
    assert lib.amf_plan_create(arr, 1, None, C.byref(sc), L.FP64, 4, 0, C.byref(h)) == L.E_INVALID
    assert lib.amf_plan_create(arr, 1, C.byref(gs), C.byref(sc), L.FP64, 4, 0, None) == L.E_INVALID
    assert len(lib.amf_last_error()) > 0
    st, h = _create([p], I.full_grid([5, 0, 3]))
    assert st == L.OK
    info = L.AmfPlanInfo()
    L.check(lib.amf_plan_info_get(h, C.byref(info)))
    assert (info.n_units, info.inner_points) == (1, 1 << 8)
    assert lib.amf_combine(h, None, None) in (L.E_INVALID, L.E_STATE)
    lib.amf_plan_destroy(h)
    lib.amf_plan_destroy(None)


def test_header_is_plain_c():
    """include/amfrw.h compiles as C99 and as C++17 without warnings (plain types only)."""
    import shutil
    import subprocess
    for cc, args in (("gcc", ["-std=c99", "-x", "c"]), ("g++", ["-std=c++17", "-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip("%s not available" % cc)
        r = subprocess.run([cc, *args, "-Wall", "-Wextra", "-Werror", "-fsyntax-only", HEADER],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_bind_rejects_small_or_misaligned_workspace():
    """amf_plan_bind checks size and alignment before touching the memory."""
    lib = L.lib()
    p = I.draw_instances(1, seed=4, d=3)[0]
    st, h = _create([p], I.combination(4, 1))
    info = L.AmfPlanInfo()
    L.check(lib.amf_plan_info_get(h, C.byref(info)))
    fake = C.c_void_p(1 << 40)                     # never dereferenced: the checks fail first
    assert lib.amf_plan_bind(h, fake, info.workspace_bytes - 1, None) == L.E_INVALID
    assert "too small" in lib.amf_last_error().decode()
    assert lib.amf_plan_bind(h, C.c_void_p((1 << 40) + 64), info.workspace_bytes, None) == L.E_INVALID
    assert lib.amf_plan_bind(h, None, info.workspace_bytes, None) == L.E_INVALID
    lib.amf_plan_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU's share only: --gpus N > 1 exits with status 2 and says why."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
