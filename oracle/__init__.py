"""FP64 CPU oracle: ctypes front end of ``amfrw_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by the benchmark's
CPU-baseline leg, never by the GPU library or its binding.  The C source follows the paper's
Section 3 (Sketch 1, full-grid vector with Outer entries), Section 4 (eq. amfrw, Lemma lema:ls)
and Section 5 (combination formulas) in FP64.

Functions take `paper_2408_00559_amd.inputs.Problem` objects (plain data) and numpy arrays.
Grid vectors here are FULL vectors: prod(M_i + 1) entries, axis 1 fastest (theta_0 of Section 3).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amfrw_oracle.c")
# AMF_ORACLE_LIB names another build of the same source (the sanitizer test loads one built with
# ASan/UBSan); by default the library beside this file is used and built on first use.
_LIB = os.environ.get("AMF_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
MAXD = 8
MAXS = 6


class OrcProblem(C.Structure):
    _fields_ = [("N", C.c_int32), ("model", C.c_int32), ("payoff", C.c_int32), ("bc", C.c_int32),
                ("beta", C.c_double), ("sigma", C.c_double),
                ("alpha", C.c_double * MAXD), ("phi", C.c_double * MAXD), ("tau", C.c_double * MAXD),
                ("rho", C.c_double * (MAXD * MAXD)), ("xmax", C.c_double * MAXD),
                ("T", C.c_double), ("K", C.c_double), ("xeval", C.c_double * MAXD),
                ("discount", C.c_double), ("D", C.c_double * (MAXD * MAXD)), ("c", C.c_double * MAXD),
                ("gcenter", C.c_double * MAXD), ("gwidth", C.c_double)]


class OrcScheme(C.Structure):
    _fields_ = [("s", C.c_int32), ("wkind", C.c_int32), ("a", C.c_double * (MAXS * MAXS)),
                ("q", C.c_double * (MAXS * MAXS)), ("b", C.c_double * MAXS),
                ("theta", C.c_double), ("nu", C.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, FP contraction off so that rounding follows the
    source order)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        pp = C.POINTER(OrcProblem)
        sp = C.POINTER(OrcScheme)
        L.orc_abi.restype = C.c_int32
        L.orc_grid_size.restype = C.c_long
        L.orc_grid_size.argtypes = [C.c_int32, ip]
        L.orc_scheme_amfrw2.argtypes = [sp]
        L.orc_scheme_theta_gs.argtypes = [C.c_double, C.c_int32, sp]
        L.orc_solve_lower.argtypes = [pp, ip, C.c_double, dp, dp]
        L.orc_payoff.restype = C.c_double
        L.orc_payoff.argtypes = [pp, dp]
        L.orc_coefficients.argtypes = [pp, dp, dp, dp, dp]
        L.orc_initial_data.argtypes = [pp, ip, dp]
        L.orc_eval_F.argtypes = [pp, ip, dp, dp]
        L.orc_solve_axis.argtypes = [pp, ip, C.c_int32, C.c_double, dp, dp]
        L.orc_interpolate.restype = C.c_double
        L.orc_interpolate.argtypes = [pp, ip, dp, dp]
        L.orc_advance.restype = C.c_int32
        L.orc_advance.argtypes = [pp, ip, sp, C.c_double, C.c_int32, dp]
        L.orc_solve_grid.restype = C.c_int32
        L.orc_solve_grid.argtypes = [pp, ip, sp, C.c_int32, dp]
        L.orc_ct_grids.restype = C.c_long
        L.orc_ct_grids.argtypes = [C.c_int32, C.c_int32, C.c_int32, ip, dp, C.c_long]
        L.orc_price_grids.restype = C.c_int32
        L.orc_price_grids.argtypes = [pp, ip, dp, C.c_int32, sp, C.c_int32, C.c_int32, dp, dp]
        L.orc_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


PAYOFF = {"caplet": 0, "swaption": 1, "gaussian": 2}
BOUNDARY = {"neumann": 0, "dirichlet": 1}     # eq (bound1) / eq (bound1_0)
W_AMF, W_LOWER = 0, 1


def problem_struct(p, model: int = 0, D=None, c=None, gcenter=None, gwidth: float = 0.0) -> OrcProblem:
    """Marshal an `inputs.Problem` (or a duck-typed equivalent) into the oracle's C struct."""
    s = OrcProblem()
    s.N = p.d
    s.model = model
    s.payoff = PAYOFF[p.payoff]
    s.bc = BOUNDARY[getattr(p, "boundary", "neumann")]
    s.beta = p.beta
    s.sigma = p.sigma
    for i in range(p.d - 1):
        s.alpha[i] = p.alpha[i]
        s.phi[i] = p.phi[i]
        s.tau[i] = p.tau[i]
        for j in range(p.d - 1):
            s.rho[i * MAXD + j] = p.rho[i][j]
    for i in range(p.d):
        s.xmax[i] = p.xmax[i]
        s.xeval[i] = p.xeval[i]
    s.T = p.T
    s.K = p.K
    s.discount = p.discount
    if D is not None:
        for i in range(p.d):
            for k in range(p.d):
                s.D[i * MAXD + k] = D[i][k]
    if c is not None:
        for i in range(p.d):
            s.c[i] = c[i]
    if gcenter is not None:
        for i in range(p.d):
            s.gcenter[i] = gcenter[i]
    s.gwidth = gwidth
    return s


def scheme_amfrw2(nu: float | None = None) -> OrcScheme:
    s = OrcScheme()
    lib().orc_scheme_amfrw2(C.byref(s))
    if nu is not None:
        s.nu = nu
    return s


def scheme_theta_gs(theta: float, stages: int) -> OrcScheme:
    """theta-method with `stages` Gauss-Seidel sweeps as a W-method (Section 4.2): W = P, a = theta,
    q = -1, b = 1."""
    s = OrcScheme()
    lib().orc_scheme_theta_gs(float(theta), int(stages), C.byref(s))
    return s


def scheme_generic(a, q, b, theta, nu, wkind: int = W_AMF) -> OrcScheme:
    s = OrcScheme()
    st = len(b)
    s.s = st
    s.wkind = wkind
    for r in range(st):
        s.b[r] = b[r]
        for j in range(r):
            s.a[r * MAXS + j] = a[r][j]
            s.q[r * MAXS + j] = q[r][j]
    s.theta = theta
    s.nu = nu
    return s


def _levels(levels):
    return np.ascontiguousarray(levels, dtype=np.int32)


def grid_shape(levels):
    """numpy shape (C order, last axis fastest) of a full vector: axis N-1 first."""
    return tuple((1 << int(l)) + 1 for l in reversed(list(levels)))


def grid_size(levels) -> int:
    return int(np.prod([(1 << int(l)) + 1 for l in levels]))


def payoff(p, x, **kw) -> float:
    ps = kw.pop("ps", None) or problem_struct(p, **kw)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_payoff(C.byref(ps), _dp(xx))


def coefficients(p, x, **kw):
    ps = kw.pop("ps", None) or problem_struct(p, **kw)
    N = p.d
    xx = np.ascontiguousarray(x, dtype=np.float64)
    d = np.zeros(N)
    m = np.zeros(N * N)
    a = np.zeros(N)
    lib().orc_coefficients(C.byref(ps), _dp(xx), _dp(d), _dp(m), _dp(a))
    return d, m.reshape(N, N), a


def initial_data(p, levels, ps=None):
    ps = ps or problem_struct(p)
    lv = _levels(levels)
    Y = np.empty(grid_size(levels))
    lib().orc_initial_data(C.byref(ps), _ip(lv), _dp(Y))
    return Y


def eval_F(p, levels, Y, ps=None):
    ps = ps or problem_struct(p)
    lv = _levels(levels)
    Yc = np.ascontiguousarray(Y, dtype=np.float64)
    out = np.empty_like(Yc)
    lib().orc_eval_F(C.byref(ps), _ip(lv), _dp(Yc), _dp(out))
    return out


def solve_axis(p, levels, axis, nudt, G, ps=None):
    ps = ps or problem_struct(p)
    lv = _levels(levels)
    Gc = np.ascontiguousarray(G, dtype=np.float64)
    K = np.empty_like(Gc)
    lib().orc_solve_axis(C.byref(ps), _ip(lv), int(axis), float(nudt), _dp(Gc), _dp(K))
    return K


def solve_lower(p, levels, thdt, R, ps=None):
    """(I - thdt P) K = R with P the lower triangle (diagonal included) of the semi-discrete matrix,
    by forward substitution in the theta_0 order (Section 4.2)."""
    ps = ps or problem_struct(p)
    lv = _levels(levels)
    Rc = np.ascontiguousarray(R, dtype=np.float64)
    K = np.empty_like(Rc)
    lib().orc_solve_lower(C.byref(ps), _ip(lv), float(thdt), _dp(Rc), _dp(K))
    return K


def interpolate(p, levels, Y, x=None, ps=None) -> float:
    ps = ps or problem_struct(p)
    lv = _levels(levels)
    Yc = np.ascontiguousarray(Y, dtype=np.float64)
    xx = np.ascontiguousarray(p.xeval if x is None else x, dtype=np.float64)
    return lib().orc_interpolate(C.byref(ps), _ip(lv), _dp(Yc), _dp(xx))


def advance(p, levels, Y, dt, steps, scheme=None, ps=None):
    """Advance the full vector Y in place by `steps` AMFR-W steps of size dt."""
    ps = ps or problem_struct(p)
    sc = scheme or scheme_amfrw2()
    lv = _levels(levels)
    assert Y.dtype == np.float64 and Y.flags.c_contiguous
    rc = lib().orc_advance(C.byref(ps), _ip(lv), C.byref(sc), float(dt), int(steps), _dp(Y))
    if rc != 0:
        raise MemoryError("oracle advance failed")
    return Y


def solve_grid(p, levels, steps, scheme=None, ps=None):
    ps = ps or problem_struct(p)
    sc = scheme or scheme_amfrw2()
    lv = _levels(levels)
    Y = np.empty(grid_size(levels))
    rc = lib().orc_solve_grid(C.byref(ps), _ip(lv), C.byref(sc), int(steps), _dp(Y))
    if rc != 0:
        raise MemoryError("oracle solve failed")
    return Y


def ct_grids(d, n, psi):
    """(levels[count, d] int32, coef[count]) of the combination technique at level n, offset psi."""
    L = lib()
    cnt = L.orc_ct_grids(d, n, psi, None, None, 0)
    lv = np.zeros((max(cnt, 1), d), dtype=np.int32)
    cf = np.zeros(max(cnt, 1))
    L.orc_ct_grids(d, n, psi, _ip(lv), _dp(cf), cnt)
    return lv[:cnt], cf[:cnt]


def grids_for(p, grid):
    if grid.full:
        return np.asarray([grid.levels], dtype=np.int32), np.ones(1)
    return ct_grids(p.d, grid.n, grid.psi)


def price(p, grid, steps, scheme=None, nthreads=0, richardson=False, ps=None, return_units=False):
    """Price of one instance on a full grid or by the (modified) combination technique.  With
    richardson=True the result is (8 P(2 steps) - P(steps)) / 7."""
    if richardson:
        pc = price(p, grid, steps, scheme, nthreads, False, ps, return_units)
        pf = price(p, grid, 2 * steps, scheme, nthreads, False, ps, return_units)
        if return_units:
            return (8.0 * pf[0] - pc[0]) / 7.0, (pc[1], pf[1])
        return (8.0 * pf - pc) / 7.0
    ps = ps or problem_struct(p)
    sc = scheme or scheme_amfrw2()
    lv, cf = grids_for(p, grid)
    lv = np.ascontiguousarray(lv)
    cf = np.ascontiguousarray(cf)
    units = np.empty(len(cf))
    out = np.zeros(1)
    rc = lib().orc_price_grids(C.byref(ps), _ip(lv), _dp(cf), len(cf), C.byref(sc), int(steps),
                               int(nthreads), _dp(units), _dp(out))
    if rc != 0:
        raise MemoryError("oracle price failed")
    if return_units:
        return float(out[0]), units
    return float(out[0])


def inner_view(Y, levels):
    """Inner nodes (all j_i >= 1) of a full vector, as a flat array with axis 1 fastest."""
    shp = grid_shape(levels)
    A = np.asarray(Y).reshape(shp)
    sl = tuple(slice(1, None) for _ in shp)
    return np.ascontiguousarray(A[sl]).reshape(-1)


def full_from_inner(inner, levels, outer_value=0.0, outer_from=None):
    """Full vector with the given inner nodes; outer nodes from `outer_from` (a full vector) or a
    constant."""
    shp = grid_shape(levels)
    F = (np.array(outer_from, dtype=np.float64).reshape(shp).copy() if outer_from is not None
         else np.full(shp, outer_value))
    sl = tuple(slice(1, None) for _ in shp)
    F[sl] = np.asarray(inner, dtype=np.float64).reshape(tuple(s - 1 for s in shp))
    return F.reshape(-1)


def max_threads() -> int:
    return int(lib().orc_max_threads())
