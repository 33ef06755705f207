"""Python front end of libamfrw: marshals `inputs.Problem` / `inputs.GridSpec` into the C ABI and
owns the device workspace as a torch tensor.  Every step of the method runs in the HIP kernels."""
from __future__ import annotations

import ctypes as C
from typing import List, Sequence

import torch

from . import _lib as L
from .inputs import CAPLET, DIRICHLET, NEUMANN, GridSpec, Problem

PAYOFF = {CAPLET: L.PAYOFF_CAPLET, "swaption": L.PAYOFF_SWAPTION}
BOUNDARY = {NEUMANN: L.BC_NEUMANN, DIRICHLET: L.BC_DIRICHLET}


def problem_struct(p: Problem) -> L.AmfProblem:
    s = L.AmfProblem()
    s.struct_size = C.sizeof(L.AmfProblem)
    s.d = p.d
    s.payoff = PAYOFF[p.payoff]
    s.boundary = BOUNDARY[p.boundary]
    s.beta = p.beta
    s.sigma = p.sigma
    for i in range(p.d - 1):
        s.alpha[i] = p.alpha[i]
        s.phi[i] = p.phi[i]
        s.tau[i] = p.tau[i]
        for k in range(p.d - 1):
            s.rho[i * L.RHO_LD + k] = p.rho[i][k]
    for i in range(p.d):
        s.x_max[i] = p.xmax[i]
        s.x_eval[i] = p.xeval[i]
    s.maturity = p.T
    s.strike = p.K
    s.discount = p.discount
    return s


def grid_struct(g: GridSpec) -> L.AmfGridSpec:
    s = L.AmfGridSpec()
    s.struct_size = C.sizeof(L.AmfGridSpec)
    s.full_grid = 1 if g.full else 0
    if g.full:
        for i, l in enumerate(g.levels):
            s.levels[i] = l
    s.n = g.n
    s.psi = g.psi
    return s


def scheme_amfrw2(nu: float | None = None) -> L.AmfScheme:
    s = L.AmfScheme()
    L.check(L.lib().amf_scheme_amfrw2(C.byref(s)))
    if nu is not None:
        s.nu = nu
    return s


def scheme_theta_gs(theta: float, stages: int) -> L.AmfScheme:
    """theta-method with `stages` Gauss-Seidel sweeps as a W-method (W = P)."""
    s = L.AmfScheme()
    L.check(L.lib().amf_scheme_theta_gs(float(theta), int(stages), C.byref(s)))
    return s


def scheme_generic(a, q, b, theta: float, nu: float, w_matrix: int = L.W_AMF) -> L.AmfScheme:
    """A W-method table: a[r][j], q[r][j] for j < r, b[r]; W the AMF W or the lower triangle P."""
    s = L.AmfScheme()
    s.struct_size = C.sizeof(L.AmfScheme)
    s.stages = len(b)
    for r in range(len(b)):
        s.b[r] = b[r]
        for j in range(r):
            s.a[r * L.MAX_STAGES + j] = a[r][j]
            s.q[r * L.MAX_STAGES + j] = q[r][j]
    s.theta = theta
    s.nu = nu
    s.w_matrix = w_matrix
    return s


def _stream(stream=None) -> C.c_void_p:
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


class StaticPlan:
    """An unbound plan for amf_solve_static: host tables only; each price() call runs the whole
    solve in the library's static per-GPU workspace (no device allocation by the library or here,
    apart from the output tensor the caller may pass in)."""

    def __init__(self, problems: Sequence[Problem], grid: GridSpec, steps: int, precision: str = "fp64",
                 richardson: bool = False, scheme: L.AmfScheme | None = None):
        lib = L.lib()
        self.problems = list(problems)
        n = len(self.problems)
        arr = (L.AmfProblem * n)(*[problem_struct(p) for p in self.problems])
        gs = grid_struct(grid)
        sc = scheme if scheme is not None else scheme_amfrw2()
        h = C.c_void_p()
        L.check(lib.amf_plan_create(arr, n, C.byref(gs), C.byref(sc), L.FP64 if precision == "fp64" else L.FP32,
                                    int(steps), 1 if richardson else 0, C.byref(h)))
        self._h = h

    def price(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        assert out.dtype == torch.float64 and out.numel() >= len(self.problems) and out.is_contiguous()
        L.check(L.lib().amf_solve_static(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.lib().amf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A bound plan: problems x component grids, the workspace on `device`, and the solve calls."""

    def __init__(self, problems: Sequence[Problem], grid: GridSpec, steps: int, precision: str = "fp64",
                 richardson: bool = False, scheme: L.AmfScheme | None = None, device: str = "cuda:0"):
        lib = L.lib()
        self.problems = list(problems)
        n = len(self.problems)
        arr = (L.AmfProblem * n)(*[problem_struct(p) for p in self.problems])
        gs = grid_struct(grid)
        sc = scheme if scheme is not None else scheme_amfrw2()
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        prec = L.FP64 if precision == "fp64" else L.FP32
        h = C.c_void_p()
        L.check(lib.amf_plan_create(arr, n, C.byref(gs), C.byref(sc), prec, int(steps),
                                    1 if richardson else 0, C.byref(h)))
        self._h = h
        self.info = L.AmfPlanInfo()
        L.check(lib.amf_plan_info_get(h, C.byref(self.info)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(self.info.workspace_bytes) + 256, dtype=torch.uint8,
                                     device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        with torch.cuda.device(self.device):
            L.check(lib.amf_plan_bind(h, C.c_void_p(base + self._ws_off), int(self.info.workspace_bytes),
                                      _stream()))

    # -- metadata -------------------------------------------------------------------------------
    @property
    def n_units(self) -> int:
        return int(self.info.n_units)

    @property
    def inner_points(self) -> int:
        return int(self.info.inner_points)

    @property
    def vector_len(self) -> int:
        """Elements of one grid vector (inner points of all units plus alignment padding)."""
        return int(self.info.vector_bytes) // (8 if self.dtype == torch.float64 else 4)

    @property
    def stage_updates(self) -> int:
        return int(self.info.stage_updates_per_solve)

    def unit(self, u: int):
        prob = C.c_int32()
        lv = (C.c_int32 * L.MAX_D)()
        cf = C.c_double()
        off = C.c_int64()
        L.check(L.lib().amf_unit_info(self._h, int(u), C.byref(prob), lv, C.byref(cf), C.byref(off)))
        d = int(self.info.d)
        return dict(problem=prob.value, levels=[lv[i] for i in range(d)], coef=cf.value, offset=off.value)

    def units(self) -> List[dict]:
        return [self.unit(u) for u in range(self.n_units)]

    # -- calls ----------------------------------------------------------------------------------
    def init(self, stream=None):
        L.check(L.lib().amf_init(self._h, _stream(stream)))

    def time_step(self, n: int, stream=None):
        L.check(L.lib().amf_time_step(self._h, int(n), _stream(stream)))

    def solve(self, stream=None):
        L.check(L.lib().amf_solve(self._h, _stream(stream)))

    def use_graph(self, on: bool = True):
        L.check(L.lib().amf_graph_enable(self._h, 1 if on else 0))

    def combine(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(len(self.problems), dtype=torch.float64, device=self.device)
        L.check(L.lib().amf_combine(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def combine_checked(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """combine(), then wait and raise AmfError(AMF_E_NUMERIC) if a price is not finite."""
        if out is None:
            out = torch.empty(len(self.problems), dtype=torch.float64, device=self.device)
        L.check(L.lib().amf_combine_checked(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def unit_values(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n_units, dtype=torch.float64, device=self.device)
        L.check(L.lib().amf_unit_values(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def state(self, stream=None) -> torch.Tensor:
        """The current solution Y (inner-node layout of all units, plan precision), as a copy."""
        out = torch.empty(self.vector_len, dtype=self.dtype, device=self.device)
        L.check(L.lib().amf_state_read(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def apply_operator(self, x: torch.Tensor, increment: bool, scale: float = 1.0, stream=None) -> torch.Tensor:
        assert x.dtype == self.dtype and x.numel() == self.vector_len and x.is_contiguous()
        out = torch.empty_like(x)
        L.check(L.lib().amf_apply_operator(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                           1 if increment else 0, float(scale), _stream(stream)))
        return out

    def axis_solve(self, axis: int, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        assert x.dtype == self.dtype and x.numel() == self.vector_len and x.is_contiguous()
        if out is None:
            out = torch.zeros_like(x)          # the padding between units is never written
        L.check(L.lib().amf_axis_solve(self._h, int(axis), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def price(self, stream=None) -> torch.Tensor:
        self.solve(stream)
        return self.combine(stream=stream)

    def schedule(self) -> dict:
        sc = L.AmfSchedule()
        L.check(L.lib().amf_schedule_get(self._h, C.byref(sc)))
        return dict(stencil_nodes=sc.stencil_nodes, xcd_remap=sc.xcd_remap,
                    max_stencil_nodes=sc.max_stencil_nodes, resident=sc.resident,
                    resident_available=sc.resident_available, fuse_axis0=sc.fuse_axis0,
                    fuse_max_axis0=sc.fuse_max_axis0, march=sc.march, march_available=sc.march_available)

    def fuse_allowed(self, stencil_nodes: int) -> bool:
        """Whether the operator launches can also solve axis 0 at this many nodes per thread: the
        fused solve runs every unit at stencil_nodes (at most the shortest axis-0 line) and takes
        whole axis-0 lines of at most 256 * stencil_nodes and 1024 rows."""
        if not hasattr(self, "_min_m0"):
            self._min_m0 = min(1 << u["levels"][0] for u in self.units())
        m0 = self.schedule()["fuse_max_axis0"]
        return 2 <= stencil_nodes <= self._min_m0 and 256 * stencil_nodes >= m0 and m0 <= 1024

    def set_schedule(self, stencil_nodes: int | None = None, xcd_remap: int | None = None,
                     resident: int | None = None, fuse_axis0: int | None = None, march: int | None = None):
        """Change launch knobs; unspecified ones keep their value (fuse_axis0 is switched off when
        a new stencil_nodes does not allow it, or the marching operator is chosen, and it was not
        given)."""
        cur = self.schedule()
        sc = L.AmfSchedule()
        sc.struct_size = C.sizeof(L.AmfSchedule)
        sc.stencil_nodes = cur["stencil_nodes"] if stencil_nodes is None else int(stencil_nodes)
        sc.xcd_remap = cur["xcd_remap"] if xcd_remap is None else int(xcd_remap)
        sc.resident = cur["resident"] if resident is None else int(resident)
        sc.march = cur["march"] if march is None else int(march)
        if fuse_axis0 is None:
            sc.fuse_axis0 = cur["fuse_axis0"] if self.fuse_allowed(sc.stencil_nodes) and not sc.march else 0
        else:
            sc.fuse_axis0 = int(fuse_axis0)
        L.check(L.lib().amf_schedule_set(self._h, C.byref(sc)))

    def profile_begin(self):
        L.check(L.lib().amf_profile_begin(self._h))

    def profile_end(self) -> dict:
        """Per kernel class: launches, summed event milliseconds and algorithmic bytes."""
        arr = (L.AmfKernelStat * L.K_COUNT)()
        L.check(L.lib().amf_profile_end(self._h, arr))
        return {L.K_NAMES[s.kernel]: dict(launches=int(s.launches), ms=float(s.total_ms),
                                          algo_bytes=float(s.algo_bytes)) for s in arr}

    def close(self):
        if getattr(self, "_h", None):
            L.lib().amf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for(workload: dict, precision: str = "fp64", **kw) -> Plan:
    return Plan(workload["problems"], workload["grid"], workload["steps"], precision=precision,
                richardson=kw.pop("richardson", workload.get("richardson", False)), **kw)
