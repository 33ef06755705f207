"""ctypes declarations of libamfrw's C ABI (include/amfrw.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamfrw.so")
ABI_VERSION = 2                       # AMF_ABI_VERSION of include/amfrw.h

MAX_D = 8
MAX_STAGES = 6
RHO_LD = MAX_D - 1

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP, E_NUMERIC, E_STATE = range(7)
FP64, FP32 = 0, 1
PAYOFF_CAPLET, PAYOFF_SWAPTION = 0, 1
BC_NEUMANN, BC_DIRICHLET = 0, 1
W_AMF, W_LOWER = 0, 1
STATIC_WORKSPACE_BYTES = 64 << 20
STATUS_NAMES = {0: "AMF_OK", 1: "AMF_E_INVALID", 2: "AMF_E_UNSUPPORTED", 3: "AMF_E_NOMEM",
                4: "AMF_E_HIP", 5: "AMF_E_NUMERIC", 6: "AMF_E_STATE"}


class AmfProblem(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("d", C.c_int32), ("payoff", C.c_int32),
                ("boundary", C.c_int32), ("beta", C.c_double), ("sigma", C.c_double),
                ("alpha", C.c_double * (MAX_D - 1)), ("phi", C.c_double * (MAX_D - 1)),
                ("tau", C.c_double * (MAX_D - 1)), ("rho", C.c_double * (RHO_LD * RHO_LD)),
                ("x_max", C.c_double * MAX_D), ("maturity", C.c_double), ("strike", C.c_double),
                ("x_eval", C.c_double * MAX_D), ("discount", C.c_double)]


class AmfScheme(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("stages", C.c_int32),
                ("a", C.c_double * (MAX_STAGES * MAX_STAGES)),
                ("q", C.c_double * (MAX_STAGES * MAX_STAGES)), ("b", C.c_double * MAX_STAGES),
                ("theta", C.c_double), ("nu", C.c_double), ("w_matrix", C.c_int32), ("reserved", C.c_int32)]


class AmfGridSpec(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("full_grid", C.c_int32),
                ("levels", C.c_int32 * MAX_D), ("n", C.c_int32), ("psi", C.c_int32)]


class AmfPlanInfo(C.Structure):
    _fields_ = [("n_problems", C.c_int64), ("n_units", C.c_int64), ("inner_points", C.c_int64),
                ("stage_updates_per_solve", C.c_int64), ("workspace_bytes", C.c_uint64),
                ("state_offset", C.c_uint64), ("vector_bytes", C.c_uint64), ("d", C.c_int32),
                ("precision", C.c_int32), ("n_steps", C.c_int32), ("richardson", C.c_int32)]


class AmfSchedule(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("stencil_nodes", C.c_int32), ("xcd_remap", C.c_int32),
                ("max_stencil_nodes", C.c_int32), ("resident", C.c_int32), ("resident_available", C.c_int32),
                ("fuse_axis0", C.c_int32), ("fuse_max_axis0", C.c_int32), ("march", C.c_int32),
                ("march_available", C.c_int32)]


class AmfKernelStat(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("reserved", C.c_int32), ("launches", C.c_int64),
                ("total_ms", C.c_double), ("algo_bytes", C.c_double)]


K_NAMES = ["init", "operator", "stage1", "stage2", "refine", "sweep_contig", "sweep_contig_long",
           "sweep_strided", "sweep_strided_long", "sweep_update", "sweep_update_long", "unit_values",
           "combine", "resident", "lincomb", "lower"]
# device kernel symbol of each class (template arguments omitted)
K_SYMBOLS = {"init": "k_node", "operator": "k_stencil<OP_F_PAYOFF>", "stage1": "k_stencil_vec<OP_STAGE1, R, FUSE>",
             "stage2": "k_stencil_vec<OP_STAGE2, R, FUSE>", "refine": "k_stencil_vec<OP_REFINE, R, FUSE>",
             "sweep_contig": "k_sweep_contig<false>", "sweep_contig_long": "k_sweep_contig<true>",
             "sweep_strided": "k_sweep_strided<EPI_STORE>",
             "sweep_strided_long": "k_sweep_strided_long<EPI_STORE, V>",
             "sweep_update": "k_sweep_strided<EPI_UPDATE>",
             "sweep_update_long": "k_sweep_strided_long<EPI_UPDATE, V>",
             "unit_values": "k_unit_values", "combine": "k_combine", "resident": "k_resident",
             "lincomb": "k_lincomb", "lower": "k_lower"}
K_COUNT = len(K_NAMES)


class AmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """Load libamfrw.so.  Fails loudly when the library has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libamfrw.so is not built (run python -m paper_2408_00559_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        st = C.c_int32
        L.amf_abi_version.restype = C.c_int32
        L.amf_last_error.restype = C.c_char_p
        L.amf_scheme_amfrw2.restype = st
        L.amf_scheme_amfrw2.argtypes = [C.POINTER(AmfScheme)]
        L.amf_scheme_theta_gs.restype = st
        L.amf_scheme_theta_gs.argtypes = [C.c_double, C.c_int32, C.POINTER(AmfScheme)]
        L.amf_plan_create.restype = st
        L.amf_plan_create.argtypes = [C.POINTER(AmfProblem), C.c_int32, C.POINTER(AmfGridSpec),
                                      C.POINTER(AmfScheme), C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(vp)]
        L.amf_plan_info_get.restype = st
        L.amf_plan_info_get.argtypes = [vp, C.POINTER(AmfPlanInfo)]
        L.amf_unit_info.restype = st
        L.amf_unit_info.argtypes = [vp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.amf_plan_bind.restype = st
        L.amf_plan_bind.argtypes = [vp, vp, C.c_uint64, vp]
        L.amf_init.restype = st
        L.amf_init.argtypes = [vp, vp]
        L.amf_time_step.restype = st
        L.amf_time_step.argtypes = [vp, C.c_int32, vp]
        L.amf_solve.restype = st
        L.amf_solve.argtypes = [vp, vp]
        L.amf_graph_enable.restype = st
        L.amf_graph_enable.argtypes = [vp, C.c_int32]
        L.amf_unit_values.restype = st
        L.amf_unit_values.argtypes = [vp, vp, vp]
        L.amf_combine.restype = st
        L.amf_combine.argtypes = [vp, vp, vp]
        L.amf_combine_checked.restype = st
        L.amf_combine_checked.argtypes = [vp, vp, vp]
        L.amf_solve_static.restype = st
        L.amf_solve_static.argtypes = [vp, vp, vp]
        L.amf_state_read.restype = st
        L.amf_state_read.argtypes = [vp, vp, vp]
        L.amf_apply_operator.restype = st
        L.amf_apply_operator.argtypes = [vp, vp, vp, C.c_int32, C.c_double, vp]
        L.amf_axis_solve.restype = st
        L.amf_axis_solve.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.amf_schedule_get.restype = st
        L.amf_schedule_get.argtypes = [vp, C.POINTER(AmfSchedule)]
        L.amf_schedule_set.restype = st
        L.amf_schedule_set.argtypes = [vp, C.POINTER(AmfSchedule)]
        L.amf_profile_begin.restype = st
        L.amf_profile_begin.argtypes = [vp]
        L.amf_profile_end.restype = st
        L.amf_profile_end.argtypes = [vp, C.POINTER(AmfKernelStat)]
        L.amf_plan_destroy.restype = None
        L.amf_plan_destroy.argtypes = [vp]
        _lib = L
    return _lib


def check(status: int):
    if status != OK:
        raise AmfError(status, lib().amf_last_error().decode())


EXPORTED = ["amf_abi_version", "amf_last_error", "amf_scheme_amfrw2", "amf_scheme_theta_gs", "amf_plan_create",
            "amf_plan_info_get", "amf_unit_info", "amf_plan_bind", "amf_init", "amf_time_step",
            "amf_solve", "amf_graph_enable", "amf_unit_values", "amf_combine", "amf_combine_checked",
            "amf_state_read", "amf_apply_operator",
            "amf_axis_solve", "amf_schedule_get", "amf_schedule_set", "amf_profile_begin", "amf_profile_end", "amf_plan_destroy",
            "amf_mlp_last_error", "amf_mlp_create", "amf_mlp_info_get", "amf_mlp_bind",
            "amf_mlp_set_normalization", "amf_mlp_params", "amf_mlp_grads", "amf_mlp_forward", "amf_mlp_infer",
            "amf_mlp_backward", "amf_mlp_train_step", "amf_mlp_destroy", "amf_mlp_set_router",
            "amf_price_or_fallback", "amf_solve_static"]
