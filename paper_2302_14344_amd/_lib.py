"""ctypes binding of libsubadmm.so (the C ABI in include/subadmm.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
Importing this module fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsubadmm.so")

OK = 0
E_ARG, E_NOT_SPD, E_NONFINITE, E_DEVICE, E_WORKSPACE, E_STATE = -1, -2, -3, -4, -5, -6
IF_EQUALITY, IF_CONTACT, IF_HARD_INEQ, IF_SOFT = 0, 1, 2, 3
F32, F64 = 0, 1
WARM_COLD, WARM_PREV, WARM_GIVEN, WARM_LEARNED = 0, 1, 2, 3
CONTACT_IN, CONTACT_OUT, JOINT_IN, JOINT_OUT = 12, 6, 27, 15

EXPORTS = (
    "subadmm_setup", "subadmm_get_sizes", "subadmm_rigid_set_model", "subadmm_workspace_bytes",
    "subadmm_bind", "subadmm_solve", "subadmm_rigid_assemble", "subadmm_rigid_step",
    "subadmm_read_stats", "subadmm_copy_beta", "subadmm_check", "subadmm_destroy", "subadmm_last_error",
    "subadmm_reset_totals", "subadmm_timing_begin", "subadmm_timing_end", "subadmm_set_option",
    "subadmm_mlp_create", "subadmm_mlp_param_count", "subadmm_mlp_workspace_bytes", "subadmm_mlp_bind",
    "subadmm_mlp_set_params", "subadmm_mlp_get_params", "subadmm_mlp_forward", "subadmm_mlp_backward",
    "subadmm_mlp_adam", "subadmm_mlp_destroy", "subadmm_mlp_last_error",
    "subadmm_set_warm_model", "subadmm_warm_class_counts", "subadmm_set_recording", "subadmm_get_warm",
    "subadmm_set_warm", "subadmm_mlp_set_input_affine",
    "subadmm_fem_set_model", "subadmm_fem_assemble", "subadmm_fem_step", "subadmm_fem_step_graph",
    "subadmm_rigid_step_graph",
    "subadmm_fem_loop_form", "subadmm_solve_scratch", "subadmm_rigid_steps",
    "subadmm_set_scene_order", "subadmm_rigid_set_links", "subadmm_constraint_error",
    "subadmm_fem_block_precision", "subadmm_mlp_gather_rows", "subadmm_mlp_infer",
)
OPT_FACTOR_FP64 = 1
OPT_TEAM_KERNEL = 2
OPT_LEARNED_BUDGET = 3
OPT_FACTOR_STREAMS = 4
OPT_FEM_RESIDENT = 5
OPT_SPLIT_ROWS = 6
OPT_CONTACT_MODEL = 7
OPT_LARGE_PATH = 8
OPT_BOYD_RESIDUALS = 9
OPT_FEM_KAPPA_MAX = 10
OPT_IMPULSE_OUTPUT = 11
MAX_MEMBERS = 4
ERR_LAWS, ERR_SOFT = 7, 8
K_ASSEMBLE, K_FACTOR, K_LOOP, K_ADVANCE, K_STEPS, K_WARM, NUM_KERNELS = 0, 1, 2, 3, 4, 5, 6
SCRATCH_BYTES = 32 << 20


class Subsystem(C.Structure):
    _fields_ = [("n_dof", C.c_int32), ("scene", C.c_int32)]


class Interface(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_sub", C.c_int32), ("sub", C.c_int32 * MAX_MEMBERS),
                ("mu", C.c_double), ("k", C.c_double), ("alpha", C.c_double)]


class Sizes(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_slot", C.c_int64), ("n_rows", C.c_int64), ("n_A", C.c_int64),
                ("n_J", C.c_int64), ("n_sub", C.c_int32), ("n_if", C.c_int32), ("n_scene", C.c_int32),
                ("max_dof", C.c_int32), ("max_slot_sub", C.c_int32), ("max_slot_scene", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("theta", C.c_double), ("r_theta", C.c_double),
                ("iters_total", C.c_int64), ("unconverged_total", C.c_int64), ("fallback_total", C.c_int64),
                ("r_prim", C.c_double), ("r_dual", C.c_double)]


class SubadmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsubadmm error {code}: {msg}")
        self.code = code


_LIB = None
vp = C.c_void_p
i32 = C.c_int32
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    # PyTorch ships its own HIP runtime; load it first so that the library binds to the
    # same runtime instance (one device context per process).
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    L.subadmm_setup.argtypes = [C.POINTER(Subsystem), i32, C.POINTER(Interface), i32, C.c_double, i32, C.POINTER(vp)]
    L.subadmm_get_sizes.argtypes = [vp, C.POINTER(Sizes)]
    L.subadmm_rigid_set_model.argtypes = [vp, i32, i32p, i32p, f64p, f64p, i32, i32p, f64p, f64p, f64p, i32p,
                                          i32, i32p, f64p, i32p, C.c_double, C.c_double]
    L.subadmm_workspace_bytes.argtypes = [vp]
    L.subadmm_workspace_bytes.restype = C.c_size_t
    L.subadmm_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.subadmm_solve.argtypes = [vp, vp, vp, vp, vp, i32, C.c_double, i32, vp, vp, vp, vp, vp, vp]
    L.subadmm_solve_scratch.argtypes = [vp, vp, vp, vp, vp, vp, i32, C.c_double, i32, vp, vp, vp, vp, vp, vp,
                                        C.POINTER(Stats)]
    L.subadmm_rigid_assemble.argtypes = [vp, vp, vp, vp, vp, C.c_double, vp, vp, vp, vp]
    L.subadmm_rigid_step.argtypes = [vp, vp, vp, vp, vp, C.c_double, i32, C.c_double, i32, vp, vp]
    L.subadmm_rigid_step_graph.argtypes = [vp, vp, vp, vp, vp, C.c_double, i32, C.c_double, i32, vp, vp]
    L.subadmm_fem_step_graph.argtypes = [vp, vp, vp, C.c_double, i32, C.c_double, i32, vp, vp]
    L.subadmm_rigid_steps.argtypes = [vp, vp, vp, vp, vp, C.c_double, i32, i32, C.c_double, i32, vp, vp]
    L.subadmm_set_scene_order.argtypes = [vp, i32p]
    L.subadmm_rigid_set_links.argtypes = [vp, i32, i32p, i32p, f64p, f64p, i32p, i32p, f64p, f64p]
    L.subadmm_constraint_error.argtypes = [vp, vp, vp, vp, vp, i32, f64p]
    L.subadmm_read_stats.argtypes = [vp, C.POINTER(Stats)]
    L.subadmm_copy_beta.argtypes = [vp, vp]
    L.subadmm_reset_totals.argtypes = [vp]
    L.subadmm_set_option.argtypes = [vp, i32, C.c_int64]
    L.subadmm_timing_begin.argtypes = [vp, i32]
    L.subadmm_timing_end.argtypes = [vp, f64p, i32p]
    L.subadmm_check.argtypes = [vp]
    L.subadmm_destroy.argtypes = [vp]
    L.subadmm_destroy.restype = None
    L.subadmm_last_error.argtypes = [vp]
    L.subadmm_last_error.restype = C.c_char_p
    fp = C.POINTER(C.c_float)
    L.subadmm_fem_set_model.argtypes = [vp, i32, f64p, i32, i32p, f64p, f64p, C.c_double, i32p, C.c_double,
                                        C.c_double]
    L.subadmm_fem_assemble.argtypes = [vp, vp, vp, C.c_double, vp, vp, vp, vp]
    L.subadmm_fem_step.argtypes = [vp, vp, vp, C.c_double, i32, C.c_double, i32, vp, vp]
    L.subadmm_fem_loop_form.argtypes = [vp, i32p]
    L.subadmm_fem_block_precision.argtypes = [vp, vp, vp]
    L.subadmm_set_warm_model.argtypes = [vp, i32, vp]
    L.subadmm_warm_class_counts.argtypes = [vp, i32p, i32p]
    L.subadmm_set_recording.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.subadmm_get_warm.argtypes = [vp, vp, vp]
    L.subadmm_set_warm.argtypes = [vp, vp, vp]
    L.subadmm_mlp_create.argtypes = [i32, i32p, i32, C.POINTER(vp)]
    L.subadmm_mlp_param_count.argtypes = [vp]
    L.subadmm_mlp_param_count.restype = C.c_int64
    L.subadmm_mlp_workspace_bytes.argtypes = [vp]
    L.subadmm_mlp_workspace_bytes.restype = C.c_size_t
    L.subadmm_mlp_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.subadmm_mlp_set_params.argtypes = [vp, vp]
    L.subadmm_mlp_get_params.argtypes = [vp, vp]
    L.subadmm_mlp_set_input_affine.argtypes = [vp, vp, vp]
    L.subadmm_mlp_forward.argtypes = [vp, i32, vp, vp]
    L.subadmm_mlp_backward.argtypes = [vp, i32, vp, vp, vp, vp]
    L.subadmm_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, i32]
    L.subadmm_mlp_gather_rows.argtypes = [vp, vp, C.c_int64, i32, vp, i32, vp]
    L.subadmm_mlp_infer.argtypes = [vp, i32, vp, vp]
    L.subadmm_mlp_destroy.argtypes = [vp]
    L.subadmm_mlp_destroy.restype = None
    L.subadmm_mlp_last_error.argtypes = [vp]
    L.subadmm_mlp_last_error.restype = C.c_char_p
    no_status = ("subadmm_workspace_bytes", "subadmm_destroy", "subadmm_last_error", "subadmm_mlp_param_count",
                 "subadmm_mlp_workspace_bytes", "subadmm_mlp_destroy", "subadmm_mlp_last_error")
    for name in EXPORTS:
        if name not in no_status:
            getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def check(rc, handle=None):
    if rc != OK:
        msg = lib().subadmm_last_error(handle)
        raise SubadmmError(rc, msg.decode() if msg else "")


def check_mlp(rc, handle=None):
    if rc != OK:
        msg = lib().subadmm_mlp_last_error(handle)
        raise SubadmmError(rc, msg.decode() if msg else "")
