"""ctypes declarations for libctpd.so (argument marshalling only).

The structures mirror include/ctpd.h field by field.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_uint32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctpd.so")

CT_OK = 0
ERRORS = {-1: "CT_E_INVALID", -2: "CT_E_UNSUPPORTED", -3: "CT_E_DEVICE",
          -4: "CT_E_NONFINITE", -5: "CT_E_DIVERGED", -6: "CT_E_STATE"}
CT_FLAG_VALIDATE = 1
CT_FLAG_NONNEG = 2
CT_METHOD_SHIFT = 4
METHODS = {"pdrqs1": 0, "richardson": 1, "cp": 2, "pdrqs2": 3, "admm": 4, "pdrqs3": 5}
FITS = {"standard": 0, "weighted": 1, "ignore": 2, "everywhere": 3, "hard": 4}
PRECONDS = {"invnorm": 0, "impulse": 1, "circulant": 2}
CT_PRECOND_SHIFT = 8


class CtGeom(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_angles", c_int32), ("n_bins", c_int32),
                ("h", c_double), ("ds", c_double)]


class CtProblem(ctypes.Structure):
    _fields_ = [("sino", c_void_p), ("mask", c_void_p), ("bound", c_void_p),
                ("bound_scalar", c_float), ("pad_", c_float), ("lambda_", c_double)]


class CtParams(ctypes.Structure):
    _fields_ = [("sigma", c_double), ("tau", c_double), ("eps", c_double), ("c", c_double),
                ("c_safety", c_double), ("beta", c_double), ("k_max", c_int32),
                ("gap_every", c_int32), ("power_iters", c_int32), ("flags", c_uint32),
                ("start_norm", c_void_p), ("start_precond", c_void_p),
                ("bp_slices", c_int32), ("bp_kernel", c_int32), ("tv_blocks", c_int32),
                ("options", c_uint32), ("tune_cache", c_char_p), ("fwd_walk", c_int32)]


class CtPlanOpts(ctypes.Structure):
    _fields_ = [("bp_kernel", c_int32), ("fwd_angles_per_walk", c_int32)]


# backprojector kernels (ct_plan_opts.bp_kernel, ct_params.bp_kernel)
BP_KERNELS = {"auto": -1, "one_angle": 0, "pairs4": 4, "pairs8": 8}
# ct_params.options bits
CT_OPT_NO_TUNE = 1
CT_OPT_NO_DEFER = 2
CT_OPT_SEPARATE_TV = 4
CT_OPT_NO_GRAPH = 8


# name -> (restype, argtypes)
SIGNATURES = {
    "ct_version": (c_int32, []),
    "ct_last_error": (c_char_p, []),
    "ct_plan_create": (c_int32, [POINTER(CtGeom), c_void_p, POINTER(c_void_p)]),
    "ct_plan_create_ex": (c_int32, [POINTER(CtGeom), c_void_p, POINTER(CtPlanOpts),
                                    POINTER(c_void_p)]),
    "ct_plan_check_ex": (c_int32, [POINTER(CtGeom), c_void_p, POINTER(CtPlanOpts),
                                   POINTER(ctypes.c_int64)]),
    "ct_solver_tuning": (c_int32, [c_void_p, POINTER(c_int32)]),
    "ct_plan_destroy": (c_int32, [c_void_p]),
    "ct_plan_layout": (c_int32, [c_void_p, POINTER(c_int32)]),
    "ct_radon_fwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ct_d0_estimate": (c_int32, [c_void_p, c_void_p, c_float, c_int32, c_float, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p]),
    "ct_radon_adj": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ct_grad": (c_int32, [c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    "ct_div": (c_int32, [c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    "ct_precond_create": (c_int32, [c_int32, c_double, c_double, c_double, c_double,
                                    POINTER(c_void_p)]),
    "ct_precond_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ct_precond_destroy": (c_int32, [c_void_p]),
    "ct_prox_sino": (c_int32, [c_int32, c_int32, c_void_p, c_double, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p]),
    "ct_tv_project": (c_int32, [c_int32, c_void_p, c_double, c_void_p, c_void_p]),
    "ct_power_norm": (c_int32, [c_void_p, c_int32, c_void_p, POINTER(c_double), c_void_p]),
    "ct_power_norm_noalloc": (c_int32, [c_void_p, c_int32, c_void_p, POINTER(c_double),
                                        c_void_p]),
    "ct_valu_probe": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "ct_copy_probe": (c_int32, [c_void_p, c_void_p, ctypes.c_int64, c_int32, c_void_p]),
    "ct_params_default": (None, [POINTER(CtParams)]),
    "ct_solver_create": (c_int32, [c_void_p, POINTER(CtProblem), POINTER(CtParams), c_void_p,
                                   POINTER(c_void_p)]),
    "ct_solver_create_batch": (c_int32, [c_void_p, POINTER(CtProblem), c_int32,
                                         POINTER(CtParams), c_void_p, POINTER(c_void_p)]),
    "ct_solver_destroy": (c_int32, [c_void_p]),
    "ct_solver_layout": (c_int32, [c_void_p, POINTER(c_int32)]),
    "ct_solver_info": (c_int32, [c_void_p, POINTER(c_double)]),
    "ct_objective": (c_int32, [c_void_p, POINTER(CtProblem), c_void_p, POINTER(c_double),
                               c_void_p]),
    "ct_plan_check": (c_int32, [POINTER(CtGeom), c_void_p, POINTER(ctypes.c_int64)]),
    "ct_pd_step": (c_int32, [c_void_p, c_int32, c_void_p]),
    "ct_solver_set_fit": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "ct_solver_set_admm": (c_int32, [c_void_p, c_int32, c_double]),
    "ct_pd_step_timed": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_void_p]),
    "ct_state_export": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ct_state_import": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ct_state_export_ubar": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ct_state_import_ubar": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ct_gap": (c_int32, [c_void_p, POINTER(c_double), c_void_p]),
    "ct_reconstruct": (c_int32, [c_void_p, POINTER(CtProblem), POINTER(CtParams), c_void_p,
                                 POINTER(c_double), c_int32, c_void_p]),
    "ct_unrolled_forward": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_void_p), c_void_p]),
    "ct_unrolled_backward": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                       c_void_p]),
    "ct_tape_destroy": (c_int32, [c_void_p]),
    "ct_group_create": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p)]),
    "ct_group_step": (c_int32, [c_void_p, c_int32, c_void_p]),
    "ct_group_destroy": (c_int32, [c_void_p]),
    "ct_reconstruct_batched": (c_int32, [c_int32, POINTER(c_void_p), POINTER(CtProblem),
                                         POINTER(CtParams), POINTER(c_void_p),
                                         POINTER(c_double), c_int32, c_void_p]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libctpd.so and declare every entry point; raises if it is missing."""
    if not os.path.exists(path):
        raise ImportError(
            f"{path} not found: the HIP library is not built (run "
            "`python paper_1810_03275_amd/build.py` or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
