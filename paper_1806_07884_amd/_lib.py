"""ctypes declarations of librbf's C-ABI (see include/rbf.h).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any step.  RBF_LIBRARY=checked in the environment
loads the checked build (librbf_checked.so: device index checks) instead.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librbf.so")
CHECKED_LIB_PATH = os.path.join(_PKG, "librbf_checked.so")

RBF_OK = 0
RBF_WARN_MAXITER = 1
RBF_WARN_FALLBACK = 2
RBF_ERR_INVALID = -1
RBF_ERR_NONFINITE = -2
RBF_ERR_SINGULAR = -3
RBF_ERR_BREAKDOWN = -4
RBF_ERR_HIP = -5
RBF_ERR_OOM = -6

KERNEL = {"cg_iter": 0, "cg_iter_batch": 1, "assemble": 2}
PLAN_NO_STAGING = 1
PLAN_ROW_ASSEMBLY = 2
MLP_PARAMS = 5313
MLP_INPUTS = 16
MAX_RADII = 8
PHI = {"w30": 0, "w31": 1, "w32": 2, "w33": 3}
PREC = {"fp64": 0, "fp32": 1}

c_dp = ctypes.POINTER(ctypes.c_double)


class PlanDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_points", ctypes.c_int64),
                ("n_centers", ctypes.c_int64), ("points", ctypes.c_void_p),
                ("centers", ctypes.c_void_p), ("rho", ctypes.c_double),
                ("rho_per_center", ctypes.c_void_p), ("min_support", ctypes.c_int32),
                ("lambda_rel", ctypes.c_double), ("polynomial", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("grid", ctypes.c_int32 * 3),
                ("n_points", ctypes.c_int64), ("n_centers", ctypes.c_int64),
                ("n_points_in_box", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("nnz_upper", ctypes.c_int64), ("nnz_full", ctypes.c_int64),
                ("density", ctypes.c_double), ("support_total", ctypes.c_int64),
                ("support_max", ctypes.c_int32), ("row_max", ctypes.c_int32),
                ("cell_size", ctypes.c_double), ("solver_entries", ctypes.c_int64),
                ("solver_col_bytes", ctypes.c_int32), ("solver_lanes", ctypes.c_int32),
                ("n_poly", ctypes.c_int32), ("solver_staged", ctypes.c_int32),
                ("assembly_tiles", ctypes.c_int32), ("tile_window", ctypes.c_int32),
                ("solver_rows_sorted", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class StreamDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_centers", ctypes.c_int64),
                ("centers", ctypes.c_void_p), ("rho", ctypes.c_double),
                ("rho_per_center", ctypes.c_void_p), ("min_support", ctypes.c_int32),
                ("lambda_rel", ctypes.c_double), ("phi", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_chunk", ctypes.c_int64),
                ("flags", ctypes.c_uint32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("warm_start", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("reliable_delta", ctypes.c_double), ("stall_limit", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("reliable_updates", ctypes.c_int64),
                ("rel_residual", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("precision", ctypes.c_int32), ("status", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", ctypes.c_void_p)]


# exported symbol -> (restype, argtypes); also the list the load test checks
SIGNATURES = {
    "rbf_fit_plan": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.POINTER(Allocator),
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanStats)]),
    "rbf_plan_pattern": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "rbf_assemble": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p]),
    "rbf_system_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "rbf_poly_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "rbf_set_values": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.POINTER(SolveOpts), ctypes.c_void_p,
                                       ctypes.POINTER(SolveInfo)]),
    "rbf_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SolveOpts), ctypes.c_void_p,
                                 ctypes.POINTER(SolveInfo)]),
    "rbf_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_double)]),
    "rbf_stream_begin": (ctypes.c_int, [ctypes.POINTER(StreamDesc), ctypes.POINTER(Allocator),
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_stream_add": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32]),
    "rbf_stream_finish": (ctypes.c_int, [ctypes.c_void_p]),
    "rbf_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rbf_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]),
    "rbf_plan_destroy": (None, [ctypes.c_void_p]),
    "rbf_density_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p]),
    "rbf_block_sq_err": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_radius_broadcast": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_void_p]),
    "rbf_mlp_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_mlp_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_mlp_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_mlp_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_float, ctypes.c_void_p]),
    "rbf_mlp_infer_bf16": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p]),
    "rbf_mlp_set_input_scaling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "rbf_mlp_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "rbf_mlp_load_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "rbf_mlp_destroy": (None, [ctypes.c_void_p]),
    "rbf_solve_lsqr": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SolveOpts), ctypes.c_void_p,
                                      ctypes.POINTER(SolveInfo)]),
    "rbf_eval_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double)]),
    "rbf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rbf_last_error": (ctypes.c_char_p, []),
    "rbf_build_checked": (ctypes.c_int, []),
}

_lib = None


def load(path: str) -> ctypes.CDLL:
    """A handle on the library at path with the C-ABI's signatures set;
    raises when it was not built."""
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1806_07884_amd.build)")
    handle = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    return handle


def lib() -> ctypes.CDLL:
    """The loaded librbf.so (librbf_checked.so with RBF_LIBRARY=checked)."""
    global _lib
    if _lib is None:
        _lib = load(CHECKED_LIB_PATH if os.environ.get("RBF_LIBRARY") == "checked"
                    else LIB_PATH)
    return _lib


def use(handle: ctypes.CDLL) -> ctypes.CDLL:
    """Makes handle (from load) the library every later call goes through;
    returns the previous one.  A plan must be used and destroyed through the
    library that made it."""
    global _lib
    prev = lib()
    _lib = handle
    return prev


class RbfError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.rbf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.rbf_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise RbfError(status, where)
    return status
