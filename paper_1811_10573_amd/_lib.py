"""ctypes declarations for libppals.so (the C ABI in include/ppals.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppals.so")

PPALS_OK = 0
PPALS_E_ARG = -1
PPALS_E_UNSUPPORTED = -2
PPALS_E_HIP = -3
PPALS_E_WORKSPACE = -4
PPALS_E_STATE = -5

PPALS_FP64, PPALS_FP32, PPALS_BF16 = 0, 1, 2
SWEEP_ALS, SWEEP_PP_INIT, SWEEP_PP_APPROX = 0, 1, 2
MAX_ORDER = 8
MAX_RANK = 128


class Desc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("tensor_dtype", ctypes.c_int32),
        ("level1_dtype", ctypes.c_int32),
        ("use_second_order", ctypes.c_int32),
        ("pp_build_levels", ctypes.c_int32),
        ("step_size", ctypes.c_double),
    ]


class SweepRecord(ctypes.Structure):
    _fields_ = [
        ("fit_est", ctypes.c_double),
        ("grad_norm", ctypes.c_double * MAX_ORDER),
        ("rel_change", ctypes.c_double * MAX_ORDER),
        ("chol_status", ctypes.c_int32 * MAX_ORDER),
        ("sweep_kind", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("ctrl_pred", ctypes.c_double),
        ("ctrl_true_err", ctypes.c_double),
        ("ctrl_leave", ctypes.c_int32),
        ("ctrl_fallback", ctypes.c_int32),
        ("chol_pivot", ctypes.c_int32 * MAX_ORDER),
        ("nonfinite", ctypes.c_int32 * MAX_ORDER),
    ]


RECORD_BYTES = ctypes.sizeof(SweepRecord)


class BatchProblem(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("rank", ctypes.c_int32)]


class BatchResult(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("converged_sweep", ctypes.c_int32),
        ("n_als", ctypes.c_int32),
        ("n_pp_init", ctypes.c_int32),
        ("n_pp_approx", ctypes.c_int32),
        ("done", ctypes.c_int32),
        ("chol_status", ctypes.c_int32 * 3),
        ("pad", ctypes.c_int32),
        ("fit", ctypes.c_double),
        ("normX2", ctypes.c_double),
        ("rel_change", ctypes.c_double * 3),
        ("time_to_converge_ms", ctypes.c_double),
    ]


class Controller(ctypes.Structure):
    _fields_ = [
        ("params", ctypes.c_void_p),
        ("hidden", ctypes.c_int32),
        ("check_period", ctypes.c_int32),
        ("log10_tau", ctypes.c_double),
        ("rho_cap", ctypes.c_double),
        ("fallback_factor", ctypes.c_double),
    ]

PROF_CLASSES = 8


class TuckerRecord(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("iters", ctypes.c_int32 * MAX_ORDER),
        ("converged", ctypes.c_int32 * MAX_ORDER),
        ("rr_status", ctypes.c_int32 * MAX_ORDER),
        ("pad", ctypes.c_int32),
        ("fit", ctypes.c_double),
        ("core_norm", ctypes.c_double),
        ("f_norm", ctypes.c_double),
        ("rel_change", ctypes.c_double * MAX_ORDER),
        ("ritz_residual", ctypes.c_double * MAX_ORDER),
        ("ms", ctypes.c_double),
    ]


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_ptrs = ctypes.POINTER(ctypes.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "ppals_last_error": (ctypes.c_char_p, []),
    "ppals_plan_create": (_i32, [ctypes.POINTER(Desc), ctypes.POINTER(_vp)]),
    "ppals_plan_destroy": (None, [_vp]),
    "ppals_workspace_bytes": (_sz, [_vp]),
    "ppals_plan_describe": (_i32, [_vp, ctypes.c_char_p, _sz]),
    "cp_als_sweep": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _dbl, _vp, _vp, _vp]),
    "pp_build_operators": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _vp]),
    "pp_sweep": (_i32, [_vp, _ptrs, _vp, _dbl, _vp, _vp, _vp]),
    "ppals_gram_solve_workspace_bytes": (_sz, [_i32, _i64]),
    "gram_solve": (_i32, [_i32, _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "gram_solve_noalloc": (_i32, [_i32, _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "ppals_norm2_workspace_bytes": (_sz, []),
    "ppals_tensor_norm2": (_i32, [_vp, _i32, _i64, _vp, _vp, _vp]),
    "ppals_cast_bf16": (_i32, [_vp, _vp, _i64, _vp]),
    "ppals_mttkrp": (_i32, [_vp, _vp, _vp, _ptrs, _i32, _vp, _vp, _vp]),
    "ppals_level1": (_i32, [_vp, _vp, _vp, _ptrs, _u32, _vp, _vp, _vp]),
    "ppals_pp_rhs": (_i32, [_vp, _ptrs, _vp, _i32, _vp, _vp, _vp]),
    "ppals_get_operator": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp]),
    "ppals_exact_residual2": (_i32, [_vp, _vp, _ptrs, _vp, _vp, _vp]),
    "ppals_run": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _dbl, _vp, _vp, _dbl, _dbl, _i32,
                         ctypes.POINTER(_i32), ctypes.POINTER(SweepRecord),
                         ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_i32), _vp]),
    "ppals_mlp_forward": (_i32, [_vp, _i32, _i32, _vp, _i64, _vp, _vp, _vp]),
    "ppals_mlp_backward": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "ppals_mlp_adam": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, _vp]),
    "ppals_pp_rhs_error": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _vp, _vp, _vp]),
    "ppals_set_controller": (_i32, [_vp, ctypes.POINTER(Controller)]),
    "ppals_batch_create": (_i32, [ctypes.POINTER(BatchProblem), _i32, _i32, ctypes.POINTER(_vp)]),
    "ppals_batch_destroy": (None, [_vp]),
    "ppals_batch_workspace_bytes": (_sz, [_vp]),
    "ppals_batch_bind": (_i32, [_vp, _ptrs, _ptrs, _vp, _dbl, _dbl, _i32, _vp]),
    "ppals_batch_autotune": (_i32, [_vp, _vp, _i32, _vp]),
    "ppals_batch_sweep": (_i32, [_vp, _vp, _vp]),
    "ppals_batch_run": (_i32, [_vp, _vp, _i32, _i32, _vp]),
    "ppals_batch_results": (_i32, [_vp, _vp, ctypes.POINTER(BatchResult), _vp]),
    "ppals_batch_kind_log": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_uint8), _vp]),
    "ppals_batch_describe": (_i32, [_vp, ctypes.c_char_p, _sz]),
    "ppals_set_profiling": (_i32, [_vp, _i32]),
    "tucker_plan_create": (_i32, [_i32, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_vp)]),
    "tucker_plan_destroy": (None, [_vp]),
    "tucker_workspace_bytes": (_sz, [_vp]),
    "tucker_set_solver": (_i32, [_vp, _dbl, _i32, _i32]),
    "tucker_ttmc": (_i32, [_vp, _vp, _vp, _ptrs, _i32, _vp, _vp]),
    "tucker_factor_update": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(_i32),
                                    ctypes.POINTER(_dbl), _vp]),
    "tucker_hosvd": (_i32, [_vp, _vp, _vp, _ptrs, _ptrs, _vp, ctypes.POINTER(_i32), _vp]),
    "tucker_hosvd_interlaced": (_i32, [_vp, _vp, _vp, _ptrs, _ptrs, _vp, ctypes.POINTER(_i32),
                                       _vp]),
    "tucker_als_sweep": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _dbl, ctypes.POINTER(TuckerRecord), _vp]),
    "tucker_pp_build": (_i32, [_vp, _vp, _vp, _ptrs, _vp]),
    "tucker_pp_rhs": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "tucker_pp_sweep": (_i32, [_vp, _vp, _ptrs, _vp, _dbl, _i32, ctypes.POINTER(TuckerRecord), _vp]),
    "tucker_run": (_i32, [_vp, _vp, _vp, _ptrs, _vp, _dbl, _i32, _dbl, ctypes.POINTER(_i32), _i32,
                          ctypes.POINTER(TuckerRecord), ctypes.POINTER(_i32), _vp]),
    "ppals_get_profile": (_i32, [_vp, ctypes.POINTER(KernelStat), _i32, ctypes.POINTER(_i32), _i32]),
}

_LIB = None


class PPALSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ppals status {status}: {msg}")
        self.status = status


def load(path: str | None = None):
    """Load libppals.so (built in-tree by paper_1811_10573_amd.build); raise if absent."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def check(status: int):
    if status != PPALS_OK:
        msg = load().ppals_last_error().decode(errors="replace")
        raise PPALSError(status, msg)
