"""ctypes declarations of the C ABI in ``include/addk.h``.

Loading fails loudly (ImportError) when ``libaddk.so`` has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaddk.so")

ADDK_OK = 0
ADDK_ERR_INVALID_ARG = 1
ADDK_ERR_UNSUPPORTED = 2
ADDK_ERR_ACCURACY = 3
ADDK_ERR_OOM = 4
ADDK_ERR_HIP = 5

ADDK_GAUSSIAN = 1
ADDK_MATERN12 = 3
ADDK_MATERN32 = 5
ADDK_FP64 = 0
ADDK_FP32 = 1

ADDK_COEF_ANALYTIC = 0
ADDK_COEF_SAMPLED = 1
ADDK_TORUS_AUTO = 0
ADDK_TORUS_PAPER = 2
ADDK_NO_ACCURACY_CHECK = 4
ADDK_TILE_KERNELS_ONLY = 8
ADDK_VECTOR_ALU_ONLY = 16
ADDK_NEAR_FIELD = 32
ADDK_NSTAGES = 14
ADDK_KNOB_SPREAD_MFMA = 1
ADDK_KNOB_INTERP_DENSE_MFMA = 2
ADDK_KNOB_INTERP_TILE_MFMA = 4
ADDK_KNOB_ALL_MFMA = 7
ADDK_KNOB_SPREAD_SPLIT = 8
ADDK_KNOB_ALL = 15
ADDK_KNOB_SPARSE_ATOMIC = 16


class AddkPlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("P", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n_os", ctypes.c_int32), ("precision", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("err_estimate", ctypes.c_double),
                ("dense_points", ctypes.c_int64), ("tile_points", ctypes.c_int64),
                ("knobs", ctypes.c_uint32), ("tuned", ctypes.c_int32),
                ("n_sources", ctypes.c_int64), ("n_targets", ctypes.c_int64)]


_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "addk_plan_create": [ctypes.POINTER(_vp), _i64, _i32, _vp, _i64, _i32, _pi32, _pi32, _i32, _pd, _pd,
                         _i32, _i32, _d, _i32, _u32, _vp],
    "addk_matvec": [_vp, _i32, _vp, _i64, _vp, _i64, _vp],
    "addk_matvec_noalloc": [_vp, _i32, _vp, _i64, _vp, _i64, _vp],
    "addk_dmatvec": [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _i64, _vp],
    "addk_vjp": [_vp, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp],
    "addk_plan_update_params": [_vp, _pd, _pd, _vp],
    "addk_gsi": [_vp, _vp, _pd, _vp],
    "addk_gsi_indices": [_vp, _vp, _i32, _pi32, _pd, _pi32, _vp],
    "addk_cg": [_vp, _d, _i32, _vp, _i64, _vp, _i64, _d, _i32, _pi32, _pd, _vp],
    "addk_plan_create_targets": [ctypes.POINTER(_vp), _i64, _i64, _i32, _vp, _i64, _vp, _i64, _i32, _pi32, _pi32,
                                 _i32, _pd, _pd, _i32, _i32, _d, _i32, _u32, _vp],
    "addk_plan_query": [_vp, ctypes.POINTER(AddkPlanInfo), _pd, _pd, _pi32],
    "addk_plan_destroy": [_vp],
    "addk_batch_create": [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _pi64,
                          ctypes.POINTER(_vp), _pi64, _vp],
    "addk_batch_launch": [_vp, _vp],
    "addk_plan_autotune": [_vp, _i32, _i32, _i32, ctypes.POINTER(_u32), _vp],
    "addk_batch_autotune": [_vp, _i32, ctypes.POINTER(_u32), _vp],
    "addk_tune_cache_lookup": [_vp, _i32, _i32, ctypes.POINTER(_u32), _pi32],
    "addk_plan_set_knobs": [_vp, _u32],
    "addk_tune_cache_clear": [],
    "addk_batch_run_eager": [_vp, _vp],
    "addk_batch_destroy": [_vp],
    "addk_plan_profile": [_vp, _i32],
    "addk_plan_profile_read": [_vp, _pd, _pi32],
    "addk_stage_name": [_i32],
    "addk_torus_period": [_i32, _d, _d, _i32, _u32, _i32, _pd],
    "addk_window_ft": [_i32, _i32, _d, _d, _pd],
    "addk_choose_n": [_i32, _d, _d, _i32, _d, _d, _pi32, _pd],
    "addk_choose_n_windows": [_i32, _i64, _i32, _vp, _i64, _i32, _pi32, _pi32, _pd, _i32, _d, _d, _pi32, _pd, _vp],
    "addk_status_string": [_i32],
    "addk_last_error": [],
    "addk_version": [],
}


def load():
    """Load libaddk.so and declare its signatures (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libaddk.so is not built: run `python -m paper_2404_17344_amd.build` "
                          "(the package has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("addk_status_string", "addk_last_error", "addk_version",
                                               "addk_stage_name") else _i32
    _lib = lib
    return lib


class AddkError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.addk_status_string(status).decode()
        detail = lib.addk_last_error().decode()
        super().__init__("%s failed: %s (%s)" % (where, msg, detail))
        self.status = status


def check(status: int, where: str):
    if status != ADDK_OK:
        raise AddkError(status, where)
