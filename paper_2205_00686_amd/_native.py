"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every computation happens in the HIP library ``liblbm.so`` next to this file; if it is missing
the first use raises ``NativeLibraryMissing`` -- there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NUMERIC, LBM_E_STATE = 0, -1, -2, -3, -4, -5
LBM_FP32, LBM_FP64 = 0, 1
LBM_FREEZE_FLOW, LBM_NO_S, LBM_BGK = 1, 2, 8
LBM3D_PATH_FUSED, LBM3D_PATH_PER_NODE = 0, 1

# every symbol include/lbm.h declares
EXPORTS = (
    "lbm_params_default", "lbm_validate", "lbm_footprint_bytes", "lbm_create", "lbm_init", "lbm_step",
    "lbm_steps_done", "lbm_shape_count", "lbm_shape_info", "lbm_shape_fits", "lbm_set_shape", "lbm_get_shape",
    "lbm_set_tile_order", "lbm_get_tile_order",
    "lbm_sync", "lbm_read_fields", "lbm_vapour_rows", "lbm_vapour_components", "lbm_diagnostics", "lbm_set_diagnostics_interval",
    "lbm_read_diagnostics_log", "lbm_state_bytes", "lbm_save_state",
    "lbm_load_state", "lbm_read_state", "lbm_eos_coexistence", "lbm_critical_temperature", "lbm_destroy", "lbm_strerror",
    "lbm_last_error", "lbm_device_copy", "lbm_batch_footprint_bytes", "lbm_batch_create", "lbm_batch_set_budget", "lbm_batch_step",
    "lbm_batch_remaining", "lbm_batch_set_shape", "lbm_batch_get_shape", "lbm_batch_sync", "lbm_batch_destroy",
    "lbm_batch_create_noalloc", "lbm_batch_set_persistent", "lbm_batch_set_diagnostics_interval",
    "lbm3d_params_default", "lbm3d_validate", "lbm3d_footprint_bytes", "lbm3d_create", "lbm3d_init", "lbm3d_step",
    "lbm3d_sync", "lbm3d_read_fields", "lbm3d_diagnostics", "lbm3d_steps_done", "lbm3d_state_bytes",
    "lbm3d_save_state", "lbm3d_load_state", "lbm3d_destroy",
)


class NativeLibraryMissing(RuntimeError):
    pass


class Lbm3dParams(ctypes.Structure):
    """Mirror of lbm3d_params (include/lbm3d.h)."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("acentric", ctypes.c_double),
        ("G", ctypes.c_double),
        ("nu", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("sigma", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("cv", ctypes.c_double), ("wdot", ctypes.c_double), ("vs3", ctypes.c_double),
        ("thermal_box", ctypes.c_int32), ("z_chunk", ctypes.c_int32), ("T_box", ctypes.c_double),
        ("flags", ctypes.c_uint32), ("path", ctypes.c_uint32),
    ]


class LbmComponent(ctypes.Structure):
    """Mirror of lbm_component (include/lbm.h)."""
    _fields_ = [("root", ctypes.c_int32), ("area", ctypes.c_int32), ("y_min", ctypes.c_int32),
                ("y_max", ctypes.c_int32), ("x_min", ctypes.c_int32), ("x_max", ctypes.c_int32),
                ("y_sum", ctypes.c_int64)]


LBM_MAX_COMPONENTS = 4096


class LbmParams(ctypes.Structure):
    """Mirror of lbm_params (include/lbm.h)."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("precision", ctypes.c_int32), ("thermal_q", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("acentric", ctypes.c_double),
        ("G", ctypes.c_double),
        ("nu", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("cv", ctypes.c_double), ("wdot", ctypes.c_double), ("vs3", ctypes.c_double),
        ("vs4", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("rho_ave", ctypes.c_double),
        ("y_walls", ctypes.c_int32), ("thermal_box", ctypes.c_int32),
        ("T_box", ctypes.c_double), ("T_top", ctypes.c_double), ("T_bot", ctypes.c_double),
        ("hot_dT", ctypes.c_double), ("hot_x0", ctypes.c_double), ("hot_sigma", ctypes.c_double),
        ("theta_bot_deg", ctypes.c_double), ("theta_top_deg", ctypes.c_double),
        ("flags", ctypes.c_uint32), ("open_top", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load liblbm.so and declare the signatures of include/lbm.h."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one liblbm.so binds to,
    # so device pointers from torch allocations and streams are valid in the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(LbmParams)
    P3 = ctypes.POINTER(Lbm3dParams)
    vp, d, i32, i64, sz = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    st = ctypes.c_int
    sig = {
        "lbm_params_default": ([P, i32, i32], None),
        "lbm_validate": ([P], st),
        "lbm_footprint_bytes": ([P], sz),
        "lbm_create": ([P, vp, sz, vp, ctypes.POINTER(vp)], st),
        "lbm_init": ([vp, dp, dp, dp, dp], st),
        "lbm_step": ([vp, i64], st),
        "lbm_steps_done": ([vp], i64),
        "lbm_shape_count": ([i32], ctypes.c_int),
        "lbm_shape_info": ([i32, ctypes.c_int, ip, ip, ip, ip], st),
        "lbm_shape_fits": ([P, ctypes.c_int], ctypes.c_int),
        "lbm_set_shape": ([vp, ctypes.c_int], st),
        "lbm_get_shape": ([vp], ctypes.c_int),
        "lbm_set_tile_order": ([vp, ctypes.c_int], st),
        "lbm_get_tile_order": ([vp], ctypes.c_int),
        "lbm_sync": ([vp], st),
        "lbm_read_fields": ([vp, dp, dp, dp, dp], st),
        "lbm_vapour_rows": ([vp, d, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)], st),
        "lbm_vapour_components": ([vp, d, ctypes.c_int, ctypes.c_int, ctypes.POINTER(LbmComponent), ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)], st),
        "lbm_diagnostics": ([vp, dp, dp], st),
        "lbm_set_diagnostics_interval": ([vp, i64], st),
        "lbm_read_diagnostics_log": ([vp, ctypes.POINTER(ctypes.c_int64), dp, dp, ctypes.c_int, ip], st),
        "lbm_state_bytes": ([vp], sz),
        "lbm_save_state": ([vp, vp, sz], st),
        "lbm_load_state": ([vp, vp, sz], st),
        "lbm_read_state": ([vp, dp, dp, dp], st),
        "lbm_eos_coexistence": ([P, d, dp, dp, dp], st),
        "lbm_critical_temperature": ([P], d),
        "lbm_destroy": ([vp], st),
        "lbm_strerror": ([st], ctypes.c_char_p),
        "lbm_last_error": ([vp], ctypes.c_char_p),
        "lbm_device_copy": ([vp, vp, sz, vp], st),
        "lbm_batch_footprint_bytes": ([ctypes.c_int], sz),
        "lbm_batch_create": ([ctypes.POINTER(vp), ctypes.c_int, vp, sz, vp, ctypes.POINTER(vp)], st),
        "lbm_batch_set_budget": ([vp, ctypes.c_int, i64], st),
        "lbm_batch_step": ([vp, i64], st),
        "lbm_batch_remaining": ([vp, ctypes.c_int], i64),
        "lbm_batch_set_shape": ([vp, ctypes.c_int], st),
        "lbm_batch_get_shape": ([vp], ctypes.c_int),
        "lbm_batch_sync": ([vp, ctypes.POINTER(ctypes.c_int)], st),
        "lbm_batch_set_diagnostics_interval": ([vp, ctypes.c_int64], st),
        "lbm_batch_destroy": ([vp], st),
        "lbm_batch_create_noalloc": ([ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(vp)], st),
        "lbm_batch_set_persistent": ([vp, ctypes.c_int, ctypes.c_uint32], st),
        "lbm3d_params_default": ([P3, i32, i32, i32], None),
        "lbm3d_validate": ([P3], st),
        "lbm3d_footprint_bytes": ([P3], sz),
        "lbm3d_create": ([P3, vp, sz, vp, ctypes.POINTER(vp)], st),
        "lbm3d_init": ([vp, dp, dp, dp, dp, dp], st),
        "lbm3d_step": ([vp, i64], st),
        "lbm3d_sync": ([vp], st),
        "lbm3d_read_fields": ([vp, dp, dp, dp, dp, dp], st),
        "lbm3d_diagnostics": ([vp, dp, dp], st),
        "lbm3d_steps_done": ([vp], i64),
        "lbm3d_state_bytes": ([vp], sz),
        "lbm3d_save_state": ([vp, vp, sz], st),
        "lbm3d_load_state": ([vp, vp, sz], st),
        "lbm3d_destroy": ([vp], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L
