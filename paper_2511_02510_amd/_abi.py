"""ctypes declarations of the C-ABI in include/litevoxel.h.

Loads the in-tree liblitevoxel.so; raises if it has not been built (there is
no fallback implementation).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_uint8, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblitevoxel.so")

LV_OK, LV_ERR_ARG, LV_ERR_HIP, LV_ERR_CAPACITY, LV_ERR_UNSUPPORTED, LV_ERR_STATE = range(6)
LV_MAX_VIEWS = 256
PHASES = ["setup", "preprocess", "scan", "emit", "sort", "order", "composite_fwd",
          "bwd_setup", "composite_bwd", "sh_bwd"]


class LvCamera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("o", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32)]


class LvVoxels(ctypes.Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("root_min", c_float * 3),
                ("root_size", c_float), ("ijk", c_void_p), ("level", c_void_p),
                ("density", c_void_p), ("sh", c_void_p), ("corner_idx", c_void_p),
                ("n_grid", c_int64), ("density_act", c_int32)]


ACT_NONE, ACT_SOFTPLUS, ACT_EXP = 0, 1, 2


class LvFrame(ctypes.Structure):
    _fields_ = [("n_views", c_int32), ("cams_host", POINTER(LvCamera)), ("cams_dev", c_void_p),
                ("bg", c_float * 3)]


class LvSettings(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("chunk", c_int32), ("chunk_bwd", c_int32), ("t_eps", c_float),
                ("pair_capacity", c_uint64)]


class LvGuardParams(ctypes.Structure):
    _fields_ = [("alpha", c_float), ("m_low", c_float), ("m_high", c_float), ("rho", c_float),
                ("w_keep", c_float), ("cap_frac", c_double)]


class LvSplitParams(ctypes.Structure):
    _fields_ = [("kappa", c_float), ("beta", c_float), ("max_splits", ctypes.c_uint32)]


# name -> (restype, argtypes)
P = c_void_p
_SIGS = {
    "lv_create": (c_int32, [POINTER(c_void_p), c_int32]),
    "lv_destroy": (None, [P]),
    "lv_status_str": (ctypes.c_char_p, [c_int32]),
    "lv_last_error": (ctypes.c_char_p, [P]),
    "lv_default_settings": (None, [POINTER(LvSettings)]),
    "lv_validate": (c_int32, [POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings)]),
    "lv_query_sizes": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings),
                                 POINTER(c_uint64), POINTER(c_uint64)]),
    "lv_forward": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P, P,
                             P, P, P, P, P]),
    "lv_backward": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P, P,
                              P, P, P, P, P, P]),
    "lv_forward_aux": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P, P,
                                 P, P, P, P, P, P, P, P]),
    "lv_backward_aux": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P, P,
                                  P, P, P, P, P, P, P, P, P]),
    "lv_aux_loss": (c_int32, [P, POINTER(LvFrame), P, P, P, P, P, c_float, c_float, c_float,
                              c_float, P, P, P, P, P, P]),
    "lv_check_overflow": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings),
                                    P, POINTER(c_uint64), P]),
    "lv_pass_stats": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P,
                                POINTER(c_uint64), POINTER(c_uint64), P]),
    "lv_export_bins": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), POINTER(LvSettings), P,
                                 P, P, P, P, P, P]),
    "lv_lf_weight_workspace_size": (c_uint64, [c_int32]),
    "lv_lf_weight": (c_int32, [P, POINTER(LvFrame), P, c_float, c_int32, c_float, P, P, P]),
    "lv_lf_weight_noalloc": (c_int32, [P, POINTER(LvFrame), P, c_float, c_int32, c_float, P, P]),
    "lv_l1_grad": (c_int32, [P, POINTER(LvFrame), P, P, P, P, P, P]),
    "lv_gamma_schedule": (c_float, [c_float, c_float, c_float, c_float, c_float]),
    "lv_quantile_workspace_size": (c_uint64, [c_int64, c_int32]),
    "lv_depth_quantile": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), P, c_int32, c_double,
                                    P, P, P, P, P]),
    "lv_depth_bins": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), c_int32, P, P, P]),
    "lv_depth_cutoff": (c_int32, [P, POINTER(LvVoxels), P, c_int32, c_double, P, P, P, P]),
    "lv_default_guard": (None, [POINTER(LvGuardParams)]),
    "lv_guard_workspace_size": (c_uint64, [c_int64]),
    "lv_prune_guard": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), P, P, P, c_int32,
                                 POINTER(LvGuardParams), P, P, P, P, P, P]),
    "lv_default_split": (None, [POINTER(LvSplitParams)]),
    "lv_split_workspace_size": (c_uint64, [c_int64]),
    "lv_footprint_range": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), P, P, P]),
    "lv_subdivide_select": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), P, P,
                                      POINTER(LvSplitParams), P, P, P, P, P]),
    "lv_subdivide_apply": (c_int32, [P, POINTER(LvVoxels), P, c_int64, P, P, P, P, P, P, P]),
    "lv_graph_begin": (c_int32, [P, P]),
    "lv_graph_end": (c_int32, [P, P]),
    "lv_graph_launch": (c_int32, [P, P]),
    "lv_graph_reset": (c_int32, [P]),
    "lv_autotune": (c_int32, [P, POINTER(LvVoxels), POINTER(LvFrame), c_int32,
                              POINTER(LvSettings), P, P]),
    "lv_set_timing": (c_int32, [P, c_int32]),
    "lv_read_timings": (c_int32, [P, P, P]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def symbols():
    return list(_SIGS)
