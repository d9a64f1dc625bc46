"""ctypes loader for libairhip.so: argument types of every C-ABI entry point.

The library is built in-tree by `build.py`; importing this module never
builds it, and a missing library is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# AIRHIP_LIB_VARIANT=debug selects the bounds-checked debug build
# (libairhip_debug.so, the same entry points).
LIB_PATH = os.path.join(HERE, "libairhip_debug.so" if os.environ.get("AIRHIP_LIB_VARIANT") == "debug"
                        else "libairhip.so")

AIR_OK = 0
STATUS_NAMES = {
    0: "AIR_OK", 1: "AIR_ERR_INVALID_ARG", 2: "AIR_ERR_SHAPE", 3: "AIR_ERR_ALIGN",
    4: "AIR_ERR_WORKSPACE", 5: "AIR_ERR_UNSUPPORTED", 6: "AIR_ERR_LAUNCH",
    7: "AIR_ERR_NONFINITE", 8: "AIR_ERR_DEVICE",
}


class AirError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} "
                         f"({_strerror(status)})")


class AirProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("transform", ctypes.c_int32), ("spacing", ctypes.c_int32 * 3),
                ("similarity", ctypes.c_int32), ("lambda_diff", ctypes.c_float),
                ("diffeo_steps", ctypes.c_int32), ("regulariser", ctypes.c_int32),
                ("sigma", ctypes.c_float * 3), ("lcc_radius", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float
_sz = ctypes.c_size_t

# name -> (restype, argtypes); mirrors include/airhip.h
SIGNATURES = {
    "air_plan_create": (_i32, [ctypes.POINTER(AirProblem), _i32, ctypes.POINTER(_vp)]),
    "air_plan_destroy": (None, [_vp]),
    "air_plan_prepare": (_i32, [_vp]),
    "air_plan_workspace_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "air_plan_param_count": (_i32, [_vp, _i32, ctypes.POINTER(_i64)]),
    "air_tiling_count": (_i32, [_i32]),
    "air_tiling_describe": (_i32, [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                   ctypes.POINTER(_i32)]),
    "air_plan_set_tiling": (_i32, [_vp, _i32]),
    "air_plan_get_tiling": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "air_warp": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "air_displacement": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "air_similarity": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "air_regulariser": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "air_objective_and_grad": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "air_objective_and_grad_batched": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "air_objective_and_grad_noalloc": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "air_synth_blobs": (_i32, [_vp, _i32, ctypes.POINTER(_i32), _vp, _vp]),
    "air_autotune_workspace_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "air_autotune": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, ctypes.c_char_p,
                            ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double), _vp]),
    "air_autotune_cached": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_i32)]),
    "air_cnn_create": (_i32, [_i32, _i32, ctypes.POINTER(_vp)]),
    "air_cnn_destroy": (None, [_vp]),
    "air_cnn_sizes": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_sz)]),
    "air_cnn_layer": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                             ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "air_cnn_forward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "air_cnn_backward": (_i32, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "air_synth_add_normal": (_i32, [_vp, _i64, ctypes.c_uint64, _f32, _vp]),
    "air_adam_step": (_i32, [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _i32, _vp]),
    "air_adam_bias_terms": (_i32, [_f32, _f32, _f32, _i32, _vp]),
    "air_adam_step_dev": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _f32, _f32, _f32, _vp]),
    "air_scale": (_i32, [_vp, _vp, _i64, _vp]),
    "air_get_flags": (_i32, [_vp, _vp, _vp, _vp]),
    "air_pyramid_workspace_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "air_pyramid_down": (_i32, [_vp, _vp, _f32, _vp, _vp, _sz, _vp]),
    "air_field_resample": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "air_conv3d_fwd": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _i32, _vp,
                              _i32, _i32, _vp, _i32, _vp]),
    "air_conv3d_flip_weights": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "air_conv3d_bwd_weight_workspace": (_i32, [_vp, _i32, _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "air_conv3d_bwd_weight": (_i32, [_vp, _vp, _i32, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _sz,
                                     _vp]),
    "air_cast_bf16": (_i32, [_vp, _vp, _i64, _vp]),
    "air_pool2": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "air_pool2_bwd": (_i32, [_vp, _vp, _i32, _vp, _i32, _i32, _i32, _vp]),
    "air_up2": (_i32, [_vp, _vp, _i32, _vp, _i32, _i32, _vp]),
    "air_up2_bwd": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "air_lrelu_bwd": (_i32, [_vp, _i32, _i32, _vp, _i32, _i32, _i64, _i32, _vp, _vp]),
    "air_pool2_lrelu_bwd": (_i32, [_vp, _vp, _i32, _vp, _i32, _i32, _vp, _i32, _i32, _i32, _vp,
                                   _vp]),
    "air_conv3d_bwd_weight_xb_workspace": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32,
                                                  ctypes.POINTER(_sz)]),
    "air_conv3d_bwd_weight_xb": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _vp, _vp,
                                        _sz, _vp]),
    "air_up2_lrelu_bwd": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _vp]),
    "air_cnn_input": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "air_cnn_output": (_i32, [_vp, _vp, _i32, _i32, _f32, _vp, _vp]),
    "air_cnn_output_bwd": (_i32, [_vp, _vp, _i32, _i32, _f32, _vp, _vp, _vp]),
    "air_add_f32": (_i32, [_vp, _vp, _i64, _vp]),
    "air_plan_timing": (_i32, [_vp, _i32]),
    "air_plan_timing_read": (_i32, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)]),
    "air_strerror": (ctypes.c_char_p, [_i32]),
    "air_debug_bounds_take": (_i32, [ctypes.POINTER(ctypes.c_uint32)]),
}

_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_1806_09907_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return lib().air_strerror(int(status)).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "?"


def check(status: int, where: str) -> None:
    if status != AIR_OK:
        raise AirError(status, where)
