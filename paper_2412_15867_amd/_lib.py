"""ctypes binding of libirgs.so (declared in include/irgs.h).

Argument marshalling only: every step of the trace runs in the HIP library.
If the library is missing the import of this module's ``lib()`` raises --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirgs.so")

c_i32, c_i64, c_u32, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p

IRGS_OK = 0
IRGS_E_INVALID = -1
IRGS_E_OOM = -2
IRGS_E_HIP = -3
IRGS_E_STATE = -4
FLAG_BRUTE_FORCE = 1
FLAG_RECOMPUTE = 2
FLAG_SH = 4          # features are RGB SH coefficients; 3 composited channels
FLAG_NORMAL = 8      # 3 more composited channels: the ray-facing normal (forward only)
FLAG_RADIX_TREE = 16  # scene build: Morton radix tree instead of PLOC clustering
FLAG_SORT_RAYS = 32  # trace rays in the Morton order of their origins (same results)


class Surfels(ctypes.Structure):
    _fields_ = [("mu", c_vp), ("quat", c_vp), ("scale", c_vp), ("opacity", c_vp), ("feat", c_vp)]


class Params(ctypes.Structure):
    _fields_ = [("k", c_i32), ("feature_dim", c_i32), ("alpha_min", c_f32), ("T_min", c_f32),
                ("t_min", c_f32), ("t_max", c_f32), ("support_sigma", c_f32), ("flags", c_u32),
                ("leaf_size", c_i32)]


class Out(ctypes.Structure):
    _fields_ = [("opacity", c_vp), ("feat", c_vp), ("depth", c_vp), ("T", c_vp), ("n_hits", c_vp),
                ("hit_ids", c_vp), ("hit_T", c_vp), ("H_cap", c_i32), ("counters", c_vp)]


class GradIn(ctypes.Structure):
    _fields_ = [("g_opacity", c_vp), ("g_feat", c_vp), ("g_depth", c_vp)]


class Grads(ctypes.Structure):
    _fields_ = [("mu", c_vp), ("quat", c_vp), ("scale", c_vp), ("opacity", c_vp), ("feat", c_vp)]


class Work(ctypes.Structure):
    _fields_ = [("scene", c_i32), ("pad", c_i32), ("ray_begin", c_i64), ("ray_count", c_i64),
                ("ro", c_vp), ("rd", c_vp), ("out", Out)]


class ShadeIn(ctypes.Structure):
    _fields_ = [("P", c_i64), ("N", c_i32), ("E", c_i32), ("n", c_vp), ("wo", c_vp), ("albedo", c_vp),
                ("rough", c_vp), ("wi", c_vp), ("O", c_vp), ("Lind", c_vp), ("env", c_vp), ("wgt", c_vp)]


class ShadeGrads(ctypes.Structure):
    _fields_ = [("albedo", c_vp), ("rough", c_vp), ("env", c_vp), ("O", c_vp), ("Lind", c_vp)]


# name -> (restype, argtypes); the exported symbols of include/irgs.h
SIGNATURES = {
    "irgs_scene_bytes": (ctypes.c_size_t, [c_i64, c_i32]),
    "irgs_trace_bytes": (ctypes.c_size_t, [c_i64, c_i32, c_u32]),
    "irgs_scene_create": (ctypes.c_int, [c_i64, c_i32, ctypes.POINTER(Surfels), ctypes.POINTER(c_vp)]),
    "irgs_scene_set_params": (ctypes.c_int, [c_vp, ctypes.POINTER(Surfels)]),
    "irgs_scene_build": (ctypes.c_int, [c_vp, ctypes.POINTER(Params), c_vp]),
    "irgs_scene_refit": (ctypes.c_int, [c_vp, c_vp]),
    "irgs_trace": (ctypes.c_int, [c_vp, ctypes.POINTER(Params), c_i64, c_vp, c_vp, ctypes.POINTER(Out), c_vp]),
    "irgs_trace_noalloc": (ctypes.c_int, [c_vp, ctypes.POINTER(Params), c_i64, c_vp, c_vp, ctypes.POINTER(Out),
                                          c_vp]),
    "irgs_trace_backward": (ctypes.c_int, [c_vp, ctypes.POINTER(Params), c_i64, c_vp, c_vp, ctypes.POINTER(Out),
                                           ctypes.POINTER(GradIn), ctypes.POINTER(Grads), c_vp]),
    "irgs_trace_packed": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32, ctypes.POINTER(Params),
                                         ctypes.POINTER(Work), c_i32, c_vp]),
    "irgs_scene_info": (ctypes.c_int, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i32)]),
    "irgs_scene_export": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "irgs_scene_destroy": (ctypes.c_int, [c_vp]),
    "irgs_mc_rays": (ctypes.c_int, [c_i64, c_i32, c_i32, c_vp, c_vp, c_vp, c_f32, c_vp, c_vp, c_vp]),
    "irgs_env_prefilter": (ctypes.c_int, [c_i32, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "irgs_brdf_table": (ctypes.c_int, [c_i32, c_vp, c_vp]),
    "irgs_relight_lind": (ctypes.c_int, [c_i64, c_vp, c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "irgs_env_cdf": (ctypes.c_int, [c_i32, c_vp, c_vp, c_vp]),
    "irgs_env_rays": (ctypes.c_int, [c_i64, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_f32, c_vp, c_vp, c_vp,
                                     c_vp]),
    "irgs_mc_shade": (ctypes.c_int, [ctypes.POINTER(ShadeIn), c_vp, c_vp]),
    "irgs_mc_shade_backward": (ctypes.c_int, [ctypes.POINTER(ShadeIn), c_vp, ctypes.POINTER(ShadeGrads), c_vp]),
    "irgs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "irgs_last_error": (ctypes.c_char_p, []),
    "irgs_version": (ctypes.c_char_p, []),
}

_lib = None


class IrgsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def lib():
    """Load libirgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_15867_amd.build` "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != IRGS_OK:
        msg = lib().irgs_last_error().decode(errors="replace")
        raise IrgsError(status, where, msg)
