"""ctypes declarations of the libdass C ABI (include/dass.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdass.so")

DASS_OK, DASS_E_INVALID, DASS_E_OOM, DASS_E_CAPACITY, DASS_E_HIP, DASS_E_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "DASS_OK", 1: "DASS_E_INVALID", 2: "DASS_E_OOM", 3: "DASS_E_CAPACITY", 4: "DASS_E_HIP",
                5: "DASS_E_UNSUPPORTED"}
DASS_FWD, DASS_ADJOINT = 0, 1
MAX_VIEWS = 32
NOALLOC_MAX_PIXELS = 1 << 21  # DASS_NOALLOC_MAX_PIXELS

# Every exported symbol of include/dass.h (checked by the ABI test).
EXPORTS = ("dass_create", "dass_reserve", "dass_destroy", "dass_last_error", "dass_sync", "render_fwd",
           "dass_render_fwd_l1", "render_bwd", "shift_apply", "adam_step", "densify_append", "dass_l1_loss_grad", "dass_fidelity_loss_grad", "dass_fidelity_loss_grad_noalloc", "dass_debug_keys",
           "dass_debug_projection", "dass_autotune_tile", "dass_profile_begin", "dass_profile_end", "dass_debug_pair_counts",
           "adam_step_device_count", "dass_hash_field_fwd", "dass_hash_field_bwd",
           "dass_inherit_apply", "dass_inherit_adjoint", "dass_compact_var", "dass_render_features",
           "dass_dynamic_mask")
FLAG_COUNT_PAIRS = 1
FLAG_SUBTILE8 = 2
STAGES = ("project", "depth_sort", "binning", "key_sort", "ranges", "blend_fwd", "blend_bwd", "project_bwd",
          "shift", "adam", "l1", "densify", "field", "inherit")


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("capacity", C.c_int32), ("n_base", C.c_int32), ("sh_degree", C.c_int32),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("sh", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("campos", C.c_float * 3), ("width", C.c_int32),
                ("height", C.c_int32)]


class Image(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("t_final", C.c_void_p), ("n_contrib", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("sh", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("batch", C.c_int32), ("flags", C.c_uint32)]


class Limits(C.Structure):
    _fields_ = [("max_gaussians", C.c_int32), ("max_views", C.c_int32), ("max_keys", C.c_int64),
                ("max_tiles", C.c_int64)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float)]


HASH_MAX_LEVELS = 16


class HashField(C.Structure):
    _fields_ = [("levels", C.c_int32), ("features", C.c_int32), ("log2_table", C.c_int32), ("hidden", C.c_int32),
                ("res", C.c_int32 * HASH_MAX_LEVELS), ("aabb_min", C.c_float * 3), ("aabb_max", C.c_float * 3),
                ("table", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p),
                ("b2", C.c_void_p)]


class HashFieldGrads(C.Structure):
    _fields_ = [("table", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p),
                ("b2", C.c_void_p)]


_lib = None


class MissingLibrary(RuntimeError):
    pass


def lib():
    """Loads libdass.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MissingLibrary(f"{LIB_PATH} is missing: build it with `python -m paper_2411_14847_amd.build` "
                                 "(the HIP extension is required; there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_uint64
        P = C.POINTER
        sig = {
            "dass_create": (i32, [P(vp), i32, P(Limits)]),
            "dass_reserve": (i32, [vp, P(Limits)]),
            "dass_destroy": (None, [vp]),
            "dass_last_error": (C.c_char_p, [vp]),
            "dass_sync": (i32, [vp, vp]),
            "render_fwd": (i32, [vp, P(Gaussians), P(Camera), i32, P(f32), P(Image), P(Opts), vp]),
            "dass_render_fwd_l1": (i32, [vp, P(Gaussians), P(Camera), i32, P(f32), P(Image), P(vp), P(vp), P(vp), vp,
                                         P(Opts), vp]),
            "render_bwd": (i32, [vp, P(Gaussians), P(Camera), i32, P(f32), P(Image), P(vp), P(Grads), vp, vp,
                                 P(Opts), vp]),
            "shift_apply": (i32, [vp, i32, vp, i32, vp, vp, P(Gaussians), P(Gaussians), P(Grads), vp, vp, vp]),
            "adam_step": (i32, [vp, P(AdamGroup), i32, f32, f32, f32, i32, vp]),
            "adam_step_device_count": (i32, [vp, P(AdamGroup), i32, f32, f32, f32, vp, vp]),
            "densify_append": (i32, [vp, P(Gaussians), P(vp), P(Camera), i32, vp, vp, f32, f32, f32, i32, u64, vp,
                                     vp]),
            "dass_l1_loss_grad": (i32, [vp, P(Camera), i32, P(vp), P(vp), P(vp), P(vp), vp, vp]),
            "dass_fidelity_loss_grad": (i32, [vp, P(Camera), i32, P(vp), P(vp), f32, P(vp), P(vp), vp, P(vp), vp]),
            "dass_fidelity_loss_grad_noalloc": (i32, [vp, P(Camera), i32, P(vp), P(vp), f32, P(vp), P(vp), vp, vp]),
            "dass_debug_keys": (i32, [vp, i32, vp, vp, i64, vp, P(i64)]),
            "dass_debug_projection": (i32, [vp, P(Gaussians), P(Camera), P(Opts), vp]),
            "dass_autotune_tile": (i32, [vp, P(Gaussians), P(Camera), i32, P(f32), P(Image), P(vp), P(Grads), P(Opts),
                                         i32, i32, P(i32), P(f32), vp]),
            "dass_profile_begin": (i32, [vp, i32]),
            "dass_profile_end": (i32, [vp, P(C.c_double), P(i32)]),
            "dass_debug_pair_counts": (i32, [vp, P(u64), P(u64)]),
            "dass_hash_field_fwd": (i32, [vp, P(HashField), vp, i64, i32, vp, i32, vp, vp, i64, vp]),
            "dass_hash_field_bwd": (i32, [vp, P(HashField), vp, i64, i32, vp, i32, vp, vp, i64, P(HashFieldGrads),
                                          vp]),
            "dass_inherit_apply": (i32, [vp, P(Gaussians), vp, vp, vp, vp]),
            "dass_inherit_adjoint": (i32, [vp, P(Gaussians), vp, vp, vp, f32, vp, vp, vp]),
            "dass_compact_var": (i32, [vp, P(Gaussians), vp, f32, vp, vp]),
            "dass_render_features": (i32, [vp, P(Gaussians), P(Camera), i32, vp, i32, P(vp), P(Opts), vp]),
            "dass_dynamic_mask": (i32, [vp, P(Camera), i32, P(vp), P(vp), f32, vp, vp, i32, i32, vp, i64, i32, vp, vp,
                                        vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
