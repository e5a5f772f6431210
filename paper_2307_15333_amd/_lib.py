"""ctypes declarations of the libdot C ABI (include/dot.h).

Loading fails loudly if the HIP library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdot.so")

DOT_OK, DOT_EINVAL, DOT_ENOMEM, DOT_EHIP, DOT_EUNSUPPORTED, DOT_EBUSY = 0, -1, -2, -3, -4, -5
DOT_F32, DOT_F16, DOT_BF16, DOT_PAL16 = 0, 1, 2, 3
DOT_RAYS_CAMERAS, DOT_RAYS_PIXELS, DOT_RAYS_EXPLICIT = 0, 1, 2
DOT_SIGNAL_MAX, DOT_SIGNAL_SUM = 0, 1
DOT_MAX_DEPTH = 16

STORAGE = {"f32": DOT_F32, "f16": DOT_F16, "bf16": DOT_BF16}
STORAGE_NAME = {**{v: k for k, v in STORAGE.items()}, DOT_PAL16: "pal16"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class dot_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class dot_tree_desc(C.Structure):
    _fields_ = [("n_internal", C.c_int64), ("n_leaves", C.c_int64), ("sh_degree", C.c_int32),
                ("reserved", C.c_int32), ("child", C.c_void_p), ("sigma", C.c_void_p),
                ("sh", C.c_void_p), ("bbox_min", C.c_float * 3), ("bbox_size", C.c_float)]


class dot_camera(C.Structure):
    _fields_ = [("c2w", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class dot_rays(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_cams", C.c_int32), ("cams", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32), ("n_rays", C.c_int64),
                ("cam_idx", C.c_void_p), ("pix_idx", C.c_void_p), ("origins", C.c_void_p),
                ("dirs", C.c_void_p)]


class dot_render_opts(C.Structure):
    _fields_ = [("bg", C.c_float * 3), ("t_stop", C.c_float), ("signal_mode", C.c_int32),
                ("reserved", C.c_int32)]


class dot_tree_info_t(C.Structure):
    _fields_ = [("n_internal", C.c_int64), ("n_leaves", C.c_int64), ("sh_degree", C.c_int32),
                ("storage", C.c_int32), ("max_depth", C.c_int32), ("sh_stride", C.c_int32),
                ("child", C.c_void_p), ("sigma", C.c_void_p), ("sh", C.c_void_p),
                ("leaf_depth", C.c_void_p), ("bbox_min", C.c_float * 3), ("bbox_size", C.c_float),
                ("palette", C.c_void_p), ("palette_bits", C.c_int32), ("reserved", C.c_int32),
                ("links", C.c_void_p)]


class dot_refine_params(C.Structure):
    _fields_ = [("prune_tau", C.c_float), ("sample_frac", C.c_float), ("prune_le", C.c_int32),
                ("max_depth", C.c_int32), ("recursive", C.c_int32), ("reinit", C.c_int32)]


class dot_refine_stats(C.Structure):
    _fields_ = [("leaves_before", C.c_int64), ("leaves_after", C.c_int64),
                ("internal_after", C.c_int64), ("merged", C.c_int64), ("subdivided", C.c_int64)]


class dot_adam_params(C.Structure):
    _fields_ = [("lr_sigma", C.c_float), ("lr_sh", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("step", C.c_int32)]


class dot_rmsprop_params(C.Structure):
    _fields_ = [("lr_sigma", C.c_float), ("lr_sh", C.c_float), ("alpha", C.c_float), ("eps", C.c_float)]


class dot_render_job(C.Structure):
    _fields_ = [("tree", C.c_void_p), ("cam", C.c_void_p), ("rgb_out", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("tile_begin", C.c_int64), ("tile_count", C.c_int64),
                ("bg", C.c_float * 3), ("t_stop", C.c_float)]


class dot_serve_job(C.Structure):
    _fields_ = [("tree", C.c_void_p), ("cam", dot_camera), ("rgb_out", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("tile_begin", C.c_int64), ("tile_count", C.c_int64),
                ("bg", C.c_float * 3), ("t_stop", C.c_float)]


# name -> (restype, argtypes); every symbol declared in include/dot.h
SIGNATURES = {
    "dot_build": (C.c_int, [C.POINTER(dot_tree_desc), C.c_int32, C.POINTER(dot_allocator), C.c_void_p,
                            C.POINTER(C.c_void_p)]),
    "dot_free": (C.c_int, [C.c_void_p]),
    "dot_tree_info": (C.c_int, [C.c_void_p, C.POINTER(dot_tree_info_t)]),
    "dot_render": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts), C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p]),
    "dot_render_train_records_bytes": (C.c_size_t, [C.c_int64, C.c_int32]),
    "dot_render_train": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts), C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dot_accumulate_signal": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                        C.c_void_p, C.c_void_p]),
    "dot_render_backward": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dot_refine": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(dot_refine_params),
                             C.POINTER(dot_refine_stats), C.c_void_p]),
    "dot_adam_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.POINTER(dot_adam_params), C.c_void_p]),
    "dot_rmsprop_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(dot_rmsprop_params), C.c_void_p]),
    "dot_render_backward_atomic": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p]),
    "dot_render_backward_rmsprop": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.POINTER(dot_rmsprop_params), C.c_void_p, C.c_void_p, C.c_size_t,
                                              C.c_void_p]),
    "dot_render_backward_adam": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.POINTER(dot_adam_params), C.c_void_p, C.c_void_p,
                                           C.c_size_t, C.c_void_p]),
    "dot_sigma_signal": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dot_pixel_batch_workspace": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32, C.c_int32]),
    "dot_pixel_batch": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dot_pixel_batch_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p]),
    "dot_mse_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "dot_mse_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dot_quantize_sh": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "dot_set_links": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "dot_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dot_render_stats": (C.c_int, [C.c_void_p, C.POINTER(dot_rays), C.POINTER(dot_render_opts),
                                   C.POINTER(C.c_int64), C.c_void_p]),
    "dot_render_jobs_workspace": (C.c_size_t, [C.c_int32]),
    "dot_render_jobs": (C.c_int, [C.POINTER(dot_render_job), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dot_serve_open": (C.c_int, [C.c_int32, C.c_int32, C.c_double, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dot_serve_push": (C.c_int, [C.c_void_p, C.POINTER(dot_serve_job), C.POINTER(C.c_int64)]),
    "dot_serve_done": (C.c_int, [C.c_void_p, C.c_int64]),
    "dot_serve_close": (C.c_int, [C.c_void_p]),
    "dot_stream_read": (C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "dot_gather_rows": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "dot_atomic_count": (C.c_int, [C.c_void_p, C.c_uint32, C.c_int64, C.c_int, C.c_void_p]),
    "dot_last_error": (C.c_char_p, []),
}

_lib = None


class DotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdot error {code}: {msg}")
        self.code = code


def load():
    """Load libdot.so (built in-tree by paper_2307_15333_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_15333_amd.build` "
                              "(there is no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc):
    if rc != DOT_OK:
        msg = load().dot_last_error().decode(errors="replace")
        raise DotError(rc, msg)
    return rc
