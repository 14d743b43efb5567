"""ctypes binding of libgsmap.so (the C ABI declared in include/gsmap.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels behind these calls.  Loading fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsmap.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gsmap.h")

GS_OK, GS_E_INVALID, GS_E_CAPACITY, GS_E_OVERFLOW, GS_E_HIP = 0, 1, 2, 3, 4
GS_STATUS_KEY_OVERFLOW = 1
GS_STATUS_GAUSSIAN_OVERFLOW = 2
GS_FLAG_EMIT_KEYS = 1
GS_FLAG_FULL_BOX = 2
GS_WINDOW_PLANAR_REG = 1
GS_WINDOW_ADAM = 2


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gsmap error {code}: {msg}")
        self.code = code


class gs_params(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("log_scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity_logit", C.c_void_p),
                ("rgb", C.c_void_p), ("n_dev", C.c_void_p),
                ("capacity", C.c_int32), ("sh_degree", C.c_int32),
                ("sh", C.c_void_p)]


class gs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("near_z", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("pad_", C.c_int32)]


class gs_settings(C.Structure):
    _fields_ = [("tile", C.c_int32), ("lds_batch", C.c_int32),
                ("bg", C.c_float * 3), ("alpha_min", C.c_float),
                ("T_min", C.c_float), ("alpha_max", C.c_float),
                ("flags", C.c_int32), ("block_threads", C.c_int32)]


class gs_window_desc(C.Structure):
    _fields_ = [("ws", C.c_void_p), ("params", gs_params), ("cams", C.c_void_p),
                ("settings", gs_settings), ("out_rgb", C.c_void_p),
                ("out_T", C.c_void_p), ("out_nlast", C.c_void_p),
                ("target", C.c_void_p), ("lambda_l1", C.c_float),
                ("lambda_reg", C.c_float), ("reg_floor", C.c_float),
                ("flags", C.c_int32), ("loss_dev", C.c_void_p),
                ("sqerr_dev", C.c_void_p), ("grad", gs_params),
                ("adam_m", gs_params), ("adam_v", gs_params),
                ("lr", C.c_float * 6), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("pad_", C.c_int32),
                ("step_dev", C.c_void_p)]


class gs_geometry(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("tile", C.c_int32),
                ("capacity", C.c_int32), ("pad_", C.c_int32),
                ("key_capacity", C.c_int64)]


class gs_workspace_view(C.Structure):
    _fields_ = [("records", C.c_void_p), ("tiles_touched", C.c_void_p),
                ("render_box", C.c_void_p), ("ranges", C.c_void_p), ("vals_sorted", C.c_void_p),
                ("keys_sorted", C.c_void_p), ("grad2d", C.c_void_p),
                ("n_keys", C.c_void_p), ("status", C.c_void_p),
                ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("grad_opacity", C.c_void_p), ("grad_colour", C.c_void_p)]


_P = C.POINTER
_vp = C.c_void_p
_SIGS = {
    "gs_workspace_size": (C.c_int, [_P(gs_geometry), _P(C.c_size_t)]),
    "gs_workspace_create": (C.c_int, [_P(gs_geometry), _vp, C.c_size_t, _vp,
                                      _P(_vp)]),
    "gs_workspace_destroy": (C.c_int, [_vp]),
    "gs_workspace_get_view": (C.c_int, [_vp, _P(gs_workspace_view)]),
    "gs_project_and_bin": (C.c_int, [_vp, _P(gs_params), _vp,
                                     _P(gs_settings), _vp]),
    "gs_sort_tile_keys": (C.c_int, [_vp, _P(gs_settings), _vp]),
    "gs_render_fwd": (C.c_int, [_vp, _P(gs_params), _P(gs_settings), _vp, _vp,
                                _vp, _vp]),
    "gs_count_pairs": (C.c_int, [_vp, _P(gs_params), _P(gs_settings), _vp,
                                 _vp]),
    "gs_render_bwd": (C.c_int, [_vp, _P(gs_params), _P(gs_settings), _vp,
                                _vp, _vp, _P(gs_params), _vp]),
    "gs_render_bwd_l1": (C.c_int, [_vp, _P(gs_params), _P(gs_settings), _vp,
                                   _vp, C.c_float, _vp, _vp, _P(gs_params),
                                   _vp, _vp, _vp]),
    "gs_project_bwd": (C.c_int, [_vp, _P(gs_params), _vp, _P(gs_params),
                                 _vp]),
    "gs_loss_l1": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, C.c_int32,
                             C.c_float, _vp, _vp, _vp, _vp]),
    "gs_insert_distance": (C.c_int, [_P(gs_params), _P(gs_params),
                                     _P(gs_params), _vp, C.c_int32, C.c_int32,
                                     _vp, _vp, C.c_int32, C.c_float, C.c_int32,
                                     _vp, _vp, _vp, _vp, _vp]),
    "gs_insert_distance_noalloc": (C.c_int, [_P(gs_params), _P(gs_params),
                                             _P(gs_params), _vp, C.c_int32,
                                             C.c_int32, _vp, _vp, C.c_int32,
                                             C.c_float, C.c_int32, _vp, _vp,
                                             _vp, _vp]),
    "gs_render_dominant": (C.c_int, [_vp, _P(gs_params), _P(gs_settings), _vp,
                                     _vp, _vp, _vp, _vp]),
    "gs_densify": (C.c_int, [_P(gs_params), _P(gs_params), _P(gs_params), _vp,
                             C.c_int64, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "gs_loss_ssim": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, C.c_int32,
                               C.c_float, _vp, _vp, _vp, _vp, _vp]),
    "gs_loss_colour": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_float, C.c_float, _vp, _vp, _vp, _vp,
                                 _vp, _vp]),
    "gs_planar_reg": (C.c_int, [_P(gs_params), C.c_float, C.c_float,
                                _P(gs_params), _vp, _vp]),
    "gs_adam": (C.c_int, [_P(gs_params), _P(gs_params), _P(gs_params),
                          _P(gs_params), _vp, C.c_float, C.c_float, C.c_float,
                          C.c_int32, _vp, _vp]),
    "gs_insert_gaussians": (C.c_int, [_P(gs_params), _P(gs_params),
                                      _P(gs_params), _vp, C.c_int32, C.c_int32,
                                      _vp, _vp, _vp, C.c_int32, C.c_float,
                                      C.c_int32, _vp, _vp, _vp, _vp]),
    "gs_knn_features": (C.c_int, [_P(gs_params), _vp, C.c_int32, C.c_int32,
                                  _vp, _vp, C.c_int32, C.c_int32, _vp, _vp,
                                  _vp, _vp]),
    "gs_mlp_fwd": (C.c_int, [_vp, _vp, C.c_int32, _vp, _vp, _vp]),
    "gs_mlp_mse": (C.c_int, [_vp, _vp, C.c_int32, _vp, _vp, _vp]),
    "gs_mlp_bwd": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32, _vp, _vp]),
    "gs_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, C.c_float, C.c_float,
                              C.c_float, C.c_float, C.c_int32, _vp]),
    "gs_read_status": (C.c_int, [_vp, _vp, _P(C.c_int32), _P(C.c_int64),
                                 C.c_int32]),
    "gs_window_build": (C.c_int, [_P(gs_window_desc), _vp, _P(_vp)]),
    "gs_window_run": (C.c_int, [_vp, _vp]),
    "gs_window_destroy": (C.c_int, [_vp]),
    "gs_last_error": (C.c_char_p, []),
    "gs_version": (C.c_char_p, []),
}

_LIB = None


def lib():
    """Loads libgsmap.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def declared_symbols():
    """Names of every function include/gsmap.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"GS_API\s+[\w\s\*]*?\b(gs_\w+)\s*\(", text)))


def check(rc):
    if rc != GS_OK:
        msg = lib().gs_last_error().decode(errors="replace")
        raise GsError(rc, msg)
    return rc


def call(name, *args):
    return check(getattr(lib(), name)(*args))
