"""ctypes binding of libgeer.so (declarations in include/geer.h).

Argument marshalling only: every step of the render runs in the HIP library.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgeer.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED, ERR_STALLED = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "CAPACITY", 4: "HIP", 5: "UNSUPPORTED", 6: "STALLED"}
MODELS = {"pinhole": 0, "equidistant": 1, "kb": 2}
GRIDS = {"beap": 0, "native": 1}
BUF_RECT, BUF_COUNT, BUF_KEY, BUF_LIST, BUF_RANGES, BUF_NLAST = range(6)

# every symbol include/geer.h declares
EXPORTS = ["geer_create", "geer_destroy", "geer_last_error", "geer_default_opts", "geer_render",
           "geer_render_backward", "geer_frame_release", "geer_frame_get_stats", "geer_frame_buffer_bytes",
           "geer_frame_export", "geer_valid_mask", "geer_l1_loss", "geer_set_profiling", "geer_profile_read",
           "geer_plan_workspace_bytes", "geer_plan_create", "geer_train_plan_workspace_bytes",
           "geer_train_plan_create", "geer_plan_launch", "geer_plan_entries", "geer_plan_device_bytes", "geer_plan_destroy",
           "geer_check", "geer_debug_mark_stalled", "geer_debug_set_spin_limit", "geer_plan_get_stats",
           "geer_reproject", "geer_activate", "geer_adam_step", "geer_densify", "geer_render_static"]


class GeerView(C.Structure):
    _fields_ = [("model", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("grid", C.c_int32),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("k", C.c_double * 4), ("fov_x", C.c_double), ("fov_y", C.c_double),
                ("R", C.c_double * 9), ("t", C.c_double * 3)]


class GeerScene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class GeerOpts(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("lambda_fixed", C.c_float), ("lambda_mode", C.c_int32), ("flags", C.c_int32)]


class GeerFrameStats(C.Structure):
    _fields_ = [("n_items", C.c_int64), ("n_visible", C.c_int64), ("n_entries", C.c_int64),
                ("n_tiles", C.c_int64), ("n_pixels", C.c_int64), ("n_evaluated", C.c_int64),
                ("n_candidates", C.c_int64)]


class GeerProfileRecord(C.Structure):
    _fields_ = [("ms_preprocess", C.c_float), ("ms_sort", C.c_float), ("ms_render", C.c_float),
                ("ms_total", C.c_float), ("n_entries", C.c_int64), ("n_evaluated", C.c_int64),
                ("kind", C.c_int32), ("reserved", C.c_int32)]


class GeerTrainState(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32), ("raw", C.c_void_p),
                ("scale", C.c_void_p), ("opacity", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("accum", C.c_void_p), ("count", C.c_void_p)]


class GeerAdamOpts(C.Structure):
    _fields_ = [("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("lr_mean", C.c_float),
                ("lr_scale", C.c_float), ("lr_quat", C.c_float), ("lr_opacity", C.c_float), ("lr_sh", C.c_float),
                ("step", C.c_int32), ("reserved", C.c_int32)]


class GeerDensifyOpts(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("split_scale", C.c_float), ("min_opacity", C.c_float),
                ("split_shrink", C.c_float)]


class GeerError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("geer %s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lock = threading.Lock()
_lib = None


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgeer.so is not built (%s); run `python -m paper_2505_24053_amd.build` "
                               "or __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P, V = C.POINTER, C.c_void_p
        L.geer_create.argtypes = [C.c_int32, P(V)]
        L.geer_destroy.argtypes = [V]
        L.geer_destroy.restype = None
        L.geer_last_error.argtypes = [V]
        L.geer_last_error.restype = C.c_char_p
        L.geer_default_opts.argtypes = [P(GeerOpts)]
        L.geer_default_opts.restype = None
        L.geer_render.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts), V, V, V, P(V), V]
        L.geer_render_static.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts), V, V, V, V]
        L.geer_render_backward.argtypes = [V, V, V, V, V, V, V, V, C.c_int32, V]
        L.geer_frame_release.argtypes = [V]
        L.geer_frame_release.restype = None
        L.geer_frame_get_stats.argtypes = [V, P(GeerFrameStats)]
        L.geer_frame_buffer_bytes.argtypes = [V, C.c_int32]
        L.geer_frame_buffer_bytes.restype = C.c_int64
        L.geer_frame_export.argtypes = [V, C.c_int32, V, C.c_int64]
        L.geer_valid_mask.argtypes = [P(GeerView), V]
        L.geer_l1_loss.argtypes = [V, C.c_int64, V, V, V, V, V, V]
        L.geer_set_profiling.argtypes = [V, C.c_int32]
        L.geer_profile_read.argtypes = [V, P(GeerProfileRecord), C.c_int32]
        L.geer_profile_read.restype = C.c_int32
        L.geer_plan_workspace_bytes.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts), C.c_int64,
                                                P(C.c_int64)]
        L.geer_plan_create.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts), C.c_int64, V,
                                       C.c_int64, V, V, V, P(V)]
        L.geer_train_plan_workspace_bytes.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts),
                                                      C.c_int64, P(C.c_int64)]
        L.geer_train_plan_create.argtypes = [V, P(GeerScene), C.c_int32, P(GeerView), P(GeerOpts), C.c_int64, V,
                                             C.c_int64, V, V, V, V, V, V, V, V, V, P(V)]
        L.geer_plan_launch.argtypes = [V, P(GeerView), V]
        L.geer_plan_entries.argtypes = [V, P(C.c_int64), P(C.c_int64)]
        L.geer_plan_get_stats.argtypes = [V, P(GeerFrameStats)]
        L.geer_reproject.argtypes = [V, P(GeerView), C.c_int32, C.c_int32, C.c_int32, V, V, V, V]
        L.geer_activate.argtypes = [V, P(GeerTrainState), V]
        L.geer_adam_step.argtypes = [V, P(GeerTrainState), P(GeerAdamOpts), V, V, V, V, V, V]
        L.geer_densify.argtypes = [V, P(GeerTrainState), P(GeerDensifyOpts), V, P(GeerTrainState), V]
        L.geer_plan_device_bytes.argtypes = [V]
        L.geer_plan_device_bytes.restype = C.c_int64
        L.geer_plan_destroy.argtypes = [V]
        L.geer_plan_destroy.restype = None
        L.geer_check.argtypes = [V, V]
        L.geer_debug_mark_stalled.argtypes = [V, V]
        L.geer_debug_set_spin_limit.argtypes = [V, C.c_int64]
        _lib = L
        return L


def make_view(cam: dict) -> GeerView:
    v = GeerView()
    v.model = MODELS[cam["model"]]
    v.width, v.height = int(cam["width"]), int(cam["height"])
    v.grid = GRIDS[cam.get("grid", "beap")]
    v.fx, v.fy, v.cx, v.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    for i in range(4):
        v.k[i] = float(cam["k"][i])
    v.fov_x, v.fov_y = float(cam["fov_x"]), float(cam["fov_y"])
    R = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    t = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    for i in range(9):
        v.R[i] = R[i]
    for i in range(3):
        v.t[i] = t[i]
    return v


OPT_NO_CONE_CULL = 1
ASSOC = {"pbf": 0, "ewa": 1, "ewa_snug": 2, "ut": 3, "ut_snug": 4}


OPT_SPLAT_ALPHA = 1 << 4


def make_opts(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, lambda_mode=0, lambda_fixed=3.0,
              cone_cull=True, assoc="pbf", splat=False) -> GeerOpts:
    o = GeerOpts()
    o.alpha_min, o.alpha_max, o.t_min = float(alpha_min), float(alpha_max), float(t_min)
    o.lambda_fixed, o.lambda_mode = float(lambda_fixed), int(lambda_mode)
    o.flags = (0 if cone_cull else OPT_NO_CONE_CULL) | (ASSOC[assoc] << 1) | (OPT_SPLAT_ALPHA if splat else 0)
    return o


def check(status, ctx=None):
    if status != OK:
        msg = load().geer_last_error(ctx).decode() if ctx else ""
        raise GeerError(status, msg)


def valid_mask(cam: dict) -> np.ndarray:
    v = make_view(cam)
    out = np.zeros(int(cam["height"]) * int(cam["width"]), np.uint8)
    check(load().geer_valid_mask(C.byref(v), C.c_void_p(out.ctypes.data)))
    return out.reshape(int(cam["height"]), int(cam["width"])).astype(bool)


__all__ = ["load", "make_view", "make_opts", "check", "valid_mask", "GeerError", "EXPORTS"]
