"""ctypes view of libgs.so (include/gs.h).  Marshalling only: every stage of
the rasterizer runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_CAPACITY = -2
GS_ERR_HIP = -3
GS_ERR_BUDGET = -4
GS_EAGAIN = -5
GS_ERR_INTERNAL = -6
GS_MAX_VIEWS = 16
REC_FLOATS = 16
GRAD2D_FLOATS = 12

_ERRNAMES = {GS_ERR_INVALID_ARG: "GS_ERR_INVALID_ARG", GS_ERR_CAPACITY: "GS_ERR_CAPACITY",
             GS_ERR_HIP: "GS_ERR_HIP", GS_ERR_BUDGET: "GS_ERR_BUDGET", GS_EAGAIN: "GS_EAGAIN",
             GS_ERR_INTERNAL: "GS_ERR_INTERNAL"}


class GsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class GsCamera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("viewmat", C.c_float * 16), ("width", C.c_int32), ("height", C.c_int32),
                ("near_plane", C.c_float), ("far_plane", C.c_float)]


class GsOptions(C.Structure):
    _fields_ = [("sh_degree", C.c_int32), ("dilation", C.c_float), ("aa_compensate", C.c_int32),
                ("bg", C.c_float * 3)]


class GsGaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64), ("app", C.c_void_p)]


class GsGaussiansGrad(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacities", C.c_void_p), ("d_sh", C.c_void_p), ("d_app", C.c_void_p)]


class GsDensifyParams(C.Structure):
    _fields_ = [("box_min", C.c_float * 3), ("box_max", C.c_float * 3), ("tau_min", C.c_float), ("eta", C.c_float),
                ("d_max", C.c_float), ("prune_opacity", C.c_float), ("split_scale", C.c_float),
                ("budget", C.c_int64)]


class GsAppearanceMlp(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p)]


class GsAppearanceGrad(C.Structure):
    _fields_ = [("d_w1", C.c_void_p), ("d_b1", C.c_void_p), ("d_w2", C.c_void_p), ("d_b2", C.c_void_p),
                ("d_image_emb", C.c_void_p)]


class GsProjected(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("rect", C.c_void_p), ("tiles", C.c_void_p), ("depth_key", C.c_void_p),
                ("tile_order", C.c_void_p), ("tile_mask", C.c_void_p)]


GS_MAX_LEVELS = 8


class GsLodTable(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_parts", C.c_int32), ("part_min", C.c_void_p),
                ("part_max", C.c_void_p), ("offsets", C.c_void_p), ("counts", C.c_void_p),
                ("thresholds", C.c_float * GS_MAX_LEVELS), ("margin", C.c_float)]


class GsServeConfig(C.Structure):
    _fields_ = [("max_views_per_batch", C.c_int32), ("n_streams", C.c_int32), ("slot_capacity", C.c_int64),
                ("pair_capacity", C.c_int64), ("pixel_capacity", C.c_int64), ("queue_capacity", C.c_int32),
                ("pipeline_depth", C.c_int32), ("persistent_ctas", C.c_int32), ("pairs_per_gaussian", C.c_double)]


class GsCompletion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("batch_views", C.c_int32),
                ("n_gaussians", C.c_int64), ("n_pairs", C.c_int64), ("t_arrival", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


class GsServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("batches", C.c_int64),
                ("mean_batch_views", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("span_s", C.c_double),
                ("req_per_s", C.c_double), ("mpix_per_s", C.c_double), ("split_batches", C.c_int64),
                ("est_over_actual", C.c_double), ("rebinned_batches", C.c_int64)]


# exported symbols and their ctypes signatures
_P, _I32, _I64, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
SIGNATURES = {
    "gs_last_error": (C.c_char_p, []),
    "gs_version": (C.c_char_p, []),
    "gs_views_extent": (C.c_int, [_P, _I32, _P, _P]),
    "gs_project": (C.c_int, [_P, _P, _I32, _P, _P, _P]),
    "gs_bin_workspace_size": (_SZ, [_I64, _I64]),
    "gs_bin_sort": (C.c_int, [_P, _P, _I32, _I64, _I64, _P, _P, _P, _P, _SZ, _P]),
    "gs_render_fwd": (C.c_int, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "gs_render_fwd_seg": (C.c_int, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "gs_render_bwd_workspace_size": (_SZ, [_I64]),
    "gs_render_bwd": (C.c_int, [_P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "gs_render_bwd_grad2d": (_P, [_P]),
    "gs_composite_bwd": (C.c_int, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _I32, _I64, _P, _P, _SZ, _I32,
                                   _P]),
    "gs_seg_workspace_size": (_SZ, [_I64, _I64]),
    "gs_project_bwd": (C.c_int, [_P, _P, _I32, _P, _P, _P, _P, _P, _P, _I32, _P]),
    "gs_grads_zero": (C.c_int, [_P, _I64, _P]),
    "gs_render_count": (C.c_int, [_P, _P, _P, _P, _I32, _P, _P]),
    "gs_loss_workspace_size": (_SZ, [_I64]),
    "gs_loss_l1_depth": (C.c_int, [_P, _P, _P, _P, _P, _I64, C.c_float, _P, _P, _P, _P, _P, _SZ, _P]),
    "gs_loss_l1_depth_noalloc": (C.c_int, [_P, _P, _P, _P, _P, _I64, C.c_float, _P, _P, _P, _P, _P]),
    "gs_kernel_timing": (C.c_int, [C.c_int32]),
    "gs_kernel_timing_read": (C.c_int, [C.c_int32, _P, _P]),
    "gs_dssim_workspace_size": (_SZ, [_I32, _I32]),
    "gs_dssim": (C.c_int, [_P, _P, _I32, _I32, C.c_float, _P, _P, _P, _SZ, _P]),
    "gs_densify_accumulate": (C.c_int, [_P, _P, _P, _I32, _I64, _P, _P, _P, _P]),
    "gs_densify_workspace_size": (_SZ, [_I64]),
    "gs_densify_select": (C.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "gs_filter3d_rate": (C.c_int, [_P, _I64, _P, _I32, _P, _P]),
    "gs_filter3d_fwd": (C.c_int, [_P, _P, _P, _I64, C.c_float, _P, _P, _P]),
    "gs_filter3d_bwd": (C.c_int, [_P, _P, _P, _I64, C.c_float, _P, _P, _P, _P, _P]),
    "gs_appearance_workspace_size": (_SZ, [_I64]),
    "gs_appearance_fwd": (C.c_int, [_P, _I64, _P, _P, C.c_float, _P, _P, _P, _SZ, _P]),
    "gs_appearance_bwd": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, C.c_float, _P, _P, _P, _SZ, _P]),
    "gs_lod_select": (C.c_int, [_P, _P, _I64, _P, _P]),
    "gs_serve_create": (C.c_int, [_P, _P, _P, _P, _I32, _P]),
    "gs_serve_now": (C.c_double, [_P]),
    "gs_serve_submit": (C.c_int, [_P, _P, _I64, _P, _P, C.c_double, _P]),
    "gs_serve_poll": (C.c_int, [_P, _P, _I32, _I32, _P]),
    "gs_serve_stats_get": (C.c_int, [_P, _P]),
    "gs_serve_destroy": (C.c_int, [_P]),
}

_lock = threading.Lock()
_lib = None


def load() -> C.CDLL:
    """Loads libgs.so; raises if it has not been built (there is no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2507_23006_amd.build.build() "
                                   "(hipcc, gfx950); there is no CPU fallback")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(rc: int) -> None:
    if rc != GS_OK:
        raise GsError(rc, load().gs_last_error().decode(errors="replace"))


def make_cameras(cams) -> C.Array:
    """Camera objects with fx, fy, cx, cy, viewmat (4x4), width, height,
    near, far attributes -> gs_camera[n]."""
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        vm = [float(x) for row in c.viewmat for x in row]
        for k in range(16):
            arr[i].viewmat[k] = vm[k]
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].near_plane = float(getattr(c, "near", 0.01))
        arr[i].far_plane = float(getattr(c, "far", 1e10))
    return arr


def make_options(sh_degree=3, dilation=0.3, aa=False, bg=(0.0, 0.0, 0.0)) -> GsOptions:
    o = GsOptions()
    o.sh_degree, o.dilation, o.aa_compensate = int(sh_degree), float(dilation), int(bool(aa))
    for k in range(3):
        o.bg[k] = float(bg[k])
    return o
