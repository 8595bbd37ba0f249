"""ctypes binding of liblgs.so: the C ABI of include/lgs.h under the same names.

Argument marshalling only.  Pointers are passed as integers (device addresses,
e.g. torch's ``data_ptr()``) or None; streams as integer handles.  A non-OK status
raises LgsError carrying the library's message.  There is no fallback: if the
library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblgs.so")

LGS_OK = 0
LGS_ERR_INVALID_ARG = -1
LGS_ERR_UNSUPPORTED = -2
LGS_ERR_CAPACITY = -3
LGS_ERR_HIP = -4

LGS_F32 = 0
LGS_BF16 = 1
LGS_FP8_E4M3 = 2
DTYPES = {"f32": LGS_F32, "bf16": LGS_BF16, "fp8": LGS_FP8_E4M3}

TILE = 16


class LgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lgs status {status}: {msg}")
        self.status = status


class lgs_camera(ctypes.Structure):
    _fields_ = [("Rt", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


def make_camera(cam):
    """lgs_camera from any object with Rt[12], fx, fy, cx, cy, W, H."""
    c = lgs_camera()
    for i, v in enumerate(list(cam.Rt)):
        c.Rt[i] = float(v)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.W), int(cam.H)
    return c


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F = ctypes.c_float
_CAM = ctypes.POINTER(lgs_camera)
_SIG = {
    "lgs_project_fwd": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_bin_sort_workspace": [_I32, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_size_t)],
    "lgs_bin_sort": [_CAM, _I32, _P, _P, _P, _P, ctypes.c_size_t, _I64, _P, _P,
                     ctypes.POINTER(ctypes.c_int64), _P],
    "lgs_bin_sort_count": [_I32, _I64, _P, ctypes.POINTER(ctypes.c_int64), _P],
    "lgs_bin_sort_noalloc": [_CAM, _I32, _P, _P, _P, _I64, _P, _P, ctypes.POINTER(ctypes.c_int64), _P],
    "lgs_rasterize_topk_fwd": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                               _P, _P, _P],
    "lgs_feature_render_fwd": [_I32, _I32, _I32, _I32, _I32, ctypes.c_int, _P, _P, _P, _P,
                               ctypes.c_int, _P, _P],
    "lgs_feature_render_bwd": [_I32, _I32, _I32, _I32, _I32, ctypes.c_int, _P, _P, _P, _P,
                               ctypes.c_int, _P, _P, _P, _P],
    "lgs_feature_render_bwd_l1": [_I32, _I32, _I32, _I32, _I32, ctypes.c_int, _P, _P, _P, _P,
                                  ctypes.c_int, _P, _F, _P, _P, _P],
    "lgs_prune_stats": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_prune_select_workspace": [_I32, ctypes.POINTER(ctypes.c_size_t)],
    "lgs_prune_select": [_I32, _P, _P, _I32, _P, _F, _P, ctypes.c_size_t, _P, _P],
    "lgs_feature_render_fwd_bwd_l1": [_I32, _I32, _I32, _I32, _I32, ctypes.c_int, _P, _P, _P, _P,
                                      ctypes.c_int, _P, _P, _F, _P, _P, _P],
    "lgs_rasterize_topk_bwd": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                               _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_project_bwd": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_project_fwd_views": [_CAM, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_bin_sort_views": [_CAM, _I32, _I32, _P, _P, _P, _P, ctypes.c_size_t, _I64, _P, _P,
                           ctypes.POINTER(ctypes.c_int64), _P],
    "lgs_rasterize_topk_fwd_views": [_CAM, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                     _P, _P, _P, _P],
    "lgs_tile_order": [_CAM, _I32, _P, _P, _P, _P],
    "lgs_rasterize_topk_bwd_views": [_CAM, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                     _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_project_bwd_views": [_CAM, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_prune_stats_views": [_CAM, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_feature_render_vanilla_fwd": [_CAM, _P, _P, _P, _P, _P, _P, _I32, ctypes.c_int, _P, _P, ctypes.c_int,
                                       _P, _P],
    "lgs_feature_render_vanilla_bwd": [_CAM, _P, _P, _P, _P, _P, _P, _P, _I32, ctypes.c_int, _P, _P,
                                       ctypes.c_int, _P, _P, _P, _P, _P, _P],
    "lgs_project_bwd_pose": [_CAM, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lgs_quantize_features": [_I32, _I32, _P, ctypes.c_int, _P, _P, _P],
    "lgs_l1_grad": [_I64, ctypes.c_int, _P, _P, _F, _P, _P],
    "lgs_union_count": [_I64, _I32, _I32, _P, _P, ctypes.POINTER(ctypes.c_int64), _P],
    "lgs_mark_topk_rows": [_I64, _P, _I32, _I32, _P, _P],
    "lgs_zero_marked_rows": [_I32, _I32, _I32, _P, _P, _P],
    "lgs_quantize_marked_rows": [_I32, _I32, _I32, _P, _P, ctypes.c_int, _P, _P, _P],
}
EXPORTS = ["lgs_abi_version", "lgs_last_error", "lgs_supported_k", "lgs_tile_order_size", *_SIG]

_lib = None


def load():
    """Load liblgs.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime under the same soname; load it first so this
    # library binds to the runtime that owns torch's device memory and streams
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIG.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.lgs_abi_version.restype = ctypes.c_int
    L.lgs_last_error.restype = ctypes.c_char_p
    L.lgs_supported_k.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    L.lgs_supported_k.restype = ctypes.POINTER(ctypes.c_int32)
    L.lgs_tile_order_size.argtypes = [_I32, _I32, _I32]
    L.lgs_tile_order_size.restype = ctypes.c_int64
    _lib = L
    return L


def _check(status):
    if status != LGS_OK:
        raise LgsError(status, load().lgs_last_error().decode())
    return status


def lgs_abi_version():
    return load().lgs_abi_version()


def lgs_last_error():
    return load().lgs_last_error().decode()


def lgs_supported_k():
    n = ctypes.c_int32(0)
    p = load().lgs_supported_k(ctypes.byref(n))
    return [p[i] for i in range(n.value)]


def lgs_project_fwd(cam, n, means, log_scales, quats, opacity_logits, rgb, mean2d, conic, depth,
                    opacity, tile_rect, tiles_touched, stream=None):
    return _check(load().lgs_project_fwd(ctypes.byref(cam), n, means, log_scales, quats,
                                         opacity_logits, rgb, mean2d, conic, depth, opacity,
                                         tile_rect, tiles_touched, stream))


def lgs_bin_sort_workspace(n, width, height, max_pairs):
    b = ctypes.c_size_t(0)
    _check(load().lgs_bin_sort_workspace(n, width, height, max_pairs, ctypes.byref(b)))
    return b.value


def lgs_bin_sort(cam, n, depth, tile_rect, tiles_touched, workspace, ws_bytes, max_pairs,
                 sorted_ids, tile_ranges, stream=None, sync=True):
    """Returns (status, n_pairs); LGS_ERR_CAPACITY is returned, not raised.  With
    sync=False the C call gets n_pairs = NULL and n_pairs is returned as None."""
    m = ctypes.c_int64(0)
    st = load().lgs_bin_sort(ctypes.byref(cam), n, depth, tile_rect, tiles_touched, workspace,
                             ws_bytes, max_pairs, sorted_ids, tile_ranges,
                             ctypes.byref(m) if sync else None, stream)
    if st != LGS_ERR_CAPACITY:
        _check(st)
    return st, (m.value if sync else None)


def lgs_bin_sort_count(n, max_pairs, workspace, stream=None):
    """Returns (status, n_pairs); LGS_ERR_CAPACITY is returned, not raised."""
    m = ctypes.c_int64(0)
    st = load().lgs_bin_sort_count(n, max_pairs, workspace, ctypes.byref(m), stream)
    if st != LGS_ERR_CAPACITY:
        _check(st)
    return st, m.value


def lgs_bin_sort_noalloc(cam, n, depth, tile_rect, tiles_touched, max_pairs, sorted_ids, tile_ranges,
                         stream=None):
    """Returns (status, n_pairs); LGS_ERR_CAPACITY is returned, not raised."""
    m = ctypes.c_int64(0)
    st = load().lgs_bin_sort_noalloc(ctypes.byref(cam), n, depth, tile_rect, tiles_touched, max_pairs,
                                     sorted_ids, tile_ranges, ctypes.byref(m), stream)
    if st != LGS_ERR_CAPACITY:
        _check(st)
    return st, m.value


def lgs_rasterize_topk_fwd(cam, k, mean2d, conic, opacity, rgb, depth, sorted_ids, tile_ranges,
                           color, depth_map, alpha_map, T_final, n_contrib, topk_ids, topk_w,
                           stream=None, tile_order=None):
    return _check(load().lgs_rasterize_topk_fwd(ctypes.byref(cam), k, mean2d, conic, opacity, rgb,
                                                depth, sorted_ids, tile_ranges, color, depth_map,
                                                alpha_map, T_final, n_contrib, topk_ids, topk_w, tile_order,
                                                stream))


def lgs_feature_render_fwd(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w,
                           map_dt, F, stream=None):
    return _check(load().lgs_feature_render_fwd(width, height, views, k, d, feat_dt, feat, feat_scale,
                                                topk_ids, topk_w, map_dt, F, stream))


def lgs_feature_render_bwd(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w,
                           map_dt, dL_dF, dL_dfeat, dL_dtopkw, stream=None):
    return _check(load().lgs_feature_render_bwd(width, height, views, k, d, feat_dt, feat, feat_scale,
                                                topk_ids, topk_w, map_dt, dL_dF, dL_dfeat,
                                                dL_dtopkw, stream))


def lgs_feature_render_bwd_l1(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w,
                              map_dt, F_target, scale, dL_dfeat, dL_dtopkw, stream=None):
    return _check(load().lgs_feature_render_bwd_l1(width, height, views, k, d, feat_dt, feat, feat_scale,
                                                   topk_ids, topk_w, map_dt, F_target, scale, dL_dfeat,
                                                   dL_dtopkw, stream))


def lgs_feature_render_fwd_bwd_l1(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids,
                                  topk_w, map_dt, F, F_target, scale, dL_dfeat, dL_dtopkw, stream=None):
    return _check(load().lgs_feature_render_fwd_bwd_l1(width, height, views, k, d, feat_dt, feat,
                                                       feat_scale, topk_ids, topk_w, map_dt, F, F_target,
                                                       scale, dL_dfeat, dL_dtopkw, stream))


def lgs_prune_stats(cam, k, mean2d, conic, opacity, sorted_ids, tile_ranges, n_contrib, topk_ids, topk_count,
                    max_w, stream=None, tile_order=None):
    return _check(load().lgs_prune_stats(ctypes.byref(cam), k, mean2d, conic, opacity, sorted_ids, tile_ranges,
                                         n_contrib, topk_ids, topk_count, max_w, tile_order, stream))


def lgs_prune_select_workspace(n):
    b = ctypes.c_size_t(0)
    _check(load().lgs_prune_select_workspace(n, ctypes.byref(b)))
    return b.value


def lgs_prune_select(n, topk_count, max_w, count_below, expo, keep_ratio, workspace, ws_bytes, survive,
                     stream=None):
    return _check(load().lgs_prune_select(n, topk_count, max_w, count_below, expo, keep_ratio, workspace,
                                          ws_bytes, survive, stream))


def lgs_rasterize_topk_bwd(cam, k, mean2d, conic, opacity, rgb, depth, sorted_ids, tile_ranges,
                           T_final, n_contrib, topk_ids, topk_w, dL_dcolor, dL_ddepth, dL_dalpha,
                           dL_dtopkw, dL_dmean2d, dL_dconic, dL_dopacity, dL_drgb, dL_ddepth_g,
                           stream=None, tile_order=None):
    return _check(load().lgs_rasterize_topk_bwd(ctypes.byref(cam), k, mean2d, conic, opacity, rgb,
                                                depth, sorted_ids, tile_ranges, T_final, n_contrib,
                                                topk_ids, topk_w, dL_dcolor, dL_ddepth, dL_dalpha,
                                                dL_dtopkw, dL_dmean2d, dL_dconic, dL_dopacity,
                                                dL_drgb, dL_ddepth_g, tile_order, stream))


def lgs_project_bwd(cam, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                    dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats,
                    dL_dopacity_logits, stream=None):
    return _check(load().lgs_project_bwd(ctypes.byref(cam), n, means, log_scales, quats,
                                         opacity_logits, rgb, dL_dmean2d, dL_dconic, dL_dopacity,
                                         dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats,
                                         dL_dopacity_logits, stream))


def lgs_project_bwd_pose(cam, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                         dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats, dL_dopacity_logits,
                         dL_dpose, stream=None):
    return _check(load().lgs_project_bwd_pose(ctypes.byref(cam), n, means, log_scales, quats, opacity_logits,
                                              rgb, dL_dmean2d, dL_dconic, dL_dopacity, dL_ddepth_g, dL_dmeans,
                                              dL_dlog_scales, dL_dquats, dL_dopacity_logits, dL_dpose, stream))


def lgs_feature_render_vanilla_fwd(cam, mean2d, conic, opacity, sorted_ids, tile_ranges, n_contrib, d, feat_dt,
                                   feat, feat_scale, map_dt, F, stream=None):
    return _check(load().lgs_feature_render_vanilla_fwd(ctypes.byref(cam), mean2d, conic, opacity, sorted_ids,
                                                        tile_ranges, n_contrib, d, feat_dt, feat, feat_scale, map_dt,
                                                        F, stream))


def lgs_feature_render_vanilla_bwd(cam, mean2d, conic, opacity, sorted_ids, tile_ranges, T_final, n_contrib, d,
                                   feat_dt, feat, feat_scale, map_dt, dL_dF, dL_dfeat, dL_dmean2d, dL_dconic,
                                   dL_dopacity, stream=None):
    return _check(load().lgs_feature_render_vanilla_bwd(ctypes.byref(cam), mean2d, conic, opacity, sorted_ids,
                                                        tile_ranges, T_final, n_contrib, d, feat_dt, feat, feat_scale,
                                                        map_dt, dL_dF, dL_dfeat, dL_dmean2d, dL_dconic, dL_dopacity,
                                                        stream))


def camera_array(cams):
    """A ctypes array of lgs_camera (the host array the *_views calls take)."""
    arr = (lgs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c
    return arr


def lgs_project_fwd_views(cams, views, n, means, log_scales, quats, opacity_logits, rgb, mean2d, conic, depth,
                          opacity, tile_rect, tiles_touched, stream=None):
    return _check(load().lgs_project_fwd_views(cams, views, n, means, log_scales, quats, opacity_logits, rgb, mean2d,
                                               conic, depth, opacity, tile_rect, tiles_touched, stream))


def lgs_bin_sort_views(cams, views, n, depth, tile_rect, tiles_touched, workspace, ws_bytes, max_pairs,
                       sorted_ids, tile_ranges, stream=None, sync=True):
    """As lgs_bin_sort; returns (status, n_pairs), LGS_ERR_CAPACITY returned, not raised."""
    m = ctypes.c_int64(0)
    st = load().lgs_bin_sort_views(cams, views, n, depth, tile_rect, tiles_touched, workspace, ws_bytes, max_pairs,
                                   sorted_ids, tile_ranges, ctypes.byref(m) if sync else None, stream)
    if st != LGS_ERR_CAPACITY:
        _check(st)
    return st, (m.value if sync else None)


def lgs_rasterize_topk_fwd_views(cams, views, k, n, mean2d, conic, opacity, rgb, depth, sorted_ids, tile_ranges,
                                 color, depth_map, alpha_map, T_final, n_contrib, topk_ids, topk_w, stream=None,
                                 tile_order=None):
    return _check(load().lgs_rasterize_topk_fwd_views(cams, views, k, n, mean2d, conic, opacity, rgb, depth,
                                                      sorted_ids, tile_ranges, color, depth_map, alpha_map,
                                                      T_final, n_contrib, topk_ids, topk_w, tile_order, stream))


def lgs_tile_order_size(width, height, views):
    return int(load().lgs_tile_order_size(width, height, views))


def lgs_tile_order(cams, views, tile_ranges, n_contrib, order, stream=None):
    return _check(load().lgs_tile_order(cams, views, tile_ranges, n_contrib, order, stream))


def lgs_rasterize_topk_bwd_views(cams, views, k, n, mean2d, conic, opacity, rgb, depth, sorted_ids, tile_ranges,
                                 T_final, n_contrib, topk_ids, topk_w, dL_dcolor, dL_ddepth, dL_dalpha, dL_dtopkw,
                                 dL_dmean2d, dL_dconic, dL_dopacity, dL_drgb, dL_ddepth_g, stream=None,
                                 tile_order=None):
    return _check(load().lgs_rasterize_topk_bwd_views(cams, views, k, n, mean2d, conic, opacity, rgb, depth,
                                                      sorted_ids, tile_ranges, T_final, n_contrib, topk_ids,
                                                      topk_w, dL_dcolor, dL_ddepth, dL_dalpha, dL_dtopkw,
                                                      dL_dmean2d, dL_dconic, dL_dopacity, dL_drgb, dL_ddepth_g,
                                                      tile_order, stream))


def lgs_project_bwd_views(cams, views, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                          dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats, dL_dopacity_logits,
                          dL_dpose, stream=None):
    return _check(load().lgs_project_bwd_views(cams, views, n, means, log_scales, quats, opacity_logits, rgb,
                                               dL_dmean2d, dL_dconic, dL_dopacity, dL_ddepth_g, dL_dmeans,
                                               dL_dlog_scales, dL_dquats, dL_dopacity_logits, dL_dpose, stream))


def lgs_prune_stats_views(cams, views, k, n, mean2d, conic, opacity, sorted_ids, tile_ranges, n_contrib, topk_ids,
                          topk_count, max_w, stream=None, tile_order=None):
    return _check(load().lgs_prune_stats_views(cams, views, k, n, mean2d, conic, opacity, sorted_ids, tile_ranges,
                                               n_contrib, topk_ids, topk_count, max_w, tile_order, stream))


def lgs_quantize_features(n, d, src, dst_dt, dst, dst_scale, stream=None):
    return _check(load().lgs_quantize_features(n, d, src, dst_dt, dst, dst_scale, stream))


def lgs_l1_grad(n, dt, x, target, scale, grad, stream=None):
    return _check(load().lgs_l1_grad(n, dt, x, target, scale, grad, stream))


def lgs_mark_topk_rows(n_slots, topk_ids, n, gen, row_gen, stream=None):
    return _check(load().lgs_mark_topk_rows(n_slots, topk_ids, n, gen, row_gen, stream))


def lgs_zero_marked_rows(n, d, gen, row_gen, table, stream=None):
    return _check(load().lgs_zero_marked_rows(n, d, gen, row_gen, table, stream))


def lgs_quantize_marked_rows(n, d, gen, row_gen, src, dst_dt, dst, dst_scale, stream=None):
    return _check(load().lgs_quantize_marked_rows(n, d, gen, row_gen, src, dst_dt, dst, dst_scale, stream))


def lgs_union_count(n_pix, k, n, topk_ids, flags, stream=None):
    c = ctypes.c_int64(0)
    _check(load().lgs_union_count(n_pix, k, n, topk_ids, flags, ctypes.byref(c), stream))
    return c.value
