"""Torch-facing renderer: device memory and streams from PyTorch, every step of the
path in liblgs.so (see lgs.py for the C ABI).

    r = Renderer(K=4, feat_dtype="bf16")
    C, D, O, F = r.render(params, camera)            # a torch.autograd.Function

`params` is a dict of CUDA tensors: means[N,3], log_scales[N,3], quats[N,4],
opacity_logits[N], rgb[N,3] and feat[N,D] (FP32 master copy).  For BF16 / FP8
storage the kernels read a quantized copy of the master table; render() quantizes
it again whenever the master tensor changed since the copy was made (a different
tensor, or an in-place update, which advances the tensor's version counter), so a
stale copy is never rendered.  ``r.set_features(feat)`` refreshes it explicitly.
"""
from __future__ import annotations

import ctypes

import torch

from . import lgs

_TORCH_MAP = {"f32": torch.float32, "bf16": torch.bfloat16}


def _p(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("liblgs needs contiguous CUDA tensors")


class Binner:
    """Reusable workspace and pair buffer for lgs_bin_sort; grows on demand.

    sync=False keeps the pair count on the device after the first call (which sizes
    the buffers with a margin): no host round trip per frame, so the host can queue
    the rest of the frame.  `count()` reads the count of the last call and tells
    whether it fitted; a call that did not fit must be repeated after `count()` grew
    the buffers."""

    def __init__(self, device="cuda", sync=True):
        self.device = device
        self.sync = sync
        self.cap = 0
        self.ws = None
        self.ids = None
        self.n = 0

    def _ensure(self, n, W, H, cap):
        need = lgs.lgs_bin_sort_workspace(n, W, H, cap)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        if self.ids is None or self.ids.numel() < max(cap, 1):
            self.ids = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        self.cap = cap
        self.dims = (W, H)

    def __call__(self, cam, n, depth, tile_rect, touched, views=1):
        """Bins n Gaussians of one view, or, with views > 1, the views * n records of a
        batched projection (cam: the camera array of the views)."""
        c0 = cam[0] if views > 1 else cam
        ntiles = ((c0.width + 15) // 16) * ((c0.height + 15) // 16) * views
        ranges = torch.empty(ntiles * 2, dtype=torch.int32, device=self.device)
        rec = n * views
        first = self.cap == 0 or self.n != rec
        if self.cap == 0:
            self._ensure(rec, c0.width, c0.height, max(4 * rec, 1 << 16))
        self.n = rec

        def call(ws, sync):
            if views > 1:
                return lgs.lgs_bin_sort_views(cam, views, n, _p(depth), _p(tile_rect), _p(touched), _p(ws),
                                              ws.numel(), self.cap, _p(self.ids), _p(ranges), _stream(), sync=sync)
            return lgs.lgs_bin_sort(cam, n, _p(depth), _p(tile_rect), _p(touched), _p(ws), ws.numel(), self.cap,
                                    _p(self.ids), _p(ranges), _stream(), sync=sync)

        if not self.sync and not first:
            call(self.ws, False)
            return self.ids, ranges.view(ntiles, 2), None
        while True:
            ws = self.ws
            st, m = call(ws, True)
            if st == lgs.LGS_OK:
                out = self.ids[:m]   # the pairs this call wrote (kept alive if the buffer grows)
                if not self.sync and (m * 3 > self.cap * 2 or self.cap > 2 * m + 65536):
                    # room for frames that bring up to half as many pairs again (the
                    # asynchronous calls size their grids for the capacity, so a first
                    # guess far above the count is cut down too); the new sizes serve
                    # the next calls
                    self._ensure(rec, c0.width, c0.height, int(m * 1.5) + 4096)
                return out, ranges.view(ntiles, 2), m
            self._ensure(rec, c0.width, c0.height, int(m * 1.5) + 4096)

    def count(self):
        """(pair count, fitted) of the last call; grows the buffers if it did not fit."""
        st, m = lgs.lgs_bin_sort_count(self.n, self.cap, _p(self.ws), _stream())
        if st != lgs.LGS_OK:
            self._ensure(self.n, self.dims[0], self.dims[1], int(m * 1.5) + 4096)
            return m, False
        return m, True


def project(cam, P):
    n = P["means"].shape[0]
    dev = P["means"].device
    out = dict(mean2d=torch.empty(n, 2, device=dev), conic=torch.empty(n, 3, device=dev),
               depth=torch.empty(n, device=dev), opacity=torch.empty(n, device=dev),
               tile_rect=torch.empty(n, 4, dtype=torch.int32, device=dev),
               tiles_touched=torch.empty(n, dtype=torch.int32, device=dev))
    _need_cuda(*(P[k] for k in ("means", "log_scales", "quats", "opacity_logits", "rgb")))
    lgs.lgs_project_fwd(cam, n, _p(P["means"]), _p(P["log_scales"]), _p(P["quats"]),
                        _p(P["opacity_logits"]), _p(P["rgb"]), _p(out["mean2d"]), _p(out["conic"]),
                        _p(out["depth"]), _p(out["opacity"]), _p(out["tile_rect"]),
                        _p(out["tiles_touched"]), _stream())
    return out


def tile_order(cams, ranges, views=1, n_contrib=None, out=None):
    """The blend's dispatch order for these tile ranges (longest runs first within each
    XCD; it changes no result), weighted by the pair counts, or with the forward's
    n_contrib by the list length the adjoint walks.  cams: one camera, or the camera
    array of `views`."""
    cam0 = cams[0] if views > 1 else cams
    size = lgs.lgs_tile_order_size(cam0.width, cam0.height, views)
    if out is None or out.numel() < size:
        out = torch.empty(size, dtype=torch.int32, device=ranges.device)
    _need_cuda(ranges, out)
    if n_contrib is not None:
        _need_cuda(n_contrib)
        if n_contrib.numel() != views * cam0.width * cam0.height or n_contrib.dtype != torch.int32:
            raise ValueError("tile_order: n_contrib must be the forward's int32 map of every view")
    lgs.lgs_tile_order(cams if views > 1 else ctypes.byref(cams), views, _p(ranges), _p(n_contrib), _p(out),
                       _stream())
    return out


def rasterize(cam, K, proj, rgb, sorted_ids, ranges, order=None):
    H, W = cam.height, cam.width
    dev = rgb.device
    out = dict(C=torch.empty(H, W, 3, device=dev), D=torch.empty(H, W, device=dev),
               O=torch.empty(H, W, device=dev), T=torch.empty(H, W, device=dev),
               n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev),
               ids=torch.empty(H, W, K, dtype=torch.int32, device=dev),
               w=torch.empty(H, W, K, device=dev))
    lgs.lgs_rasterize_topk_fwd(cam, K, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                               _p(rgb), _p(proj["depth"]), _p(sorted_ids), _p(ranges), _p(out["C"]),
                               _p(out["D"]), _p(out["O"]), _p(out["T"]), _p(out["n_contrib"]),
                               _p(out["ids"]), _p(out["w"]), _stream(), tile_order=_p(order))
    return out


def prune_stats(cam, K, proj, sorted_ids, ranges, fwd, topk_count, max_w, order=None):
    """Sec. 3.3 statistics of one view, accumulated: Top-K participation counts
    (int32 [N]) and the maximum blending weight S (FP32 [N], Eq. 5)."""
    _need_cuda(topk_count, max_w)
    lgs.lgs_prune_stats(cam, K, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]), _p(sorted_ids),
                        _p(ranges), _p(fwd["n_contrib"]), _p(fwd["ids"]), _p(topk_count), _p(max_w), _stream(),
                        tile_order=_p(order))


def prune_select(topk_count, max_w, count_below, expo, keep_ratio=0.5):
    """Eq. 6 survival draw over the candidates topk_count < count_below: returns a
    uint8 [N] mask, 1 = keep.  expo: the caller's Exp(1) variates, FP32 [N]."""
    n = topk_count.shape[0]
    _need_cuda(topk_count, max_w, expo)
    need = lgs.lgs_prune_select_workspace(n)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=topk_count.device)
    survive = torch.empty(n, dtype=torch.uint8, device=topk_count.device)
    lgs.lgs_prune_select(n, _p(topk_count), _p(max_w), int(count_below), _p(expo), float(keep_ratio), _p(ws),
                         ws.numel(), _p(survive), _stream())
    return survive


def quantize(feat, dtype, out=None):
    """FP32 [N,D] -> storage (bf16 tensor, or (uint8 codes, f32 scale) for fp8).  `out`:
    an existing (store, scale) pair of the right shapes and dtypes to write into."""
    n, d = feat.shape
    _need_cuda(feat)
    if dtype == "f32":
        return feat, None
    if dtype not in ("bf16", "fp8"):
        raise ValueError(dtype)
    sdt = torch.bfloat16 if dtype == "bf16" else torch.uint8
    if out is None:
        store = torch.empty(n, d, dtype=sdt, device=feat.device)
        scale = torch.empty(n, dtype=torch.float32, device=feat.device) if dtype == "fp8" else None
    else:
        store, scale = out
        if store.shape != (n, d) or store.dtype != sdt or not store.is_contiguous():
            raise ValueError("quantize: store must be a contiguous [n, d] tensor of the storage dtype")
        if dtype == "fp8" and (scale is None or scale.shape != (n,) or scale.dtype != torch.float32):
            raise ValueError("quantize: FP8 needs a float32 scale of n rows")
    if dtype == "bf16":
        lgs.lgs_quantize_features(n, d, _p(feat), lgs.LGS_BF16, _p(store), None, _stream())
        return store, None
    lgs.lgs_quantize_features(n, d, _p(feat), lgs.LGS_FP8_E4M3, _p(store), _p(scale), _stream())
    return store, scale


def feature_fwd(ids, w, feat_store, feat_scale, feat_dtype, map_dtype, views=1):
    """Eq. 3-4 for per-pixel Top-K ids/w [V*H, W, K] (or [H, W, K])."""
    K = ids.shape[-1]
    Hs, W = ids.shape[0], ids.shape[1]
    d = feat_store.shape[1]
    F = torch.empty(Hs, W, d, dtype=_TORCH_MAP[map_dtype], device=ids.device)
    _need_cuda(ids, w, feat_store, feat_scale)
    lgs.lgs_feature_render_fwd(W, Hs // views, views, K, d, lgs.DTYPES[feat_dtype], _p(feat_store),
                               _p(feat_scale), _p(ids), _p(w), lgs.DTYPES[map_dtype], _p(F), _stream())
    return F


def feature_bwd(ids, w, feat_store, feat_scale, feat_dtype, map_dtype, dF, dfeat, views=1):
    K = ids.shape[-1]
    Hs, W = ids.shape[0], ids.shape[1]
    d = feat_store.shape[1]
    dtw = torch.empty(Hs, W, K, device=ids.device)
    _need_cuda(ids, w, feat_store, feat_scale, dF, dfeat)
    lgs.lgs_feature_render_bwd(W, Hs // views, views, K, d, lgs.DTYPES[feat_dtype], _p(feat_store),
                               _p(feat_scale), _p(ids), _p(w), lgs.DTYPES[map_dtype], _p(dF),
                               _p(dfeat), _p(dtw), _stream())
    return dtw


def feature_bwd_l1(ids, w, feat_store, feat_scale, feat_dtype, map_dtype, F_target, scale, dfeat,
                   views=1):
    """Feature adjoint of the L1 loss scale * |F - F_target|_1 without materialising dL/dF."""
    K = ids.shape[-1]
    Hs, W = ids.shape[0], ids.shape[1]
    d = feat_store.shape[1]
    dtw = torch.empty(Hs, W, K, device=ids.device)
    _need_cuda(ids, w, feat_store, feat_scale, F_target, dfeat)
    lgs.lgs_feature_render_bwd_l1(W, Hs // views, views, K, d, lgs.DTYPES[feat_dtype], _p(feat_store),
                                  _p(feat_scale), _p(ids), _p(w), lgs.DTYPES[map_dtype], _p(F_target),
                                  float(scale), _p(dfeat), _p(dtw), _stream())
    return dtw


def feature_fwd_bwd_l1(ids, w, feat_store, feat_scale, feat_dtype, map_dtype, F_target, scale, dfeat,
                       views=1):
    """The feature render and its L1 adjoint in one pass: returns (F, dL/dw), the same
    as feature_fwd followed by feature_bwd_l1."""
    K = ids.shape[-1]
    Hs, W = ids.shape[0], ids.shape[1]
    d = feat_store.shape[1]
    F = torch.empty(Hs, W, d, dtype=_TORCH_MAP[map_dtype], device=ids.device)
    dtw = torch.empty(Hs, W, K, device=ids.device)
    _need_cuda(ids, w, feat_store, feat_scale, F_target, dfeat)
    lgs.lgs_feature_render_fwd_bwd_l1(W, Hs // views, views, K, d, lgs.DTYPES[feat_dtype], _p(feat_store),
                                      _p(feat_scale), _p(ids), _p(w), lgs.DTYPES[map_dtype], _p(F),
                                      _p(F_target), float(scale), _p(dfeat), _p(dtw), _stream())
    return F, dtw


def feature_vanilla_fwd(cam, proj, sorted_ids, ranges, fwd, feat_store, feat_scale, feat_dtype):
    """The vanilla alpha-blended feature map (every blended Gaussian, Eq. 1 on the
    features): BF16 [H, W, D] from BF16 or FP8 storage."""
    H, W = cam.height, cam.width
    d = feat_store.shape[1]
    F = torch.empty(H, W, d, dtype=torch.bfloat16, device=feat_store.device)
    _need_cuda(feat_store, feat_scale)
    lgs.lgs_feature_render_vanilla_fwd(cam, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                                       _p(sorted_ids), _p(ranges), _p(fwd["n_contrib"]), d, lgs.DTYPES[feat_dtype],
                                       _p(feat_store), _p(feat_scale), lgs.LGS_BF16, _p(F), _stream())
    return F


def feature_vanilla_bwd(cam, proj, sorted_ids, ranges, fwd, feat_store, feat_scale, feat_dtype, dF, dfeat, grads):
    """Adjoint of the vanilla feature render: dL/df rows into dfeat and the feature term
    of the screen-space gradients into grads (mean2d, conic, opacity), all accumulated."""
    d = feat_store.shape[1]
    _need_cuda(feat_store, feat_scale, dF, dfeat)
    lgs.lgs_feature_render_vanilla_bwd(cam, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                                       _p(sorted_ids), _p(ranges), _p(fwd["T"]), _p(fwd["n_contrib"]), d,
                                       lgs.DTYPES[feat_dtype], _p(feat_store), _p(feat_scale), lgs.LGS_BF16, _p(dF),
                                       _p(dfeat), _p(grads["mean2d"]), _p(grads["conic"]), _p(grads["opacity"]),
                                       _stream())


def rasterize_bwd(cam, K, proj, rgb, sorted_ids, ranges, fwd, gC, gD, gO, dtw, grads, order=None):
    lgs.lgs_rasterize_topk_bwd(cam, K, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                               _p(rgb), _p(proj["depth"]), _p(sorted_ids), _p(ranges), _p(fwd["T"]),
                               _p(fwd["n_contrib"]), _p(fwd["ids"]), _p(fwd["w"]), _p(gC), _p(gD),
                               _p(gO), _p(dtw), _p(grads["mean2d"]), _p(grads["conic"]),
                               _p(grads["opacity"]), _p(grads["rgb"]), _p(grads["depth"]), _stream(),
                               tile_order=_p(order))


def project_bwd(cam, P, sgrads, pgrads):
    n = P["means"].shape[0]
    lgs.lgs_project_bwd(cam, n, _p(P["means"]), _p(P["log_scales"]), _p(P["quats"]),
                        _p(P["opacity_logits"]), _p(P["rgb"]), _p(sgrads["mean2d"]),
                        _p(sgrads["conic"]), _p(sgrads["opacity"]), _p(sgrads["depth"]),
                        _p(pgrads["means"]), _p(pgrads["log_scales"]), _p(pgrads["quats"]),
                        _p(pgrads["opacity_logits"]), _stream())


def project_bwd_pose(cam, P, sgrads, dpose, pgrads=None):
    """Camera-pose gradient dL/d(rho, phi) accumulated into dpose (FP32 [6]), and the
    parameter gradients into pgrads when given (one pass)."""
    n = P["means"].shape[0]
    pg = pgrads or {}
    lgs.lgs_project_bwd_pose(cam, n, _p(P["means"]), _p(P["log_scales"]), _p(P["quats"]),
                             _p(P["opacity_logits"]), _p(P["rgb"]), _p(sgrads["mean2d"]), _p(sgrads["conic"]),
                             _p(sgrads["opacity"]), _p(sgrads["depth"]), _p(pg.get("means")),
                             _p(pg.get("log_scales")), _p(pg.get("quats")), _p(pg.get("opacity_logits")),
                             _p(dpose), _stream())


# ---------------------------------------------------------------- batched views
# Several keyframes of one size in one launch per step (Sec. 3.4).  `cams` is the
# ctypes camera array (lgs.camera_array); projected records and screen-space
# gradients are [views * n, ...]; per-pixel outputs stack the views as [views * H, W, ...].

def project_views(cams, P):
    n = P["means"].shape[0]
    V = len(cams)
    dev = P["means"].device
    out = dict(mean2d=torch.empty(V * n, 2, device=dev), conic=torch.empty(V * n, 3, device=dev),
               depth=torch.empty(V * n, device=dev), opacity=torch.empty(V * n, device=dev),
               tile_rect=torch.empty(V * n, 4, dtype=torch.int32, device=dev),
               tiles_touched=torch.empty(V * n, dtype=torch.int32, device=dev))
    _need_cuda(*(P[k] for k in ("means", "log_scales", "quats", "opacity_logits", "rgb")))
    lgs.lgs_project_fwd_views(cams, V, n, _p(P["means"]), _p(P["log_scales"]), _p(P["quats"]),
                              _p(P["opacity_logits"]), _p(P["rgb"]), _p(out["mean2d"]), _p(out["conic"]),
                              _p(out["depth"]), _p(out["opacity"]), _p(out["tile_rect"]), _p(out["tiles_touched"]),
                              _stream())
    return out


def rasterize_views(cams, K, n, proj, rgb, sorted_ids, ranges, order=None):
    V = len(cams)
    H, W = cams[0].height, cams[0].width
    dev = rgb.device
    out = dict(C=torch.empty(V * H, W, 3, device=dev), D=torch.empty(V * H, W, device=dev),
               O=torch.empty(V * H, W, device=dev), T=torch.empty(V * H, W, device=dev),
               n_contrib=torch.empty(V * H, W, dtype=torch.int32, device=dev),
               ids=torch.empty(V * H, W, K, dtype=torch.int32, device=dev),
               w=torch.empty(V * H, W, K, device=dev))
    lgs.lgs_rasterize_topk_fwd_views(cams, V, K, n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                                     _p(rgb), _p(proj["depth"]), _p(sorted_ids), _p(ranges), _p(out["C"]),
                                     _p(out["D"]), _p(out["O"]), _p(out["T"]), _p(out["n_contrib"]),
                                     _p(out["ids"]), _p(out["w"]), _stream(), tile_order=_p(order))
    return out


def rasterize_bwd_views(cams, K, n, proj, rgb, sorted_ids, ranges, fwd, gC, gD, gO, dtw, grads, order=None):
    lgs.lgs_rasterize_topk_bwd_views(cams, len(cams), K, n, _p(proj["mean2d"]), _p(proj["conic"]),
                                     _p(proj["opacity"]), _p(rgb), _p(proj["depth"]), _p(sorted_ids), _p(ranges),
                                     _p(fwd["T"]), _p(fwd["n_contrib"]), _p(fwd["ids"]), _p(fwd["w"]), _p(gC),
                                     _p(gD), _p(gO), _p(dtw), _p(grads["mean2d"]), _p(grads["conic"]),
                                     _p(grads["opacity"]), _p(grads["rgb"]), _p(grads["depth"]), _stream(),
                                     tile_order=_p(order))


def project_bwd_views(cams, P, sgrads, pgrads=None, dpose=None):
    n = P["means"].shape[0]
    pg = pgrads or {}
    lgs.lgs_project_bwd_views(cams, len(cams), n, _p(P["means"]), _p(P["log_scales"]), _p(P["quats"]),
                              _p(P["opacity_logits"]), _p(P["rgb"]), _p(sgrads["mean2d"]), _p(sgrads["conic"]),
                              _p(sgrads["opacity"]), _p(sgrads["depth"]), _p(pg.get("means")),
                              _p(pg.get("log_scales")), _p(pg.get("quats")), _p(pg.get("opacity_logits")),
                              _p(dpose), _stream())


def screen_grad_buffers_views(n, views, device):
    """Record-indexed screen-space gradients of `views` views (rgb per Gaussian)."""
    r = n * views
    return dict(mean2d=torch.zeros(r, 2, device=device), conic=torch.zeros(r, 3, device=device),
                opacity=torch.zeros(r, device=device), rgb=torch.zeros(n, 3, device=device),
                depth=torch.zeros(r, device=device))


def screen_grad_buffers(n, device):
    return dict(mean2d=torch.zeros(n, 2, device=device), conic=torch.zeros(n, 3, device=device),
                opacity=torch.zeros(n, device=device), rgb=torch.zeros(n, 3, device=device),
                depth=torch.zeros(n, device=device))


def l1_grad(x, target, scale):
    """scale * sign(x - target) in x's dtype (f32 or bf16)."""
    g = torch.empty_like(x)
    dt = lgs.LGS_BF16 if x.dtype == torch.bfloat16 else lgs.LGS_F32
    _need_cuda(x, target)
    lgs.lgs_l1_grad(x.numel(), dt, _p(x), _p(target), float(scale), _p(g), _stream())
    return g


class SparseGradRows:
    """Clears a dense feature-gradient table [n, d] between steps by zeroing only the
    rows the previous step's Top-K lists named (the only rows the feature adjoint
    writes).  Per step: clear(), mark(topk_ids), then the adjoint.  The same marks
    name the rows of the quantized store the step's feature kernels read, which
    quantize() refreshes from the FP32 table."""

    def __init__(self, table):
        self.table = table
        n = table.shape[0]
        self.row_gen = torch.full((n,), -2**31, dtype=torch.int32, device=table.device)
        self.gen = 0

    def clear(self):
        n, d = self.table.shape
        lgs.lgs_zero_marked_rows(n, d, self.gen - 1, _p(self.row_gen), _p(self.table), _stream())

    def mark(self, topk_ids):
        n = self.table.shape[0]
        lgs.lgs_mark_topk_rows(topk_ids.numel(), _p(topk_ids), n, self.gen, _p(self.row_gen), _stream())
        self.gen += 1

    def quantize(self, feat, dtype, out):
        """Refreshes the storage form `out` = (store, scale) from the FP32 table `feat`
        in the rows the last mark() named (the rows the step's feature kernels read)."""
        n, d = feat.shape
        _need_cuda(feat)
        store, scale = out
        sdt = torch.bfloat16 if dtype == "bf16" else torch.uint8
        if dtype not in ("bf16", "fp8") or store.shape != (n, d) or store.dtype != sdt or \
                not (store.is_contiguous() and feat.is_contiguous()) or n != self.table.shape[0]:
            raise ValueError("quantize: a contiguous [n, d] store of the storage dtype over the marked table")
        if dtype == "fp8" and (scale is None or scale.shape != (n,) or scale.dtype != torch.float32):
            raise ValueError("quantize: FP8 needs a float32 scale of n rows")
        lgs.lgs_quantize_marked_rows(n, d, self.gen - 1, _p(self.row_gen), _p(feat),
                                     lgs.LGS_BF16 if dtype == "bf16" else lgs.LGS_FP8_E4M3, _p(store),
                                     _p(scale) if scale is not None else None, _stream())
        return store, scale


def union_count(ids, n):
    flags = torch.empty(n + 1, dtype=torch.int32, device=ids.device)
    K = ids.shape[-1]
    return lgs.lgs_union_count(ids.numel() // K, K, n, _p(ids), _p(flags), _stream())


class _TopKRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, rgb, feat, r, cam):
        P = dict(means=means, log_scales=log_scales, quats=quats, opacity_logits=opacity_logits,
                 rgb=rgb)
        proj = project(cam, P)
        ids, ranges, _ = r.binner(cam, means.shape[0], proj["depth"], proj["tile_rect"],
                                  proj["tiles_touched"])
        order = tile_order(cam, ranges)
        fw = rasterize(cam, r.K, proj, rgb, ids, ranges, order)
        store, scale = (feat, None) if r.feat_dtype == "f32" else (r.store, r.scale)
        F = feature_fwd(fw["ids"], fw["w"], store, scale, r.feat_dtype, r.map_dtype)
        ctx.r, ctx.cam, ctx.P, ctx.proj, ctx.fw = r, cam, P, proj, fw
        ctx.sorted_ids, ctx.ranges, ctx.order = ids.clone(), ranges, order
        ctx.store, ctx.scale, ctx.n, ctx.d = store, scale, means.shape[0], feat.shape[1]
        return fw["C"], fw["D"], fw["O"], F

    @staticmethod
    def backward(ctx, gC, gD, gO, gF):
        r, cam, fw = ctx.r, ctx.cam, ctx.fw
        dev = fw["C"].device
        gC = torch.zeros_like(fw["C"]) if gC is None else gC.contiguous()
        gD = torch.zeros_like(fw["D"]) if gD is None else gD.contiguous()
        gO = None if gO is None else gO.contiguous()
        dfeat = torch.zeros(ctx.n, ctx.d, device=dev)
        if gF is not None:
            dtw = feature_bwd(fw["ids"], fw["w"], ctx.store, ctx.scale, r.feat_dtype, r.map_dtype,
                              gF.contiguous(), dfeat)
        else:
            dtw = None
        sg = screen_grad_buffers(ctx.n, dev)
        rasterize_bwd(cam, r.K, ctx.proj, ctx.P["rgb"], ctx.sorted_ids, ctx.ranges, fw, gC, gD, gO,
                      dtw, sg, tile_order(cam, ctx.ranges, n_contrib=fw["n_contrib"], out=ctx.order))
        pg = dict(means=torch.zeros(ctx.n, 3, device=dev), log_scales=torch.zeros(ctx.n, 3, device=dev),
                  quats=torch.zeros(ctx.n, 4, device=dev), opacity_logits=torch.zeros(ctx.n, device=dev))
        project_bwd(cam, ctx.P, sg, pg)
        return (pg["means"], pg["log_scales"], pg["quats"], pg["opacity_logits"], sg["rgb"], dfeat,
                None, None)


class Renderer:
    """Top-K renderer with a fixed K and feature storage / map precision.

    feat_dtype: "f32" (map f32), "bf16" (map bf16), or "fp8" (map bf16 by default).
    """

    def __init__(self, K=4, feat_dtype="f32", map_dtype=None, device="cuda"):
        if K not in lgs.lgs_supported_k():
            raise ValueError(f"K={K} not supported")
        self.K = K
        self.feat_dtype = feat_dtype
        self.map_dtype = map_dtype or ("f32" if feat_dtype == "f32" else "bf16")
        self.binner = Binner(device)
        self.store = None
        self.scale = None
        self._src = None

    def set_features(self, feat):
        if self.feat_dtype != "f32":
            self.store, self.scale = quantize(feat.detach(), self.feat_dtype)
            self._src = (feat.data_ptr(), feat._version, tuple(feat.shape))

    def _stale(self, feat):
        return self.store is None or self._src != (feat.data_ptr(), feat._version, tuple(feat.shape))

    def render(self, params, cam):
        c = cam if isinstance(cam, lgs.lgs_camera) else lgs.make_camera(cam)
        if self.feat_dtype != "f32" and self._stale(params["feat"]):
            self.set_features(params["feat"])
        return _TopKRender.apply(params["means"], params["log_scales"], params["quats"],
                                 params["opacity_logits"], params["rgb"], params["feat"], self, c)
