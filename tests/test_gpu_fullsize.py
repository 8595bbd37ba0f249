"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

* 1200x680 px, 500k Gaussians, D = 512, K = 1, 4 and 8 (the benchmark frame and its K
  sweep), BF16 and FP32 forms: the whole frame, forward and the whole adjoint, against
  the oracle.
* 8 views of 640x480, 1M Gaussians (pitched keyframes), and one 1200x680 view of 3M
  Gaussians at K = 8: projection, binning, blend + Top-K on every pixel, and the
  geometry adjoint, against the oracle.
* 8 views of 640x480, 1M Gaussians, D = 512, K = 4, BF16: the feature kernels over
  the stacked views in one launch, Top-K taken from the oracle's render of each
  view; sampled pixels and sampled gradient rows against the oracle.
* 4 views of 1200x680, 3M Gaussians, D = 768, K = 8, FP8 E4M3 rows with per-row
  scales: as above.

The oracle always renders its own Top-K; upstream gradients are seeded draws (the
large per-pixel maps are drawn on the device with a seeded generator and only the
sampled rows travel to the host).  On the multi-view workloads the one-pass render +
L1 adjoint is also checked against the two separate launches over all views."""
import time

import numpy as np
import pytest

from gpu_util import check_forward, gpu_forward, normwise
from paper_2602_06991_amd.scenegen import make_scene, random_upstream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_06991_amd import lgs
    lgs.load()
    return t


def log(msg):
    print(msg, flush=True)


def _stored(orc, feat, form):
    """The oracle's FP64 copy of the stored rows (its own quantizers)."""
    if form == "f32":
        return feat.astype(np.float64)
    if form == "bf16":
        return orc.bf16_to_f64(orc.bf16_bits(feat)).reshape(feat.shape)
    codes, s = orc.fp8_quantize(feat)
    return orc.fp8_dequant(codes, s)


@pytest.fixture(scope="module")
def frame_scene():
    t0 = time.time()
    sc = make_scene(2)
    log(f"scene {sc.cameras[0].W}x{sc.cameras[0].H} N={sc.gaussians.n} D={sc.gaussians.d} "
        f"in {time.time() - t0:.1f}s")
    return sc


@pytest.mark.timeout(400)
@pytest.mark.parametrize("form,K", [("bf16", 4), ("f32", 4), ("bf16", 1), ("bf16", 8), ("f32", 1),
                                    ("f32", 8)])
def test_benchmark_frame(torch, orc, frame_scene, form, K):
    """The benchmark frame at every K of its sweep, in the launch configuration the
    benchmark times (the one-pass feature kernel included)."""
    from paper_2602_06991_amd import render
    from test_gpu_render import _gpu_backward, _group_err
    g, cam = frame_scene.gaussians, frame_scene.cameras[0]
    mdt = "f32" if form == "f32" else "bf16"
    out, state = gpu_forward(g, cam, K)
    r = orc.render(g, cam, K)
    fl, bfl, ids_eq = check_forward(orc, g, cam, K, out, r, f"{cam.W}x{cam.H}")
    ok = ~fl

    # feature map from the GPU's own Top-K (the benchmark's launch), on unflagged pixels
    f64 = _stored(orc, g.feat, form)
    store, scale = render.quantize(state["P"]["feat"], form)
    F = render.feature_fwd(state["fw"]["ids"], state["fw"]["w"], store, scale, form, mdt)
    torch.cuda.synchronize()
    Fo = orc.feature(r["ids"], r["w"].astype(np.float32).astype(np.float64), f64)
    err = normwise(F.float().cpu().numpy().astype(np.float64)[ok], Fo[ok], 1e-2)
    tol = 1e-4 if mdt == "f32" else 1e-2
    log(f"feature map ({form}): max normwise err {err.max():.3g}, mean {err.mean():.3g}")
    assert err.max() <= tol

    # the benchmark's one-pass render + L1 adjoint: the target is kept clear of the
    # oracle's map on unflagged pixels and equals the GPU's own map on flagged ones
    # (sign 0 there, matching the oracle's masked upstream gradient)
    rng = np.random.default_rng(5)
    P, D = cam.W * cam.H, g.d
    delta = rng.choice([-1.0, 1.0], (P, D)) * (0.02 + 0.05 * np.abs(Fo.reshape(P, D)))
    That = (Fo.reshape(P, D) + delta).astype(np.float32)
    del delta
    tmap = torch.float32 if mdt == "f32" else torch.bfloat16
    T_dev = torch.from_numpy(That).cuda().to(tmap)
    del That
    flat_ok = torch.from_numpy(ok.reshape(-1)).cuda()
    T_dev = torch.where(flat_ok[:, None], T_dev, F.reshape(P, D)).reshape(cam.H, cam.W, D).contiguous()
    T_m = T_dev.reshape(P, D).float().cpu().numpy().astype(np.float64)
    fs = 1.0 / (P * D)
    d1 = torch.zeros(g.n, D, device="cuda")
    F1, t1 = render.feature_fwd_bwd_l1(state["fw"]["ids"], state["fw"]["w"], store, scale, form, mdt, T_dev,
                                       fs, d1)
    torch.cuda.synchronize()
    assert torch.equal(F1, F)                      # the stored map is the forward's, bit for bit
    gs = fs if mdt == "f32" else float(torch.tensor(fs).to(torch.bfloat16).float())
    gF1 = gs * np.sign(Fo.reshape(P, D) - T_m) * ok.reshape(-1, 1)
    del T_m
    d_feat, d_w = orc.feature_backward(r["ids"], r["w"].astype(np.float32).astype(np.float64), f64,
                                       gF1.reshape(cam.H, cam.W, D))
    del gF1
    df = d1.cpu().numpy()
    touched = np.abs(d_feat).sum(1) > 0
    e = normwise(df[touched], d_feat[touched], 1e-12)
    gam = t1.cpu().numpy()[ok]
    dw = d_w[ok]
    eg = (np.abs(gam - dw) / (np.abs(dw).max(-1, keepdims=True) + 1e-12)).max()
    log(f"one-pass render + L1 adjoint ({form}): gradient rows max normwise err {e.max():.3g}, "
        f"dL/dw max err {eg:.3g}")
    assert e.max() <= 1e-4 and eg <= 1e-4
    assert np.all(df[~touched] == 0)
    del F, Fo, F1, d1, df, d_feat, d_w, T_dev

    # the whole adjoint, upstream gradients zeroed on flagged pixels on both sides
    gC, gD, gO, gF = random_upstream(11, cam.W * cam.H, g.d)
    m = ok.reshape(-1).astype(np.float32)
    gC *= m[:, None]; gD *= m; gO *= m; gF *= m[:, None]
    if mdt == "bf16":
        gF = torch.from_numpy(gF).to(torch.bfloat16).float().numpy()
    H, W = cam.H, cam.W
    gpu = _gpu_backward(torch, state, K, gC.reshape(H, W, 3), gD.reshape(H, W), gO.reshape(H, W),
                        gF.reshape(H, W, g.d), fdt=form, mdt=mdt)
    b = orc.backward(g, cam, K, f64, gC, gD, gO, gF.astype(np.float64))
    tol = 1e-3 if form == "f32" else 1e-2
    pairs = [("s_mean2d", "d_mean2d"), ("s_conic", "d_conic"), ("s_opacity", "d_opac"),
             ("s_rgb", "d_rgb"), ("s_depth", "d_z"), ("p_means", "d_means"),
             ("p_log_scales", "d_log_scales"), ("p_quats", "d_quats"),
             ("p_opacity_logits", "d_opacity_logits"), ("dfeat", "d_feat")]
    msg = []
    for a, o in pairs:
        fro, worst = _group_err(gpu[a], b[o])
        msg.append(f"{a} {fro:.1e}/{worst:.1e}")
        assert fro <= tol and worst <= tol, (a, fro, worst)
    log("adjoint (fro/worst): " + ", ".join(msg))


def _oracle_topk(orc, g, cams, K):
    ids, w = [], []
    for c in cams:
        r = orc.render(g, c, K)
        ids.append(r["ids"])
        w.append(r["w"].astype(np.float32))
    return np.concatenate(ids, 0), np.concatenate(w, 0)


def _sampled_feature_parity(torch, orc, g, ids, w, views, form, seed, n_rows):
    """Feature fwd and adjoint over all views in one launch; sampled pixels and
    sampled gradient rows against the oracle on the union of the selected rows."""
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(seed)
    Hs, W, K = ids.shape
    D = g.d
    P = Hs * W
    feat_dev = torch.from_numpy(g.feat).cuda()
    store, scale = render.quantize(feat_dev, form)
    del feat_dev
    ids_dev = torch.from_numpy(ids).cuda()
    w_dev = torch.from_numpy(w).cuda()
    F = render.feature_fwd(ids_dev, w_dev, store, scale, form, "bf16", views=views)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    gF = torch.empty(Hs, W, D, device="cuda", dtype=torch.bfloat16)
    for y0 in range(0, Hs, 256):
        y1 = min(Hs, y0 + 256)
        gF[y0:y1] = torch.randn(y1 - y0, W, D, device="cuda", generator=gen).to(torch.bfloat16)
    dfeat = torch.zeros(g.n, D, device="cuda")
    dtw = render.feature_bwd(ids_dev, w_dev, store, scale, form, "bf16", gF, dfeat, views=views)
    torch.cuda.synchronize()
    log(f"GPU feature fwd + adjoint over {views} views done")

    flat_ids = ids.reshape(P, K)
    union = np.unique(flat_ids[flat_ids >= 0])
    f64u = _stored(orc, g.feat[union], form)          # row quantizers act row by row
    remap = np.where(flat_ids >= 0, np.searchsorted(union, np.maximum(flat_ids, 0)), -1).astype(np.int32)
    log(f"union of the Top-K rows: {union.size}")

    # forward on sampled pixels
    px = rng.choice(P, size=min(P, 60000), replace=False)
    Fo = orc.feature(remap[px], w.reshape(P, K)[px].astype(np.float64), f64u)
    Fg = F.reshape(P, D)[torch.from_numpy(px).cuda()].float().cpu().numpy().astype(np.float64)
    err = normwise(Fg, Fo, 1e-2)
    log(f"feature map ({form}): sampled max normwise err {err.max():.3g}, mean {err.mean():.3g}")
    assert err.max() <= 1e-2   # against the stored rows: the BF16 map rounding

    # adjoint: sampled rows, with every pixel that selected them
    rows = rng.choice(union.size, size=min(union.size, n_rows), replace=False)
    want = np.zeros(union.size, bool)
    want[rows] = True
    pix = np.nonzero(np.any((remap >= 0) & want[np.maximum(remap, 0)], -1))[0]
    pix_dev = torch.from_numpy(pix).cuda()
    gF_s = gF.reshape(P, D)[pix_dev].float().cpu().numpy().astype(np.float64)
    d_feat, d_w = orc.feature_backward(remap[pix], w.reshape(P, K)[pix].astype(np.float64), f64u, gF_s)
    gpu_rows = dfeat[torch.from_numpy(union[rows]).cuda()].cpu().numpy()
    e = normwise(gpu_rows, d_feat[rows], 1e-6)
    log(f"gradient rows: {rows.size} sampled over {pix.size} pixels, max normwise err {e.max():.3g}")
    assert e.max() <= 1e-4
    gam = dtw.reshape(P, K)[pix_dev].cpu().numpy()
    scl = np.abs(d_w).max(-1, keepdims=True) + 1e-6
    eg = (np.abs(gam - d_w) / scl).max()
    log(f"dL/dw on those pixels: max err (rel to pixel max) {eg:.3g}")
    assert eg <= 1e-4
    # rows outside the union receive nothing
    outside = rng.integers(0, g.n, 4000)
    outside = outside[~np.isin(outside, union)]
    assert float(dfeat[torch.from_numpy(outside).cuda()].abs().max()) == 0.0
    del dfeat, dtw

    # the one-pass render + L1 adjoint over the same views (the drawn map as the
    # target): its map and dL/dw equal the two separate launches' bit for bit
    fs = 1.0 / (P * D)
    d1 = torch.zeros(g.n, D, device="cuda")
    t1 = render.feature_bwd_l1(ids_dev, w_dev, store, scale, form, "bf16", gF, fs, d1, views=views)
    d2 = torch.zeros(g.n, D, device="cuda")
    F2, t2 = render.feature_fwd_bwd_l1(ids_dev, w_dev, store, scale, form, "bf16", gF, fs, d2, views=views)
    torch.cuda.synchronize()
    assert torch.equal(F2, F)
    assert torch.equal(t2, t1)
    rows_t = torch.from_numpy(union).cuda()
    a, b = d1[rows_t], d2[rows_t]
    rel = ((a - b).norm(dim=1) / b.norm(dim=1).clamp_min(1e-30)).max().item()
    log(f"one-pass render + L1 adjoint over {views} views: map and dL/dw identical, dL/df rows rel {rel:.2e}")
    assert rel <= 1e-6


@pytest.fixture(scope="module")
def scene3():
    t0 = time.time()
    sc = make_scene(3)
    log(f"scene {len(sc.cameras)} views {sc.cameras[0].W}x{sc.cameras[0].H} N={sc.gaussians.n} "
        f"D={sc.gaussians.d} in {time.time() - t0:.1f}s")
    return sc


@pytest.fixture(scope="module")
def scene4():
    t0 = time.time()
    sc = make_scene(4)
    log(f"scene {len(sc.cameras)} views {sc.cameras[0].W}x{sc.cameras[0].H} N={sc.gaussians.n} "
        f"D={sc.gaussians.d} in {time.time() - t0:.1f}s")
    return sc


def _geometry_adjoint(torch, orc, g, cam, K, state, ok, seed, feat_form, with_feature):
    """The whole adjoint of one view against the oracle's, upstream gradients zeroed on
    flagged pixels on both sides; the feature term (through the Top-K weights) only when
    with_feature (the oracle then needs the dense FP64 feature table)."""
    from test_gpu_render import _gpu_backward, _group_err
    H, W = cam.H, cam.W
    gC, gD, gO, gF = random_upstream(seed, W * H, g.d if with_feature else 8)
    m = ok.reshape(-1).astype(np.float32)
    gC *= m[:, None]; gD *= m; gO *= m; gF *= m[:, None]
    if with_feature:
        gF = torch.from_numpy(gF).to(torch.bfloat16).float().numpy()
        f64 = _stored(orc, g.feat, feat_form)
    else:
        gF = np.zeros((W * H, g.d), np.float32)
        f64 = np.zeros((g.n, 8))
    gpu = _gpu_backward(torch, state, K, gC.reshape(H, W, 3), gD.reshape(H, W), gO.reshape(H, W),
                        gF.reshape(H, W, g.d), fdt=feat_form, mdt="bf16")
    b = orc.backward(g, cam, K, f64, gC, gD, gO, gF.astype(np.float64) if with_feature else None)
    pairs = [("s_mean2d", "d_mean2d"), ("s_conic", "d_conic"), ("s_opacity", "d_opac"),
             ("s_rgb", "d_rgb"), ("s_depth", "d_z"), ("p_means", "d_means"),
             ("p_log_scales", "d_log_scales"), ("p_quats", "d_quats"),
             ("p_opacity_logits", "d_opacity_logits")] + ([("dfeat", "d_feat")] if with_feature else [])
    # FP32 geometry gradients: 1e-3; with the BF16 feature term: 1e-2
    tol = 1e-2 if with_feature else 1e-3
    msg = []
    for a, o in pairs:
        fro, worst = _group_err(gpu[a], b[o])
        msg.append(f"{a} {fro:.1e}/{worst:.1e}")
        assert fro <= tol and worst <= tol, (a, fro, worst)
    log("adjoint (fro/worst): " + ", ".join(msg))


@pytest.mark.timeout(600)
def test_geometry_path_eight_pitched_views(torch, orc, scene3):
    """Projection, binning, blend + Top-K of all 8 keyframes of the 640x480 / 1M
    workload (random positions, yaw and +-15 degree pitch), every pixel against the
    oracle; the whole adjoint (BF16 features, feature term included) of two of them."""
    g, K = scene3.gaussians, 4
    for v, cam in enumerate(scene3.cameras):
        out, state = gpu_forward(g, cam, K)
        r = orc.render(g, cam, K)
        fl, _, _ = check_forward(orc, g, cam, K, out, r, f"view {v}")
        if v in (0, 5):
            _geometry_adjoint(torch, orc, g, cam, K, state, ~fl, 20 + v, "bf16", True)
        del out, state, r


@pytest.mark.timeout(600)
def test_geometry_path_large_view(torch, orc, scene4):
    """One 1200x680 view of the 3M-Gaussian workload (K = 8): every pixel of the blend
    and Top-K against the oracle, and the geometry adjoint of colour, depth and opacity."""
    g, K = scene4.gaussians, 8
    cam = scene4.cameras[1]
    out, state = gpu_forward(g, cam, K)
    r = orc.render(g, cam, K)
    fl, _, _ = check_forward(orc, g, cam, K, out, r, "3M view 1")
    _geometry_adjoint(torch, orc, g, cam, K, state, ~fl, 31, "fp8", False)


@pytest.mark.timeout(500)
def test_eight_views_bf16(torch, orc, scene3):
    t0 = time.time()
    sc = scene3
    g, K = sc.gaussians, 4
    ids, w = _oracle_topk(orc, g, sc.cameras, K)
    log(f"oracle Top-K of {len(sc.cameras)} views in {time.time() - t0:.1f}s")
    _sampled_feature_parity(torch, orc, g, ids, w, len(sc.cameras), "bf16", 3, 3000)


@pytest.mark.timeout(600)
def test_four_views_fp8_d768_k8(torch, orc, scene4):
    t0 = time.time()
    sc = scene4
    g, K = sc.gaussians, 8
    ids, w = _oracle_topk(orc, g, sc.cameras, K)
    log(f"oracle Top-K of {len(sc.cameras)} views in {time.time() - t0:.1f}s")
    _sampled_feature_parity(torch, orc, g, ids, w, len(sc.cameras), "fp8", 4, 800)
