"""Kernel-level parity of the HIP path against the oracle (and, for the sort, against
numpy's lexsort on synthetic keys).  Each kernel is fed inputs the oracle or the
seeded generator produced, never another HIP kernel's output."""
import numpy as np
import pytest

from gpu_util import FLAG_EPS, dev_params, gpu_forward, normwise, rel_close
from paper_2602_06991_amd.scenegen import make_scene, make_tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_06991_amd import lgs
    lgs.load()
    return t


@pytest.mark.parametrize("d", [8, 200, 512, 768, 2056, 2568])
def test_quantize_bit_exact(torch, orc, d):
    """Storage quantizers bit for bit, at row lengths below one 512-channel step, ragged,
    and beyond the 2048 channels the FP8 quantizer holds in registers (rows read twice)."""
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(d)
    n = 3000 if d <= 768 else 600
    x = (rng.standard_normal((n, d)) * np.exp(rng.uniform(-20, 20, (n, 1)))).astype(np.float32)
    x[0] = 0
    x[1, :] = 1e-40          # subnormal row
    x[2, min(5, d - 1)] = 448.0 * 3      # row whose amax sets a larger scale
    x[3, d - 1] = -448.0 * 5             # ... in the last channel
    t = torch.from_numpy(x).cuda()
    b, _ = render.quantize(t, "bf16")
    q, s = render.quantize(t, "fp8")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b.view(torch.int16).cpu().numpy().view(np.uint16), orc.bf16_bits(x))
    codes, scale = orc.fp8_quantize(x)
    np.testing.assert_array_equal(s.cpu().numpy(), scale)
    np.testing.assert_array_equal(q.cpu().numpy(), codes)
    # the refresh of marked rows: the same bits in the rows stamped with gen, the other
    # rows of the store untouched
    from paper_2602_06991_amd import lgs
    gen = 7
    stamp = np.where(rng.random(n) < 0.3, gen, rng.choice([gen - 1, gen + 1, -2**31], n)).astype(np.int32)
    stamp[:4] = gen
    marked = stamp == gen
    row_gen = torch.from_numpy(stamp).cuda()
    b2 = torch.full((n, d), 0x7F7F, dtype=torch.int16, device="cuda").view(torch.bfloat16)
    q2 = torch.full((n, d), 0x55, dtype=torch.uint8, device="cuda")
    s2 = torch.full((n,), -1.0, device="cuda")
    p = lambda a: a.data_ptr()
    lgs.lgs_quantize_marked_rows(n, d, gen, p(row_gen), p(t), lgs.LGS_BF16, p(b2), None)
    lgs.lgs_quantize_marked_rows(n, d, gen, p(row_gen), p(t), lgs.LGS_FP8_E4M3, p(q2), p(s2))
    torch.cuda.synchronize()
    b2 = b2.view(torch.int16).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(b2[marked], orc.bf16_bits(x)[marked])
    assert (b2[~marked] == 0x7F7F).all()
    q2, s2 = q2.cpu().numpy(), s2.cpu().numpy()
    np.testing.assert_array_equal(q2[marked], codes[marked])
    np.testing.assert_array_equal(s2[marked], scale[marked])
    assert (q2[~marked] == 0x55).all() and (s2[~marked] == -1.0).all()


@pytest.mark.parametrize("cfg", ["tiny", "c0", "c1"])
def test_project_parity(torch, orc, cfg):
    from paper_2602_06991_amd import lgs, render
    if cfg == "tiny":
        g, cam = make_tiny(3, n=200, W=48, H=40, spread=(-0.8, 1.8), scale=(-2.0, 1.0))
    else:
        sc = make_scene(int(cfg[1]))
        g, cam = sc.gaussians, sc.cameras[0]
    # a few degenerate Gaussians the culls must agree on
    g.means[0] = np.nan
    g.quats[1] = 0
    g.log_scales[2, 0] = 10.5
    g.opacity_logits[3] = -5.6
    P = dev_params(g)
    proj = render.project(lgs.make_camera(cam), P)
    torch.cuda.synchronize()
    o = orc.project(g, cam)
    valid = o["valid"].astype(bool)
    gv = proj["tiles_touched"].cpu().numpy() > 0
    # a GPU-visible Gaussian must be oracle-valid; oracle-valid ones off-screen may have 0 tiles
    assert not np.any(gv & ~valid)
    assert not valid[:4].any()
    zk = proj["depth"].cpu().numpy()
    np.testing.assert_array_equal(zk[valid], o["zkey"][valid])   # bit-exact depth key
    m2 = proj["mean2d"].cpu().numpy()
    # fx tx/tz + cx in FP32: a few ulp of the larger of the two terms
    scale_px = np.abs(o["mean2d"][valid]) + max(cam.cx, cam.cy) + max(cam.fx, cam.fy)
    assert np.all(np.abs(m2[valid] - o["mean2d"][valid]) <= 1e-6 * scale_px)
    con = proj["conic"].cpu().numpy()
    # an FP32 2x2 inverse loses about cond(Sigma2D) ulps
    A, B, C = o["cov2d"][valid].T
    disc = np.sqrt(((A - C) / 2) ** 2 + B * B)
    cond = ((A + C) / 2 + disc) / ((A + C) / 2 - disc)
    tol = np.maximum(1e-5, 1e-6 * cond) * np.abs(o["conic"][valid]).max(1)
    assert np.all(np.abs(con[valid] - o["conic"][valid]) <= tol[:, None])
    op = proj["opacity"].cpu().numpy()
    assert np.all(rel_close(op[valid], o["opacity"][valid], 1e-6, 1e-3))
    # every pixel of the oracle's support box lies in the GPU's tile box
    rect = proj["tile_rect"].cpu().numpy()
    orect = o["rect"]
    has = valid & (orect[:, 2] >= orect[:, 0]) & (orect[:, 3] >= orect[:, 1])
    assert np.all(gv[has])
    assert np.all(rect[has, 0] * 16 <= orect[has, 0]) and np.all(rect[has, 1] * 16 <= orect[has, 1])
    assert np.all(rect[has, 2] * 16 > orect[has, 2]) and np.all(rect[has, 3] * 16 > orect[has, 3])


def _synthetic_bins(n, W, H, seed, big):
    rng = np.random.default_rng(seed)
    ntx, nty = (W + 15) // 16, (H + 15) // 16
    tx0 = rng.integers(0, ntx, n)
    ty0 = rng.integers(0, nty, n)
    wide = rng.random(n) < big                             # a few Gaussians cover many tiles
    tx1 = np.minimum(tx0 + np.where(wide, rng.integers(1, 40, n), rng.integers(1, 4, n)), ntx)
    ty1 = np.minimum(ty0 + np.where(wide, rng.integers(1, 30, n), rng.integers(1, 4, n)), nty)
    touched = ((tx1 - tx0) * (ty1 - ty0)).astype(np.int32)
    touched[rng.random(n) < 0.2] = 0                       # culled
    depth = rng.choice(rng.uniform(0.3, 9.0, max(n // 3, 1)).astype(np.float32), n)  # many ties
    rect = np.stack([tx0, ty0, tx1, ty1], 1).astype(np.int32)
    return ntx, nty, tx0, ty0, tx1, ty1, touched, depth, rect


def _expected_pairs(n, ntx, tx0, ty0, tx1, touched):
    """Every (tile, Gaussian) pair of the synthetic rects, tiles of a rect row by row."""
    c = np.where(touched > 0, touched, 0).astype(np.int64)
    g = np.repeat(np.arange(n, dtype=np.int64), c)
    k = np.arange(len(g), dtype=np.int64) - np.repeat(np.cumsum(c) - c, c)
    w = (tx1 - tx0).astype(np.int64)[g]
    return (ty0.astype(np.int64)[g] + k // w) * ntx + tx0.astype(np.int64)[g] + k % w, g


@pytest.mark.parametrize("n,W,H,seed,big", [(1, 16, 16, 0, 0.0), (1000, 64, 48, 1, 0.0),
                                            (20000, 640, 480, 2, 0.0), (100000, 1200, 680, 3, 0.0),
                                            (50000, 1200, 680, 4, 0.01),
                                            # passes of 4 M items and more take blocks of 4096:
                                            # the tile sort only, then the depth sort too
                                            (1500000, 1200, 680, 5, 0.0), (4500000, 1200, 680, 6, 0.0)])
def test_bin_sort_matches_lexsort(torch, n, W, H, seed, big):
    """Synthetic rects and depth keys (with deliberate ties): the pairs must come out
    ordered by (tile, depth key, id), exactly as numpy's lexsort orders them; from 1.5 M
    Gaussians on, the asynchronous mode (grids sized for the buffer) must bin the same."""
    from paper_2602_06991_amd import lgs, render
    ntx, nty, tx0, ty0, tx1, ty1, touched, depth, rect = _synthetic_bins(n, W, H, seed, big)
    cam = lgs.lgs_camera()
    cam.width, cam.height, cam.fx, cam.fy = W, H, 1.0, 1.0
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b = render.Binner()
    b._ensure(n, W, H, 64)                                  # force the capacity retry path
    args = (cam, n, tt(depth), tt(rect), tt(touched))
    ids, ranges, m = b(*args)
    torch.cuda.synchronize()
    exp_t, exp_g = _expected_pairs(n, ntx, tx0, ty0, tx1, touched)
    order = np.lexsort((exp_g, depth[exp_g], exp_t))
    assert m == len(exp_t)
    np.testing.assert_array_equal(ids.cpu().numpy(), exp_g[order])
    r = ranges.cpu().numpy()
    cnt = np.bincount(exp_t, minlength=ntx * nty)
    np.testing.assert_array_equal(r[:, 1] - r[:, 0], cnt)
    starts = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    np.testing.assert_array_equal(r[cnt > 0, 0], starts[cnt > 0])
    if n >= 1500000:
        a = render.Binner(sync=False)
        a(*args)                                             # sizes the buffers
        ids_a, r_a, _ = a(*args)
        assert a.count() == (m, True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ids_a[:m].cpu().numpy(), exp_g[order])
        np.testing.assert_array_equal(r_a.cpu().numpy(), r)


def test_bin_sort_without_host_round_trip(torch):
    """The asynchronous mode (count left on the device) bins exactly as the synchronous
    one; a buffer that is too small is reported by the count query, and the call stays
    inside its buffers."""
    from paper_2602_06991_amd import lgs, render
    n, W, H = 60000, 1200, 680
    ntx, nty, tx0, ty0, tx1, ty1, touched, depth, rect = _synthetic_bins(n, W, H, 9, 0.005)
    cam = lgs.lgs_camera()
    cam.width, cam.height, cam.fx, cam.fy = W, H, 1.0, 1.0
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = (cam, n, tt(depth), tt(rect), tt(touched))
    ids0, r0, m = render.Binner()(*args)
    b = render.Binner(sync=False)
    _, _, m1 = b(*args)                                      # the first call sizes the buffers
    ids, r, none = b(*args)
    assert m1 == m and none is None
    assert b.count() == (m, True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.cpu().numpy(), r0.cpu().numpy())
    np.testing.assert_array_equal(ids[:m].cpu().numpy(), ids0.cpu().numpy())
    # too small: the count says so and the next call (after count() grew the buffers) fits
    b._ensure(n, W, H, m // 2)
    guard = torch.full((b.cap + 4096,), -7, dtype=torch.int32, device="cuda")
    b.ids = guard
    b(*args)
    assert b.count() == (m, False)
    assert int(guard[m // 2:].ne(-7).sum()) == 0            # nothing past max_pairs
    ids, r, _ = b(*args)
    assert b.count() == (m, True)
    np.testing.assert_array_equal(r.cpu().numpy(), r0.cpu().numpy())


def test_asynchronous_binner_growth_returns_the_written_pairs(torch):
    """Regression: a first call whose pair count passes two thirds of the buffer grows
    the buffers for the next calls; the pairs it returns must be the ones it wrote,
    not a slice of the new buffer."""
    from paper_2602_06991_amd import lgs, render
    n, W, H = 60000, 1200, 680
    ntx, nty, tx0, ty0, tx1, ty1, touched, depth, rect = _synthetic_bins(n, W, H, 12, 0.005)
    cam = lgs.lgs_camera()
    cam.width, cam.height, cam.fx, cam.fy = W, H, 1.0, 1.0
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = (cam, n, tt(depth), tt(rect), tt(touched))
    ids0, r0, m = render.Binner()(*args)
    b = render.Binner(sync=False)
    b._ensure(n, W, H, m + 16)                             # the first call fills it past 2/3
    ids1, r1, m1 = b(*args)
    torch.cuda.synchronize()
    assert m1 == m and b.cap >= int(m * 1.5)
    np.testing.assert_array_equal(ids1.cpu().numpy(), ids0.cpu().numpy())
    np.testing.assert_array_equal(r1.cpu().numpy(), r0.cpu().numpy())
    ids2, r2, none = b(*args)                              # the next call: asynchronous, grown buffers
    assert none is None and b.count() == (m, True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids2[:m].cpu().numpy(), ids0.cpu().numpy())


def _oracle_topk(orc, g, cam, K):
    r = orc.render(g, cam, K)
    return r


@pytest.mark.parametrize("K,fdt,mdt", [(4, "f32", "f32"), (1, "f32", "f32"), (8, "f32", "f32"),
                                       (4, "bf16", "bf16"), (4, "bf16", "f32"), (8, "fp8", "bf16"),
                                       (3, "fp8", "f32"), (16, "bf16", "bf16")])
def test_feature_fwd_parity(torch, orc, K, fdt, mdt):
    from paper_2602_06991_amd import render
    sc = make_scene(0)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, K)
    ids = torch.from_numpy(r["ids"]).cuda()
    w = torch.from_numpy(r["w"].astype(np.float32)).cuda()
    feat = torch.from_numpy(g.feat).cuda()
    store, scale = render.quantize(feat, fdt)
    F = render.feature_fwd(ids, w, store, scale, fdt, mdt)
    torch.cuda.synchronize()
    Fg = F.float().cpu().numpy().astype(np.float64)
    if fdt == "f32":
        f64 = g.feat.astype(np.float64)
    elif fdt == "bf16":
        f64 = orc.bf16_to_f64(orc.bf16_bits(g.feat)).reshape(g.feat.shape)
    else:
        codes, s = orc.fp8_quantize(g.feat)
        f64 = orc.fp8_dequant(codes, s)
    # the oracle takes the same FP32-rounded weights the kernel got
    Fo = orc.feature(r["ids"], r["w"].astype(np.float32).astype(np.float64), f64)
    err = normwise(Fg, Fo, 1e-2)
    tol = 1e-4 if mdt == "f32" else 1e-2
    print(f"K={K} {fdt}->{mdt}: max normwise err vs stored features {err.max():.3g}")
    assert err.max() <= tol
    if fdt != "f32":
        # end to end against the unquantized features
        Fu = orc.feature(r["ids"], r["w"], g.feat.astype(np.float64))
        e2 = normwise(Fg, Fu, 1e-2)
        print(f"   vs unquantized FP64: max {e2.max():.3g} mean {e2.mean():.3g}")
        assert e2.max() <= (1e-2 if fdt == "bf16" else 3e-2)
    W = r["w"].sum(-1)
    assert np.all(Fg[W == 0] == 0)


@pytest.mark.parametrize("K,fdt,mdt", [(4, "f32", "f32"), (1, "f32", "f32"), (8, "bf16", "bf16"),
                                       (4, "fp8", "bf16"), (16, "f32", "f32")])
def test_feature_bwd_parity(torch, orc, K, fdt, mdt):
    from paper_2602_06991_amd import render
    sc = make_scene(1, N=60000, W=200, H=150)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, K)
    rng = np.random.default_rng(K)
    gF = rng.standard_normal((cam.H, cam.W, g.d)).astype(np.float32)
    tmap = torch.float32 if mdt == "f32" else torch.bfloat16
    gF_dev = torch.from_numpy(gF).cuda().to(tmap)
    gF64 = gF_dev.float().cpu().numpy().astype(np.float64)
    ids = torch.from_numpy(r["ids"]).cuda()
    w = torch.from_numpy(r["w"].astype(np.float32)).cuda()
    feat = torch.from_numpy(g.feat).cuda()
    store, scale = render.quantize(feat, fdt)
    dfeat = torch.zeros(g.n, g.d, device="cuda")
    dtw = render.feature_bwd(ids, w, store, scale, fdt, mdt, gF_dev, dfeat)
    torch.cuda.synchronize()
    if fdt == "f32":
        f64 = g.feat.astype(np.float64)
    elif fdt == "bf16":
        f64 = orc.bf16_to_f64(orc.bf16_bits(g.feat)).reshape(g.feat.shape)
    else:
        codes, s = orc.fp8_quantize(g.feat)
        f64 = orc.fp8_dequant(codes, s)
    # the oracle's feature adjoint for the same Top-K: isolate it with gC = gD = gO = 0
    from types import SimpleNamespace
    gg = SimpleNamespace(means=g.means, log_scales=g.log_scales, quats=g.quats,
                         opacity_logits=g.opacity_logits, rgb=g.rgb, feat=g.feat)
    b = orc.backward(gg, cam, K, f64, None, None, None, gF64)
    df = dfeat.cpu().numpy()
    touched = np.abs(b["d_feat"]).sum(1) > 0
    err = normwise(df[touched], b["d_feat"][touched], 1e-6)
    print(f"K={K} {fdt}/{mdt}: dL/df rows {touched.sum()}, max normwise err {err.max():.3g}")
    assert err.max() <= 1e-4
    assert np.all(df[~touched] == 0)
    # gamma: compare with the scale of the pixel's dot products
    gam = dtw.cpu().numpy()
    scl = np.abs(b["d_topkw"]).max(-1, keepdims=True) + 1e-6
    e = np.abs(gam - b["d_topkw"]) / scl
    print(f"   gamma max err (rel to pixel max) {e.max():.3g}")
    assert e.max() <= 1e-4


def _synthetic_topk(rng, views, H, W, K, n, spread):
    """Per-pixel Top-K lists drawn at random: `spread` distinct ids per 16x16 tile on
    average (spread >= 256 K overflows any LDS row cache), with empty and short pixels."""
    ids = np.full((views * H, W, K), -1, np.int32)
    w = np.zeros((views * H, W, K), np.float32)
    pool = rng.choice(n, size=max(spread, K), replace=False)
    for v in range(views):
        for y in range(H):
            for x in range(W):
                r = rng.random()
                k = 0 if r < 0.05 else (rng.integers(1, K + 1) if r < 0.2 else K)
                if k == 0:
                    continue
                ids[v * H + y, x, :k] = rng.choice(pool, k, replace=False)
                ww = np.sort(rng.uniform(1e-3, 0.6, k))[::-1]
                w[v * H + y, x, :k] = ww
    return ids, w


@pytest.mark.parametrize("K,fdt,mdt,views,H,W,D,spread", [
    (4, "f32", "f32", 1, 37, 53, 64, 40),          # ragged tiles
    (4, "bf16", "bf16", 2, 40, 48, 512, 30000),    # union overflows the LDS cache
    (8, "fp8", "bf16", 1, 33, 70, 768, 500),
    (1, "bf16", "f32", 3, 20, 20, 520, 20),
    (16, "f32", "f32", 1, 32, 32, 128, 9000),
    # unions of 17..32 (two 16-row MFMA blocks), channel tails, idle waves
    (4, "bf16", "bf16", 1, 16, 16, 512, 28),
    (4, "bf16", "bf16", 2, 50, 70, 200, 24),
    (8, "fp8", "bf16", 1, 40, 40, 512, 30),
    (4, "fp8", "bf16", 1, 33, 35, 96, 12),
    (2, "bf16", "bf16", 1, 30, 30, 8, 10),
    (5, "bf16", "bf16", 1, 64, 64, 512, 60),
    # FP32 rows on the matrix cores (the forward), channel slabs of 256
    (4, "f32", "f32", 1, 40, 53, 512, 24),
    (8, "f32", "f32", 2, 33, 40, 768, 30),
    (3, "fp8", "f32", 1, 36, 36, 520, 20),
    # unions of 33..64 at K > 4 (four union blocks)
    (8, "bf16", "bf16", 1, 40, 53, 512, 48),
    (8, "f32", "f32", 2, 33, 35, 520, 60)])
def test_feature_kernels_on_synthetic_topk(torch, orc, K, fdt, mdt, views, H, W, D, spread):
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(K * 100 + D)
    n = 40000
    feat = rng.standard_normal((n, D)).astype(np.float32)
    ids, w = _synthetic_topk(rng, views, H, W, K, n, spread)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    store, scale = render.quantize(dev(feat), fdt)
    F = render.feature_fwd(dev(ids), dev(w), store, scale, fdt, mdt, views=views)
    gF = rng.standard_normal((views * H, W, D)).astype(np.float32)
    tmap = torch.float32 if mdt == "f32" else torch.bfloat16
    gF_dev = dev(gF).to(tmap)
    dfeat = torch.zeros(n, D, device="cuda")
    dtw = render.feature_bwd(dev(ids), dev(w), store, scale, fdt, mdt, gF_dev, dfeat, views=views)
    torch.cuda.synchronize()
    if fdt == "f32":
        f64 = feat.astype(np.float64)
    elif fdt == "bf16":
        f64 = orc.bf16_to_f64(orc.bf16_bits(feat)).reshape(feat.shape)
    else:
        c, s = orc.fp8_quantize(feat)
        f64 = orc.fp8_dequant(c, s)
    Fo = orc.feature(ids, w.astype(np.float64), f64)
    err = normwise(F.float().cpu().numpy().astype(np.float64), Fo, 1e-2)
    assert err.max() <= (1e-4 if mdt == "f32" else 1e-2), err.max()
    d_feat, d_w = orc.feature_backward(ids, w.astype(np.float64), f64,
                                       gF_dev.float().cpu().numpy().astype(np.float64))
    df = dfeat.cpu().numpy()
    touched = np.abs(d_feat).sum(1) > 0
    e = normwise(df[touched], d_feat[touched], 1e-6)
    assert e.max() <= 1e-4, e.max()
    assert np.all(df[~touched] == 0)
    scl = np.abs(d_w).max(-1, keepdims=True) + 1e-6
    assert (np.abs(dtw.cpu().numpy() - d_w) / scl).max() <= 1e-4


@pytest.mark.parametrize("K,fdt,mdt", [(4, "f32", "f32"), (4, "bf16", "bf16"), (8, "fp8", "bf16")])
def test_feature_bwd_fused_l1(torch, orc, K, fdt, mdt):
    """dL/dF = s sign(F - F^) formed inside the adjoint.  The target keeps every element
    well clear of F, so the sign is the same whichever side rounds."""
    from paper_2602_06991_amd import render
    sc = make_scene(1, N=60000, W=200, H=150)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, K)
    rng = np.random.default_rng(11)
    if fdt == "f32":
        f64 = g.feat.astype(np.float64)
    elif fdt == "bf16":
        f64 = orc.bf16_to_f64(orc.bf16_bits(g.feat)).reshape(g.feat.shape)
    else:
        c, s = orc.fp8_quantize(g.feat)
        f64 = orc.fp8_dequant(c, s)
    w32 = r["w"].astype(np.float32)
    Fo = orc.feature(r["ids"], w32.astype(np.float64), f64)
    delta = rng.choice([-1.0, 1.0], Fo.shape) * (0.02 + 0.05 * np.abs(Fo))
    That = (Fo + delta).astype(np.float32)
    tmap = torch.float32 if mdt == "f32" else torch.bfloat16
    That_dev = torch.from_numpy(That).cuda().to(tmap)
    That_m = That_dev.float().cpu().numpy().astype(np.float64)
    scale = 1.0 / Fo.size
    ids = torch.from_numpy(r["ids"]).cuda()
    w = torch.from_numpy(w32).cuda()
    store, sc8 = render.quantize(torch.from_numpy(g.feat).cuda(), fdt)
    dfeat = torch.zeros(g.n, g.d, device="cuda")
    dtw = render.feature_bwd_l1(ids, w, store, sc8, fdt, mdt, That_dev, scale, dfeat)
    torch.cuda.synchronize()
    gs = scale if mdt == "f32" else float(torch.tensor(scale).to(torch.bfloat16).float())
    gF = gs * np.sign(Fo - That_m)
    d_feat, d_w = orc.feature_backward(r["ids"], w32.astype(np.float64), f64, gF)
    df = dfeat.cpu().numpy()
    touched = np.abs(d_feat).sum(1) > 0
    e = normwise(df[touched], d_feat[touched], 1e-12)
    assert e.max() <= 1e-4, e.max()
    scl = np.abs(d_w).max(-1, keepdims=True) + 1e-12
    assert (np.abs(dtw.cpu().numpy() - d_w) / scl).max() <= 1e-4


@pytest.mark.parametrize("K,fdt,D,spread", [(4, "bf16", 512, 24), (8, "fp8", 512, 30),
                                            (4, "bf16", 256, 20000), (3, "fp8", 200, 14)])
def test_fused_l1_matches_unfused(torch, K, fdt, D, spread):
    """The fused L1 adjoint recomputes the map; it must take every sign decision as
    l1_grad does on the stored map, exact ties (F == F^) and one-ulp gaps included."""
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(7 * K + D)
    views, H, W, n = 1, 48, 64, 30000
    feat = rng.standard_normal((n, D)).astype(np.float32)
    ids, w = _synthetic_topk(rng, views, H, W, K, n, spread)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    store, sc8 = render.quantize(dev(feat), fdt)
    F = render.feature_fwd(dev(ids), dev(w), store, sc8, fdt, "bf16")
    bits = F.view(torch.int16).clone()
    pick = torch.from_numpy(rng.integers(0, 3, tuple(bits.shape))).cuda()
    step = torch.from_numpy(rng.choice([-1, 1], tuple(bits.shape)).astype(np.int16)).cuda()
    tb = torch.where(pick == 1, bits + step, bits)
    rnd = torch.from_numpy(rng.standard_normal(tuple(bits.shape)).astype(np.float32)).cuda()
    target = torch.where(pick == 2, rnd.to(torch.bfloat16), tb.view(torch.bfloat16)).contiguous()
    scale = 1.0 / F.numel()
    gF = render.l1_grad(F, target, scale)
    d1 = torch.zeros(n, D, device="cuda")
    d2 = torch.zeros(n, D, device="cuda")
    t1 = render.feature_bwd(dev(ids), dev(w), store, sc8, fdt, "bf16", gF, d1)
    t2 = render.feature_bwd_l1(dev(ids), dev(w), store, sc8, fdt, "bf16", target, scale, d2)
    torch.cuda.synchronize()
    # the fused path sums signs and scales the sums, so values agree to rounding; one
    # flipped sign would move a pixel's dot product by about a tenth
    assert torch.equal(d1 != 0, d2 != 0)
    rel = ((d1 - d2).norm(dim=1) / d2.norm(dim=1).clamp_min(1e-30)).max().item()
    assert rel <= 1e-6, rel
    scl = t2.abs().amax(-1, keepdim=True).clamp_min(1e-30)
    e = ((t1 - t2).abs() / scl).max().item()
    assert e <= 1e-5, e


@pytest.mark.parametrize("K,fdt,mdt,views,H,W,D,spread", [
    (4, "bf16", "bf16", 1, 40, 53, 512, 24),       # MFMA path, ragged tiles
    (8, "fp8", "bf16", 2, 33, 40, 768, 30),        # FP8 rows, D = 768 (two 384-channel slabs), two views
    (8, "bf16", "bf16", 1, 40, 53, 512, 24),       # K = 8 MFMA path (compact slot table), unions <= 32
    (8, "fp8", "bf16", 1, 40, 40, 512, 30),        # K = 8 MFMA path with FP8 row scales
    (4, "bf16", "bf16", 1, 48, 48, 256, 20000),    # unions beyond 32: per-pixel path in the same launch
    (3, "bf16", "f32", 1, 20, 36, 200, 14),        # FP32 map, channel tail
    (4, "f32", "f32", 1, 37, 53, 64, 40),          # FP32 form
    (4, "f32", "f32", 1, 40, 53, 512, 24),         # FP32 rows as three BF16 terms: two 256-channel slabs
    (8, "f32", "f32", 2, 33, 40, 768, 30),         # FP32 form at K = 8, D = 768: three slabs, two views
    (8, "fp8", "f32", 1, 40, 40, 520, 30),         # FP8 rows, FP32 map, channel tail (slabs of 6, 6, 5 chunks)
    (4, "f32", "f32", 1, 48, 48, 256, 20000),      # FP32 form, unions beyond 32 beside MFMA tiles
    # unions of 33..64 at K > 4: four union blocks, one chunk per wave, several slabs
    (8, "bf16", "bf16", 1, 40, 53, 512, 48),
    (8, "fp8", "bf16", 1, 33, 40, 768, 60),
    (8, "f32", "f32", 1, 32, 40, 264, 40),
    (5, "bf16", "f32", 1, 30, 30, 200, 36),
    (16, "bf16", "bf16", 1, 32, 32, 128, 300)])    # K beyond the MFMA path
def test_one_pass_render_and_l1_adjoint(torch, orc, K, fdt, mdt, views, H, W, D, spread):
    """lgs_feature_render_fwd_bwd_l1 against the two separate launches (the map bit for
    bit, dL/dw bit for bit, dL/df to summation order) on a target with exact ties and
    one-ulp gaps, and against the oracle on a target kept clear of the map."""
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(13 * K + D + views)
    n = 30000
    feat = rng.standard_normal((n, D)).astype(np.float32)
    ids, w = _synthetic_topk(rng, views, H, W, K, n, spread)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    store, sc8 = render.quantize(dev(feat), fdt)
    ids_d, w_d = dev(ids), dev(w)
    scale = 1.0 / (views * H * W * D)
    F1 = render.feature_fwd(ids_d, w_d, store, sc8, fdt, mdt, views=views)
    ibits = torch.int16 if mdt == "bf16" else torch.int32
    bits = F1.view(ibits).clone()
    pick = torch.from_numpy(rng.integers(0, 3, tuple(bits.shape))).cuda()
    step = torch.from_numpy(rng.choice([-1, 1], tuple(bits.shape))).cuda().to(ibits)
    rnd = torch.from_numpy(rng.standard_normal(tuple(bits.shape)).astype(np.float32)).cuda().to(F1.dtype)
    # one-ulp neighbours of nonzero values only (a step off +0 would make a NaN)
    near = torch.where((pick == 1) & (F1 != 0), bits + step, bits).view(F1.dtype)
    target = torch.where(pick == 2, rnd, near).contiguous()
    for _ in range(2):   # twice: everything but the order of the dL/df atomics repeats exactly
        d1 = torch.zeros(n, D, device="cuda")
        d2 = torch.zeros(n, D, device="cuda")
        t1 = render.feature_bwd_l1(ids_d, w_d, store, sc8, fdt, mdt, target, scale, d1, views=views)
        F2, t2 = render.feature_fwd_bwd_l1(ids_d, w_d, store, sc8, fdt, mdt, target, scale, d2, views=views)
        torch.cuda.synchronize()
        assert torch.equal(F2.view(ibits), F1.view(ibits))
        assert torch.equal(t2, t1)
        assert torch.equal(d1 != 0, d2 != 0)
        rel = ((d1 - d2).norm(dim=1) / d2.norm(dim=1).clamp_min(1e-30)).max().item()
        assert rel <= 1e-6, rel

    # against the oracle, with the target well clear of the map
    if fdt == "f32":
        f64 = feat.astype(np.float64)
    elif fdt == "bf16":
        f64 = orc.bf16_to_f64(orc.bf16_bits(feat)).reshape(feat.shape)
    else:
        c, s = orc.fp8_quantize(feat)
        f64 = orc.fp8_dequant(c, s)
    Fo = orc.feature(ids, w.astype(np.float64), f64)
    delta = rng.choice([-1.0, 1.0], Fo.shape) * (0.02 + 0.05 * np.abs(Fo))
    tmap = torch.float32 if mdt == "f32" else torch.bfloat16
    T_dev = dev((Fo + delta).astype(np.float32)).to(tmap)
    T_m = T_dev.float().cpu().numpy().astype(np.float64)
    d3 = torch.zeros(n, D, device="cuda")
    F3, t3 = render.feature_fwd_bwd_l1(ids_d, w_d, store, sc8, fdt, mdt, T_dev, scale, d3, views=views)
    torch.cuda.synchronize()
    err = normwise(F3.float().cpu().numpy().astype(np.float64), Fo, 1e-2)
    assert err.max() <= (1e-4 if mdt == "f32" else 1e-2), err.max()
    gs = scale if mdt == "f32" else float(torch.tensor(scale).to(torch.bfloat16).float())
    d_feat, d_w = orc.feature_backward(ids, w.astype(np.float64), f64, gs * np.sign(Fo - T_m))
    df = d3.cpu().numpy()
    touched = np.abs(d_feat).sum(1) > 0
    e = normwise(df[touched], d_feat[touched], 1e-12)
    assert e.max() <= 1e-4, e.max()
    assert np.all(df[~touched] == 0)
    scl = np.abs(d_w).max(-1, keepdims=True) + 1e-12
    assert (np.abs(t3.cpu().numpy() - d_w) / scl).max() <= 1e-4


@pytest.mark.parametrize("n,below,ratio,seed", [(1, 1, 0.5, 0), (1000, 3, 0.5, 1), (300000, 4, 0.5, 2),
                                                 (300000, 2, 0.0, 3), (300000, 5, 1.0, 4), (70001, 100, 0.37, 5)])
def test_prune_select_matches_oracle(torch, orc, n, below, ratio, seed):
    """The Eq. 6 survival draw on seeded inputs (counts, importances with zeros and
    exact key ties, exponential variates): the survive mask bit for bit."""
    from paper_2602_06991_amd import render
    rng = np.random.default_rng(seed)
    count = rng.integers(0, 8, n).astype(np.int32)
    S = np.where(rng.random(n) < 0.1, 0.0, rng.choice([0.25, 0.5, 1.0, 0.3], n) * rng.random(n) ** 2)
    S = np.where(rng.random(n) < 0.3, 0.5, S).astype(np.float32)
    E = np.where(rng.random(n) < 0.3, 1.0, rng.exponential(size=n)).astype(np.float32)
    dev = lambda a: torch.from_numpy(a).cuda()
    got = render.prune_select(dev(count), dev(S), below, dev(E), ratio).cpu().numpy()
    want = orc.prune_select(count, S, below, E, ratio)
    cand = count < below
    print(f"n={n}: candidates {cand.sum()}, survivors among them {want[cand].sum()}", flush=True)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_marked_row_refresh_feeds_the_feature_kernels_the_whole_table_bits(torch, form):
    """A store refreshed only in the rows the step's Top-K lists stamp gives the one-pass
    feature render + L1 adjoint exactly what the whole-table conversion gives, step after
    step, while the FP32 master table changes between steps and the Top-K sets change
    (three views of a room, then the first again): the map and dL/dw bit for bit, the
    gradient rows to summation order."""
    from paper_2602_06991_amd import render
    sc = make_scene(3, N=60000, W=200, H=150, D=64)
    g = sc.gaussians
    n, d = g.n, g.d
    feat = torch.from_numpy(np.ascontiguousarray(g.feat, np.float32)).cuda()
    store = render.quantize(feat, form)                # rows refreshed below; the rest stale
    rows = render.SparseGradRows(torch.zeros(n, d, device="cuda"))
    gen = torch.Generator(device="cuda").manual_seed(4)
    for step, v in enumerate([0, 1, 2, 0]):
        feat.add_(torch.randn(n, d, device="cuda", generator=gen), alpha=0.05)   # an optimiser's update
        out, st = gpu_forward(g, sc.cameras[v], 4)
        fw = st["fw"]
        rows.clear()
        rows.mark(fw["ids"])
        rows.quantize(feat, form, store)
        whole = render.quantize(feat, form)
        target = torch.randn(fw["ids"].shape[0], fw["ids"].shape[1], d, device="cuda", generator=gen)
        target = target.to(torch.bfloat16)
        res = []
        for s_, sc_ in (store, whole):
            gf = torch.zeros(n, d, device="cuda")
            F, dtw = render.feature_fwd_bwd_l1(fw["ids"], fw["w"], s_, sc_, form, "bf16", target, 1e-3, gf)
            res.append((F, dtw, gf))
        torch.cuda.synchronize()
        (F0, w0, g0), (F1, w1, g1) = res
        assert torch.equal(F0.view(torch.int16), F1.view(torch.int16)), step
        assert torch.equal(w0, w1), step
        rel = float((g0 - g1).norm() / g1.norm().clamp_min(1e-30))
        assert rel <= 1e-6, (step, rel)
        # the refreshed rows are the whole table's bits
        ids = fw["ids"].reshape(-1)
        used = torch.unique(ids[ids >= 0]).long()
        assert torch.equal(store[0][used].view(torch.uint8), whole[0][used].view(torch.uint8)), step
        if form == "fp8":
            assert torch.equal(store[1][used], whole[1][used]), step


def test_sparse_gradient_clearing_matches_dense(torch):
    """Clearing the feature-gradient table by zeroing the rows the previous step's Top-K
    lists named gives the table dense zeroing gives, step after step, with the Top-K sets
    changing between steps (three views of a room scene, then the first again)."""
    from paper_2602_06991_amd import render
    sc = make_scene(3, N=60000, W=200, H=150, D=64)
    g = sc.gaussians
    P = dev_params(g)
    n, d = g.n, g.d
    store, scale = render.quantize(P["feat"], "bf16")
    dense = torch.zeros(n, d, device="cuda")
    table = torch.zeros(n, d, device="cuda")
    rows = render.SparseGradRows(table)
    gen = torch.Generator(device="cuda").manual_seed(3)
    for step, v in enumerate([0, 1, 2, 0]):
        out, st = gpu_forward(g, sc.cameras[v], 4)
        fw = st["fw"]
        target = torch.randn(fw["ids"].shape[0], fw["ids"].shape[1], d, device="cuda", generator=gen).to(torch.bfloat16)
        dense.zero_()
        render.feature_bwd_l1(fw["ids"], fw["w"], store, scale, "bf16", "bf16", target, 1e-3, dense)
        rows.clear()
        rows.mark(fw["ids"])
        render.feature_bwd_l1(fw["ids"], fw["w"], store, scale, "bf16", "bf16", target, 1e-3, table)
        torch.cuda.synchronize()
        nz = dense.abs().sum(1) > 0
        assert torch.equal(nz, table.abs().sum(1) > 0), step
        rel = float((dense - table).norm() / dense.norm().clamp_min(1e-30))
        assert rel <= 1e-6, (step, rel)
        ids = fw["ids"].reshape(-1)
        marked = torch.zeros(n, dtype=torch.bool, device="cuda")
        marked[ids[ids >= 0].long()] = True
        assert torch.equal(rows.row_gen == step, marked), step
        assert not bool(nz[~marked].any())        # every written row was marked
