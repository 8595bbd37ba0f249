"""The blend's dispatch order (lgs_tile_order): a scheduling aid that must change no
result.  Checked on one 1200x680 view (tiles dealt to the XCDs in strips) and on the
8 keyframes of the 640x480 room workload (whole views per XCD), for both weights (the
pair counts; the forward's largest n_contrib per tile): the order is a permutation of
the padded grid; each XCD keeps the tiles the fixed mapping gives it, heaviest weight
bucket first; the blend and the pruning statistics with the order give the same bits
as without; the adjoint's atomic sums match to summation order."""
import numpy as np
import pytest

from gpu_util import dev_params
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


def _fixed_mapping(G, bands):
    """Block -> tile of the kernels without an order (host restatement, for the test)."""
    b = np.arange(G)
    if bands:
        return (b & 7) * (G // 8) + (b >> 3)
    x, l = b & 7, b >> 3
    return ((l // 16) * 8 + x) * 16 + (l % 16)


def _heaviest_first(w):
    """Each later tile's weight bucket (8 log2(w + 1), floored, at most 255) is at most
    an earlier one's; the kernel takes the logarithm in FP32, so a weight on a bucket
    edge may fall either side (1e-4)."""
    v = np.minimum(8.0 * np.log2(w.astype(np.float64) + 1.0), 255.0)
    run = np.minimum.accumulate(np.floor(v + 1e-4))
    return bool(np.all(v[1:] < run[:-1] + 1.0 + 1e-4))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cfg,K,N", [(2, 4, 200000), (3, 4, None)])
def test_tile_order_changes_no_result(torch, cfg, K, N):
    from paper_2602_06991_amd import lgs, render
    sc = make_scene(cfg, N=N, D=8) if N else make_scene(cfg, D=8)
    g = sc.gaussians
    n, V = g.n, len(sc.cameras)
    cams_l = [lgs.make_camera(c) for c in sc.cameras]
    W, H = cams_l[0].width, cams_l[0].height
    P = dev_params(g)
    if V == 1:
        cams = cams_l[0]
        proj = render.project(cams, P)
        ids, ranges, m = render.Binner()(cams, n, proj["depth"], proj["tile_rect"], proj["tiles_touched"])
        fwd = lambda o: render.rasterize(cams, K, proj, P["rgb"], ids, ranges, order=o)
        sgb = lambda: render.screen_grad_buffers(n, "cuda")
        bwd = lambda f, sg, o: render.rasterize_bwd(cams, K, proj, P["rgb"], ids, ranges, f, gC, gD, gO, dtw, sg,
                                                     order=o)
    else:
        cams = lgs.camera_array(cams_l)
        proj = render.project_views(cams, P)
        ids, ranges, m = render.Binner()(cams, n, proj["depth"], proj["tile_rect"], proj["tiles_touched"], views=V)
        fwd = lambda o: render.rasterize_views(cams, K, n, proj, P["rgb"], ids, ranges, order=o)
        sgb = lambda: render.screen_grad_buffers_views(n, V, "cuda")
        bwd = lambda f, sg, o: render.rasterize_bwd_views(cams, K, n, proj, P["rgb"], ids, ranges, f, gC, gD, gO,
                                                           dtw, sg, order=o)
    order = render.tile_order(cams, ranges, views=V)
    torch.cuda.synchronize()
    nt = ((W + 15) // 16) * ((H + 15) // 16) * V
    G = lgs.lgs_tile_order_size(W, H, V) // 2
    print(f"config {cfg}: {V} x {W}x{H}, N={n}, {nt} tiles, grid {G}, {m} pairs", flush=True)
    assert G % 128 == 0 and nt <= G < nt + 128
    fixed = _fixed_mapping(G, V % 8 == 0)
    assert np.array_equal(np.sort(fixed), np.arange(G))

    def check(order, wt):
        o = order[:G].cpu().numpy().astype(np.int64)
        assert np.array_equal(np.sort(o), np.arange(G))
        w = np.full(G, -1, np.int64)
        w[:nt] = wt
        for x in range(8):
            got, want = o[x::8], fixed[x::8]
            assert np.array_equal(np.sort(got), np.sort(want)), x    # the XCD keeps its tiles
            real = got[got < nt]
            assert np.all(got[len(real):] >= nt), x                   # padding last
            assert _heaviest_first(w[real]), x                        # heaviest bucket first

    r = ranges.cpu().numpy().astype(np.int64)
    check(order, r[:, 1] - r[:, 0])
    # the blend: the same bits with and without the order
    f0, f1 = fwd(None), fwd(order)
    torch.cuda.synchronize()
    for k in f0:
        assert torch.equal(f0[k], f1[k]), k
    # the adjoint: the same sums up to the order of the atomics
    gC, gD, gO, _ = random_upstream(5, V * W * H, 8)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    gC, gD, gO = t(gC.reshape(V * H, W, 3)), t(gD.reshape(V * H, W)), t(gO.reshape(V * H, W))
    gen = torch.Generator(device="cuda").manual_seed(11)
    dtw = torch.randn(V * H, W, K, device="cuda", generator=gen)
    # the adjoint's order, weighted by the largest n_contrib of each tile
    border = render.tile_order(cams, ranges, views=V, n_contrib=f0["n_contrib"])
    torch.cuda.synchronize()
    nc = np.zeros((V, (H + 15) // 16 * 16, (W + 15) // 16 * 16), np.int64)
    nc[:, :H, :W] = f0["n_contrib"].cpu().numpy().reshape(V, H, W)
    check(border, nc.reshape(V, (H + 15) // 16, 16, (W + 15) // 16, 16).max(axis=(2, 4)).reshape(-1))
    s0, s1, s2 = sgb(), sgb(), sgb()
    bwd(f0, s0, None)
    bwd(f0, s1, order)
    bwd(f0, s2, border)
    torch.cuda.synchronize()
    # the pruning statistics (integer counts, maxima of non-negative weights): the same bits
    stats = []
    for o in (None, border):
        cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
        mxw = torch.zeros(n, device="cuda")
        lgs.lgs_prune_stats_views(cams if V > 1 else lgs.camera_array([cams]), V, K, n, proj["mean2d"].data_ptr(),
                                  proj["conic"].data_ptr(), proj["opacity"].data_ptr(), ids.data_ptr(),
                                  ranges.data_ptr(), f0["n_contrib"].data_ptr(), f0["ids"].data_ptr(),
                                  cnt.data_ptr(), mxw.data_ptr(), torch.cuda.current_stream().cuda_stream,
                                  tile_order=None if o is None else o.data_ptr())
        stats.append((cnt, mxw))
    torch.cuda.synchronize()
    assert torch.equal(stats[0][0], stats[1][0]) and torch.equal(stats[0][1], stats[1][1])
    assert int(stats[0][0].sum()) > 0
    for k in s0:
        a = s0[k].double()
        for name, sx in (("pair-count order", s1), ("n_contrib order", s2)):
            e = float((a - sx[k].double()).norm() / a.norm().clamp_min(1e-30))
            print(f"   {k}: {name} vs fixed mapping rel {e:.2e}", flush=True)
            assert e <= 1e-5, (k, name, e)
