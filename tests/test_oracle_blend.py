"""Pins of the oracle's blend (Eq. 1) and Top-K selection (Eq. 2): single-Gaussian
closed form, hand-derived multi-Gaussian weights, brute force over every Gaussian
at every pixel, and invariants."""
import json
import math
import os

import numpy as np
import pytest

from paper_2602_06991_amd.scenegen import Gaussians, identity_camera, make_scene, make_tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gs(means, log_scales, quats, opls, rgbs, feats):
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    return Gaussians(f(means), f(log_scales), f(quats), f(opls), f(rgbs), f(feats))


def test_single_gaussian_closed_form(orc):
    cam = identity_camera(40, 32)
    g = _gs([[0.05, -0.03, 2.0]], [np.log([0.06, 0.03, 0.02])], [[0.9, 0.1, -0.2, 0.3]],
            [1.5], [[0.2, 0.6, 0.9]], [[1, 0, 0, 0]])
    r = orc.render(g, cam, 4)
    p = orc.project(g, cam)
    A, B, C = p["cov2d"][0]
    det = A * C - B * B
    qa, qb, qc = C / det, -B / det, A / det
    mx, my = p["mean2d"][0]
    o = 1 / (1 + math.exp(-float(g.opacity_logits[0])))
    z = p["tview"][0, 2]
    ys, xs = np.mgrid[0:cam.H, 0:cam.W]
    dx, dy = xs + 0.5 - mx, ys + 0.5 - my
    sig = 0.5 * (qa * dx * dx + qc * dy * dy) + qb * dx * dy
    alpha = np.minimum(0.99, o * np.exp(-sig))
    hit = alpha >= 1 / 255
    a = np.where(hit, alpha, 0.0)
    np.testing.assert_allclose(r["O"], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["T"], 1 - a, rtol=1e-12)
    np.testing.assert_allclose(r["D"], z * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["C"], a[..., None] * g.rgb[0].astype(np.float64), rtol=1e-12, atol=1e-15)
    assert hit.sum() > 20 and (~hit).sum() > 20
    assert np.all(r["ids"][hit][:, 0] == 0) and np.all(r["ids"][hit][:, 1:] == -1)
    assert np.all(r["ids"][~hit] == -1) and np.all(r["w"][~hit] == 0)
    F = orc.feature(r["ids"], r["w"], g.feat.astype(np.float64))
    np.testing.assert_array_equal(F[hit], np.broadcast_to(g.feat[0], (hit.sum(), 4)))
    assert np.all(F[~hit] == 0)


def test_hand_derived_weights_golden(orc):
    """Three Gaussians centred on one pixel centre (sigma = 0 there, so alpha = o):
    w1 = a1, w2 = a2 (1 - a1), w3 = a3 (1 - a1)(1 - a2)  (Eq. 1).  The fixture's
    expected values are derived by hand in the file."""
    fx = json.load(open(os.path.join(GOLDEN, "three_gaussians_one_pixel.json")))
    cam = identity_camera(fx["W"], fx["H"], f=fx["f"])
    g = _gs(fx["means"], fx["log_scales"], fx["quats"], fx["opacity_logits"], fx["rgb"], fx["feat"])
    r = orc.render(g, cam, fx["K"])
    py, px = fx["pixel"]
    np.testing.assert_allclose(r["w"][py, px], fx["expect_topk_w"], rtol=1e-12)
    assert list(r["ids"][py, px]) == fx["expect_topk_ids"]
    np.testing.assert_allclose(r["C"][py, px], fx["expect_C"], rtol=1e-12)
    np.testing.assert_allclose(r["T"][py, px], fx["expect_T"], rtol=1e-12)
    F = orc.feature(r["ids"], r["w"], g.feat.astype(np.float64))
    np.testing.assert_allclose(F[py, px], fx["expect_F"], rtol=1e-12)


def test_t_floor_stops_before_the_saturating_gaussian(orc):
    # Four opaque Gaussians (alpha = 0.95 at the pixel): T after three is 1.25e-4; the
    # fourth would take it to 6.25e-6 < 1e-4, so it is not blended.
    cam = identity_camera(16, 16, f=16.0)
    n = 4
    o = 0.95
    opl = math.log(o / (1 - o))
    g = _gs([[0.5 / 16 * z, 0.5 / 16 * z, z] for z in (1.0, 1.5, 2.0, 2.5)], [np.log([0.05] * 3)] * n,
            [[1, 0, 0, 0]] * n, [opl] * n, [[1, 1, 1]] * n, [[1, 0]] * n)
    r = orc.render(g, cam, 8)
    p = orc.project(g, cam)
    # pixel (8, 8) has its centre at (8.5, 8.5) = every mean2D
    np.testing.assert_allclose(p["mean2d"], [[8.5, 8.5]] * n, atol=1e-12)
    oo = 1 / (1 + np.exp(-g.opacity_logits.astype(np.float64)))
    assert r["nblend"][8, 8] == 3
    np.testing.assert_allclose(r["T"][8, 8], np.prod(1 - oo[:3]), rtol=1e-12)
    assert list(r["ids"][8, 8][:4]) == [0, 1, 2, -1]


def test_equal_depths_blend_in_id_order(orc):
    # A fronto-parallel wall: identical depth keys, so the blend order is by id.
    cam = identity_camera(16, 16, f=16.0)
    z = 2.0
    m = [0.5 / 16 * z, 0.5 / 16 * z, z]
    g = _gs([m, m], [np.log([0.05] * 3)] * 2, [[1, 0, 0, 0]] * 2, [0.0, 2.0],
            [[1, 0, 0], [0, 1, 0]], [[1, 0], [0, 1]])
    r = orc.render(g, cam, 2)
    p = orc.project(g, cam)
    assert p["zkey"][0] == p["zkey"][1]
    o = 1 / (1 + np.exp(-g.opacity_logits.astype(np.float64)))
    np.testing.assert_allclose(r["C"][8, 8], [o[0], o[1] * (1 - o[0]), 0], rtol=1e-12)
    # swap the ids: the other Gaussian now blends first
    g2 = _gs([m, m], [np.log([0.05] * 3)] * 2, [[1, 0, 0, 0]] * 2, [2.0, 0.0],
             [[0, 1, 0], [1, 0, 0]], [[0, 1], [1, 0]])
    r2 = orc.render(g2, cam, 2)
    np.testing.assert_allclose(r2["C"][8, 8], [o[0] * (1 - o[1]), o[1], 0], rtol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_equals_tiled(orc, seed):
    W, H = [(24, 20), (37, 29), (64, 64), (17, 45), (50, 33), (64, 48)][seed]
    g, cam = make_tiny(seed, n=[16, 40, 64, 30, 64, 50][seed], W=W, H=H, scale=(-2.5, 0.7))
    a = orc.render(g, cam, 4)
    b = orc.render(g, cam, 4, brute=True)
    assert a["nblend"].sum() > 0
    for k in ("C", "D", "O", "T", "nblend", "ids", "w", "sig"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_brute_force_equals_tiled_room(orc):
    sc = make_scene(0, N=3000, W=64, H=48)
    g, cam = sc.gaussians, sc.cameras[0]
    a = orc.render(g, cam, 4)
    b = orc.render(g, cam, 4, brute=True)
    assert a["nblend"].mean() > 1
    for k in ("C", "D", "O", "T", "nblend", "ids", "w"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("K", [1, 3, 4, 8])
def test_topk_invariants(orc, K):
    sc = make_scene(1, N=20000, W=96, H=72)
    g, cam = sc.gaussians, sc.cameras[0]
    full = orc.render(g, cam, 63)
    r = orc.render(g, cam, K)
    n = full["nblend"]
    ok = n <= 63
    assert ok.mean() > 0.99 and n.max() > K
    # every blended weight is listed in the K=63 run for these pixels: it sums to O
    np.testing.assert_allclose(full["w"].sum(-1)[ok], full["O"][ok], rtol=1e-10, atol=1e-13)
    # 0 <= O <= 1 and T_final = 1 - O > 0
    assert np.all(full["O"] <= 1) and np.all(full["T"] > 0)
    # selected weights are the K largest, in non-increasing order
    w = r["w"]
    assert np.all(np.diff(w, axis=-1) <= 0)
    np.testing.assert_array_equal(w, full["w"][..., :K])
    np.testing.assert_array_equal(r["ids"], full["ids"][..., :K])
    # the K-th selected weight is >= every unselected blended weight
    kth = w[..., -1]
    rest = full["w"][..., K:].max(-1)
    sel = n > K
    assert np.all(kth[sel] >= rest[sel])
    # padding
    for k in range(K):
        pad = n <= k
        assert np.all(r["ids"][..., k][pad] == -1) and np.all(r["w"][..., k][pad] == 0)
    # colour, depth, opacity do not depend on K
    for key in ("C", "D", "O", "T", "nblend"):
        np.testing.assert_array_equal(r[key], full[key])


def test_transmittance_non_increasing_along_the_ray(orc):
    # Per pixel, weights in blend order are w_i = alpha_i T_i with T_i non-increasing:
    # rebuilding T from the listed weights in blend order never increases.
    g, cam = make_tiny(11, n=64, W=32, H=24, scale=(-2.0, 0.5))
    r = orc.render(g, cam, 63)
    p = orc.project(g, cam)
    for (y, x) in [(y, x) for y in range(0, 24, 3) for x in range(0, 32, 3)]:
        n = r["nblend"][y, x]
        ids = r["ids"][y, x, :n]
        ws = r["w"][y, x, :n]
        order = np.lexsort((ids, p["zkey"][ids]))
        T = 1.0
        for i in order:
            assert ws[i] <= T + 1e-15
            T -= ws[i]
            assert T >= -1e-15
        assert abs(T - r["T"][y, x]) < 1e-12
