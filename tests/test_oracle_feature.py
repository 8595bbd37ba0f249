"""Pins of the oracle's feature render (Eq. 3-4) by special cases and invariants."""
import numpy as np
import pytest

from paper_2602_06991_amd.scenegen import Gaussians, make_scene, make_tiny


def test_large_k_equals_opacity_normalised_blend(orc):
    """With K >= the blended count, Top-K rendering is the alpha blend of Eq. 1 divided
    by its opacity.  Second route: put 3 feature channels into the colour slot and
    compare F * O with the colour blend C."""
    g, cam = make_tiny(3, n=48, W=40, H=30, D=3, scale=(-2.2, 0.5))
    g3 = Gaussians(g.means, g.log_scales, g.quats, g.opacity_logits,
                   np.ascontiguousarray(g.feat[:, :3]), g.feat)
    r = orc.render(g3, cam, 63)
    assert r["nblend"].max() < 63 and r["nblend"].max() >= 3
    F = orc.feature(r["ids"], r["w"], g3.feat.astype(np.float64))
    np.testing.assert_allclose(F * r["O"][..., None], r["C"], rtol=1e-12, atol=1e-14)


def test_k1_is_argmax_feature(orc):
    sc = make_scene(1, N=20000, W=64, H=48)
    g, cam = sc.gaussians, sc.cameras[0]
    full = orc.render(g, cam, 63)
    r = orc.render(g, cam, 1)
    F = orc.feature(r["ids"], r["w"], g.feat.astype(np.float64))
    n = full["nblend"]
    sel = n > 0
    best = np.argmax(full["w"], axis=-1)                      # first maximal -> smallest (z, id)
    ids = np.take_along_axis(full["ids"], best[..., None], -1)[..., 0]
    assert np.all(r["ids"][..., 0][sel] == ids[sel])
    np.testing.assert_array_equal(F[sel], g.feat[ids[sel]].astype(np.float64))
    assert np.all(F[~sel] == 0)


def test_linearity_and_affine_invariance(orc):
    sc = make_scene(0, N=4000, W=64, H=48, D=16)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, 4)
    rng = np.random.default_rng(0)
    f1 = rng.standard_normal((g.n, 16))
    f2 = rng.standard_normal((g.n, 16))
    F1 = orc.feature(r["ids"], r["w"], f1)
    F2 = orc.feature(r["ids"], r["w"], f2)
    F12 = orc.feature(r["ids"], r["w"], 2.0 * f1 - 3.0 * f2)
    np.testing.assert_allclose(F12, 2.0 * F1 - 3.0 * F2, rtol=1e-12, atol=1e-12)
    v = rng.standard_normal(16)
    Fv = orc.feature(r["ids"], r["w"], f1 + v)
    W = r["w"].sum(-1)
    pos = W > 0
    assert pos.mean() > 0.3 and (~pos).sum() > 0
    np.testing.assert_allclose(Fv[pos], F1[pos] + v, rtol=1e-12, atol=1e-12)
    assert np.all(Fv[~pos] == 0)


def test_renormalised_weights_sum_to_one(orc):
    sc = make_scene(0, N=4000, W=64, H=48, D=4)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, 4)
    ones = np.ones((g.n, 1))
    F = orc.feature(r["ids"], r["w"], ones)[..., 0]
    W = r["w"].sum(-1)
    np.testing.assert_allclose(F[W > 0], 1.0, rtol=1e-14)


def test_topk_selection_ties_keep_blend_order(orc):
    """Eq. 2 orders by weight only; equal weights keep the earlier Gaussian in blend
    order, i.e. the smaller depth key, then the smaller id."""
    assert list(orc.topk_select([0.2, 0.5, 0.2, 0.5, 0.1], 5)) == [1, 3, 0, 2, 4]
    assert list(orc.topk_select([0.3, 0.3, 0.3], 2)) == [0, 1]
    assert list(orc.topk_select([0.1, 0.4], 4)) == [1, 0]
    assert list(orc.topk_select([], 3)) == []
    w = np.random.default_rng(1).random(40)
    np.testing.assert_array_equal(orc.topk_select(w, 10), np.argsort(-w, kind="stable")[:10])
