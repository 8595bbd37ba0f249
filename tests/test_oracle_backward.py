"""Pins of the oracle's adjoint: FP64 central finite differences of a random linear
functional of (C, D, O, F), conservation laws of the feature terms, and the K = 1
special case."""
import numpy as np
import pytest

from paper_2602_06991_amd.scenegen import Gaussians, make_scene, make_tiny

H_STEP = 2.0 ** -13     # x +- h is exact in float32 for |x| < 1024


def _loss(orc, g, cam, K, R):
    r = orc.render(g, cam, K)
    F = orc.feature(r["ids"], r["w"], g.feat.astype(np.float64))
    L = ((r["C"] * R["C"]).sum() + (r["D"] * R["D"]).sum() + (r["O"] * R["O"]).sum()
         + (F * R["F"]).sum())
    return L, (r["sig"].tobytes(), r["ids"].tobytes())


def _with(g, name, idx, val):
    arrs = {k: getattr(g, k).copy() for k in ("means", "log_scales", "quats", "opacity_logits", "rgb", "feat")}
    arrs[name][idx] = val
    return Gaussians(**arrs)


@pytest.mark.parametrize("seed,K,spread", [(0, 4, (-0.1, 1.1)), (1, 3, (-0.1, 1.1)), (2, 1, (-0.1, 1.1)),
                                           (3, 8, (-0.1, 1.1)), (4, 4, (-0.7, 1.7))])
def test_adjoint_matches_central_differences(orc, seed, K, spread):
    # the wide spread puts Gaussians beyond the 1.3x guard band (clamped Jacobian)
    g, cam = make_tiny(100 + seed, n=14, W=22, H=18, D=6, scale=(-2.3, 0.4), opl=(0.3, 0.8),
                       spread=spread)
    if spread[0] < -0.5:
        g = Gaussians(g.means, (g.log_scales + 1.2).astype(np.float32), g.quats, g.opacity_logits,
                      g.rgb, g.feat)
    rng = np.random.default_rng(seed)
    P = cam.W * cam.H
    R = dict(C=rng.standard_normal((cam.H, cam.W, 3)), D=rng.standard_normal((cam.H, cam.W)),
             O=rng.standard_normal((cam.H, cam.W)), F=rng.standard_normal((cam.H, cam.W, g.d)))
    b = orc.backward(g, cam, K, g.feat.astype(np.float64), R["C"], R["D"], R["O"], R["F"])
    base_L, base_sig = _loss(orc, g, cam, K, R)
    names = {"means": "d_means", "log_scales": "d_log_scales", "quats": "d_quats",
             "opacity_logits": "d_opacity_logits", "rgb": "d_rgb", "feat": "d_feat"}
    checked = 0
    tried = 0
    while checked < 64 and tried < 400:
        tried += 1
        name = list(names)[rng.integers(len(names))]
        arr = getattr(g, name)
        idx = tuple(rng.integers(s) for s in arr.shape)
        x = arr[idx]
        xp, xm = np.float32(x + H_STEP), np.float32(x - H_STEP)
        Lp, sp = _loss(orc, _with(g, name, idx, xp), cam, K, R)
        Lm, sm = _loss(orc, _with(g, name, idx, xm), cam, K, R)
        if sp != base_sig or sm != base_sig:
            continue          # a discrete decision flipped inside the stencil
        fd = (Lp - Lm) / (float(xp) - float(xm))
        an = b[names[name]][idx]
        scale = max(abs(an), abs(fd), 1e-3 * np.abs(b[names[name]]).max(), 1e-8)
        assert abs(an - fd) <= 1e-5 * scale, (name, idx, an, fd)
        checked += 1
    assert checked >= 48, (checked, tried)


def test_feature_conservation_and_gamma_orthogonality(orc):
    sc = make_scene(0, N=4000, W=48, H=40, D=8)
    g, cam = sc.gaussians, sc.cameras[0]
    K = 4
    rng = np.random.default_rng(5)
    gF = rng.standard_normal((cam.H, cam.W, 8))
    r = orc.render(g, cam, K)
    b = orc.backward(g, cam, K, g.feat.astype(np.float64), None, None, None, gF)
    W = r["w"].sum(-1)
    # sum_g dL/df_g = sum over pixels with W > 0 of G_F, because the w' sum to one
    np.testing.assert_allclose(b["d_feat"].sum(0), gF[W > 0].sum(0), rtol=1e-11, atol=1e-11)
    # sum_k gamma_k w_k = 0 per pixel (F is invariant to scaling all Top-K weights)
    np.testing.assert_allclose((b["d_topkw"] * r["w"]).sum(-1), 0, atol=1e-10)


def test_k1_feature_loss_gives_no_geometry_gradient(orc):
    sc = make_scene(0, N=4000, W=48, H=40, D=8)
    g, cam = sc.gaussians, sc.cameras[0]
    gF = np.random.default_rng(6).standard_normal((cam.H, cam.W, 8))
    b = orc.backward(g, cam, 1, g.feat.astype(np.float64), None, None, None, gF)
    for k in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_rgb", "d_topkw"):
        assert np.all(b[k] == 0), k
    assert np.abs(b["d_feat"]).max() > 0


def test_screen_space_gradients_match_differences_of_a_linear_functional(orc):
    """The per-Gaussian colour and depth slots are exact sums of w (linear in c, z)."""
    g, cam = make_tiny(7, n=20, W=24, H=20, D=4)
    r = orc.render(g, cam, 63)
    ones = np.ones((cam.H, cam.W))
    b = orc.backward(g, cam, 4, g.feat.astype(np.float64), np.ones((cam.H, cam.W, 3)), None, None, None)
    tot = np.zeros(g.n)
    for k in range(63):
        ids = r["ids"][..., k]
        m = ids >= 0
        np.add.at(tot, ids[m], r["w"][..., k][m])
    np.testing.assert_allclose(b["d_rgb"][:, 0], tot, rtol=1e-12, atol=1e-15)
    b2 = orc.backward(g, cam, 4, g.feat.astype(np.float64), None, ones, None, None)
    np.testing.assert_allclose(b2["d_z"], tot, rtol=1e-12, atol=1e-15)


def test_feature_adjoint_by_differences(orc):
    """The stand-alone feature adjoint: F is linear in f and a ratio in w, so central
    differences in w and f of L = <R, F(w, f)> pin d_w and d_feat."""
    rng = np.random.default_rng(9)
    n, D, K, P = 30, 6, 4, 50
    ids = np.stack([rng.choice(n, K, replace=False) for _ in range(P)]).astype(np.int32)
    ids[3, 2:] = -1
    w = rng.uniform(0.01, 0.5, (P, K))
    w[ids < 0] = 0
    w[7] = 0
    ids[7] = -1
    f = rng.standard_normal((n, D))
    R = rng.standard_normal((P, D))
    d_feat, d_w = orc.feature_backward(ids, w, f, R)
    L = lambda w_, f_: (orc.feature(ids, w_, f_) * R).sum()
    h = 1e-6
    for _ in range(40):
        p, k = rng.integers(P), rng.integers(K)
        if ids[p, k] < 0:
            assert d_w[p, k] == 0
            continue
        wp, wm = w.copy(), w.copy()
        wp[p, k] += h
        wm[p, k] -= h
        fd = (L(wp, f) - L(wm, f)) / (2 * h)
        assert abs(fd - d_w[p, k]) <= 1e-6 * max(1, abs(fd))
    for _ in range(40):
        g, c = rng.integers(n), rng.integers(D)
        fp, fm = f.copy(), f.copy()
        fp[g, c] += h
        fm[g, c] -= h
        fd = (L(w, fp) - L(w, fm)) / (2 * h)
        assert abs(fd - d_feat[g, c]) <= 1e-6 * max(1, abs(fd))
    assert np.all(d_w[7] == 0)


def test_feature_adjoint_agrees_with_full_adjoint(orc):
    sc = make_scene(0, N=3000, W=48, H=40, D=8)
    g, cam = sc.gaussians, sc.cameras[0]
    r = orc.render(g, cam, 4)
    gF = np.random.default_rng(2).standard_normal((cam.H, cam.W, 8))
    b = orc.backward(g, cam, 4, g.feat.astype(np.float64), None, None, None, gF)
    d_feat, d_w = orc.feature_backward(r["ids"], r["w"], g.feat.astype(np.float64), gF)
    np.testing.assert_allclose(d_feat, b["d_feat"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(d_w, b["d_topkw"], rtol=1e-12, atol=1e-13)
