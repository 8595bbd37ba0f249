"""Pins of the oracle's decision margins (the relative distance of each exp- or
product-dependent decision of the blend to its threshold; Eq. 1, Eq. 2).

The GPU parity tests trust these margins to pick the pixels where an FP32
implementation may legitimately decide otherwise, so each margin is pinned on a
scene built to put that decision at a chosen relative distance delta from its
threshold: one to three Gaussians whose means project exactly onto the centre of
pixel (8, 8), where sigma = 0 and alpha = min(0.99, o).  The only rounding between
the construction and the margin is the FP32 opacity logit (a few 1e-7 relative), so
every margin must equal its delta to 1e-6."""
import json
import math
import os

import numpy as np
import pytest

from paper_2602_06991_amd.scenegen import Gaussians, identity_camera

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PX, PY = 8, 8
SKIP, CLAMP, TFLOOR, TOPK = range(4)


def _logit(o):
    return math.log(o / (1.0 - o))


def _stack(opacities, K=4):
    """Gaussians at depths 1, 2, ... on the ray through the centre of pixel (8, 8)
    of a 16x16 identity camera with f = 16 (mean2D = (8.5, 8.5) exactly)."""
    n = len(opacities)
    zs = [1.0 + i for i in range(n)]
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    g = Gaussians(f([[0.5 / 16 * z, 0.5 / 16 * z, z] for z in zs]), f([np.log([0.05] * 3)] * n),
                  f([[1, 0, 0, 0]] * n), f([_logit(o) for o in opacities]), f([[0.5, 0.5, 0.5]] * n),
                  f([[1.0, 0.0]] * n))
    return g, identity_camera(16, 16, f=16.0)


def _margins(orc, opacities, K=4):
    g, cam = _stack(opacities, K)
    p = orc.project(g, cam)
    np.testing.assert_allclose(p["mean2d"], [[PX + 0.5, PY + 0.5]] * len(opacities), atol=1e-12)
    r = orc.render(g, cam, K)
    return r, r["margins"][PY, PX]


@pytest.mark.parametrize("delta", [1e-3, 3e-5, 2.0])
def test_skip_margin(orc, delta):
    # o = (1 + delta) / 255: alpha * 255 sits delta above the skip threshold
    r, m = _margins(orc, [(1.0 + delta) / 255.0])
    assert r["nblend"][PY, PX] == 1
    assert abs(m[SKIP] - delta) <= 1e-6 * max(1.0, delta)
    flagged = lambda e: bool(orc.flagged(r["margins"], eps_skip=e, eps_clamp=0, eps_T=0, eps_topk=0)[PY, PX])
    assert flagged(2 * delta) and not flagged(0.5 * delta)


@pytest.mark.parametrize("delta", [1e-3, 3e-5])
def test_skip_margin_below_the_threshold(orc, delta):
    # A Gaussian that is not culled (o = 2/255) but skipped at the next pixel, (9, 8),
    # one pixel right of its centre: isotropic on the optical axis of a 17x17 camera (so
    # pixel (8, 8) is centred on the axis), Sigma2D = ((f s / z)^2 + 0.3) I,
    # so sigma there = 1 / (2 Sigma2D_xx); the scale is chosen so that alpha = o e^-sigma =
    # (1 - delta) / 255, delta below the threshold.  The skipped candidate still counts.
    o = 2.0 / 255.0
    sig = math.log(2.0 / (1.0 - delta))
    s = math.sqrt(0.5 / sig - 0.3) / 16.0
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    g = Gaussians(f([[0.0, 0.0, 1.0]]), f([[math.log(s)] * 3]), f([[1, 0, 0, 0]]), f([_logit(o)]),
                  f([[0.5, 0.5, 0.5]]), f([[1.0, 0.0]]))
    cam = identity_camera(17, 17, f=16.0)
    p = orc.project(g, cam)
    np.testing.assert_allclose(p["mean2d"][0], [PX + 0.5, PY + 0.5], atol=1e-12)
    np.testing.assert_allclose(p["cov2d"][0], [0.5 / sig, 0.0, 0.5 / sig], rtol=1e-6, atol=1e-12)
    r = orc.render(g, cam, 4)
    assert r["nblend"][PY, PX + 1] == 0 and r["nblend"][PY, PX] == 1
    assert abs(r["margins"][PY, PX + 1, SKIP] - delta) <= 1e-6


@pytest.mark.parametrize("delta", [1e-3, -1e-3, 4e-5, -4e-5])
def test_clamp_margin(orc, delta):
    # o = 0.99 (1 + delta): o e^-sigma / 0.99 sits delta from 1, on either side of the clamp
    r, m = _margins(orc, [0.99 * (1.0 + delta)])
    assert abs(m[CLAMP] - abs(delta)) <= 1e-6
    # the clamp decides alpha: 0.99 above the threshold, o below it
    assert math.isclose(r["O"][PY, PX], 0.99 if delta > 0 else 0.99 * (1 + delta), rel_tol=1e-6)


@pytest.mark.parametrize("delta", [2e-3, -2e-3, 5e-5, -5e-5])
def test_t_floor_margin(orc, delta):
    # alphas 0.9 and 0.95 leave T = 0.005; the third alpha = 1 - 0.02 (1 + delta) (below the
    # clamp) takes T (1 - alpha) to 1e-4 (1 + delta): blended above the floor, stopped below
    r, m = _margins(orc, [0.9, 0.95, 1.0 - 0.02 * (1.0 + delta)])
    assert abs(m[TFLOOR] - abs(delta)) <= 1e-6
    assert r["nblend"][PY, PX] == (3 if delta > 0 else 2)


@pytest.mark.parametrize("delta,K", [(1e-3, 1), (1e-3, 2), (3e-5, 1), (0.25, 4)])
def test_topk_gap_margin(orc, delta, K):
    # w1 = a1, w2 = a2 (1 - a1) = w1 (1 - delta): the relative gap of the two ranked weights
    a1 = 0.4
    a2 = a1 * (1.0 - delta) / (1.0 - a1)
    r, m = _margins(orc, [a1, a2], K=K)
    w = r["w"][PY, PX]
    assert math.isclose(w[0], a1, rel_tol=1e-6) and (K == 1 or math.isclose(w[1], a1 * (1 - delta), rel_tol=1e-6))
    assert abs(m[TOPK] - delta) <= 1e-6


def test_exact_tie_has_zero_topk_margin(orc):
    # two equal weights: Top-K membership is decided by the tie rule alone, gap 0
    a1 = 0.4
    r, m = _margins(orc, [a1, a1 / (1.0 - a1)], K=1)
    assert m[TOPK] <= 1e-6
    assert r["ids"][PY, PX, 0] == 0   # equal weights keep blend order


def test_margins_of_the_hand_derived_pixel(orc):
    """The three-Gaussian golden pixel: its four margins, worked by hand in the fixture."""
    fx = json.load(open(os.path.join(GOLDEN, "three_gaussians_one_pixel.json")))
    cam = identity_camera(fx["W"], fx["H"], f=fx["f"])
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    g = Gaussians(f(fx["means"]), f(fx["log_scales"]), f(fx["quats"]), f(fx["opacity_logits"]), f(fx["rgb"]),
                  f(fx["feat"]))
    r = orc.render(g, cam, fx["K"])
    py, px = fx["pixel"]
    np.testing.assert_allclose(r["margins"][py, px], fx["expect_margins"], rtol=1e-12)
