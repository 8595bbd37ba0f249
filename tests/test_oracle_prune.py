"""Pins of the oracle's pruning statistics (Sec. 3.3, Eq. 5): Top-K participation
counts and the largest blending weight S_g of every Gaussian."""
import math

import numpy as np
import pytest

from paper_2602_06991_amd.scenegen import Gaussians, identity_camera, make_scene, make_tiny


def _gs(means, log_scales, quats, opls, rgbs, feats):
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    return Gaussians(f(means), f(log_scales), f(quats), f(opls), f(rgbs), f(feats))


@pytest.mark.parametrize("opl", [0.3, 2.0, 6.0])
def test_single_gaussian_peak_weight(orc, opl):
    # mean2D on the centre of pixel (8, 8): there sigma = 0, so the largest weight the
    # Gaussian reaches is its clamped opacity min(0.99, o); it is counted at every
    # pixel where it is blended (the only candidate, so always in the Top-K)
    cam = identity_camera(16, 16, f=16.0)
    z = 2.0
    g = _gs([[0.5 / 16 * z, 0.5 / 16 * z, z]], [np.log([0.08, 0.05, 0.05])], [[1, 0, 0, 0]], [opl],
            [[1, 1, 1]], [[1, 0]])
    np.testing.assert_allclose(orc.project(g, cam)["mean2d"], [[8.5, 8.5]], atol=1e-12)
    o = 1.0 / (1.0 + math.exp(-float(np.float32(opl))))
    count, maxw = orc.prune_stats(g, cam, 4)
    assert maxw[0] == pytest.approx(min(0.99, o), rel=1e-15)
    r = orc.render(g, cam, 4)
    assert count[0] == int((r["O"] > 0).sum()) > 1


@pytest.mark.parametrize("K", [1, 4, 8])
def test_counts_are_topk_memberships(orc, K):
    sc = make_scene(0)
    g, cam = sc.gaussians, sc.cameras[0]
    count, _ = orc.prune_stats(g, cam, K)
    r = orc.render(g, cam, K)
    ids = r["ids"].reshape(-1)
    assert count.sum() == int((ids >= 0).sum())
    np.testing.assert_array_equal(count, np.bincount(ids[ids >= 0], minlength=g.n))
    assert count.max() <= cam.W * cam.H


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_peak_weight_is_the_largest_blended_weight(orc, seed):
    # with K above every pixel's blended count the Top-K lists hold every blended
    # Gaussian and its weight, so S_g is the largest listed weight of g
    g, cam = make_tiny(seed, n=[30, 50, 64][seed], W=40, H=32, scale=(-2.3, 0.7))
    r = orc.render(g, cam, 63)
    assert r["nblend"].max() < 63
    _, maxw = orc.prune_stats(g, cam, 4)
    ids, w = r["ids"].reshape(-1), r["w"].reshape(-1)
    want = np.zeros(g.n)
    np.maximum.at(want, ids[ids >= 0], w[ids >= 0])
    np.testing.assert_array_equal(maxw, want)
    assert (want > 0).sum() > g.n // 2


def test_statistics_accumulate_over_views(orc):
    sc = make_scene(3, N=20000, W=96, H=64)
    g = sc.gaussians
    c1, m1 = orc.prune_stats(g, sc.cameras[0], 4)
    c2, m2 = orc.prune_stats(g, sc.cameras[1], 4)
    c, m = orc.prune_stats(g, sc.cameras[0], 4)
    orc.prune_stats(g, sc.cameras[1], 4, c, m)
    np.testing.assert_array_equal(c, c1 + c2)
    np.testing.assert_array_equal(m, np.maximum(m1, m2))
    assert np.all((m > 0) >= (c > 0))      # a Top-K member is blended somewhere


def test_first_survivor_follows_eq6(orc):
    # one survivor out of four candidates: over many draws candidate i is picked with
    # probability S_i / sum S (Eq. 6); two non-candidates always survive
    S = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 0.5], np.float32)
    count = np.array([0, 1, 0, 2, 9, 9], np.int32)
    rng = np.random.default_rng(42)
    trials = 40000
    hits = np.zeros(6)
    for _ in range(trials):
        s = orc.prune_select(count, S, 3, rng.exponential(size=6).astype(np.float32), 0.25)
        assert s[4] == 1 and s[5] == 1 and s[:4].sum() == 1
        hits += s
    p = S[:4] / S[:4].sum()
    sd = np.sqrt(p * (1 - p) / trials)
    assert np.all(np.abs(hits[:4] / trials - p) <= 4 * sd), (hits[:4] / trials, p)


def test_survivors_hold_the_smallest_keys(orc):
    rng = np.random.default_rng(7)
    n = 5000
    count = rng.integers(0, 6, n).astype(np.int32)
    S = rng.choice([0.0, 0.25, 0.5, 1.0], n).astype(np.float32)      # zeros and many ties
    E = rng.choice([0.5, 1.0, 2.0], n).astype(np.float32)
    for ratio in (0.0, 0.3, 0.5, 1.0):
        s = orc.prune_select(count, S, 3, E, ratio)
        cand = count < 3
        assert np.all(s[~cand] == 1)
        assert s[cand].sum() == int(np.floor(np.float64(np.float32(ratio)) * cand.sum()))
        key = np.where(S > 0, E / np.where(S > 0, S, 1), np.inf)
        kept, gone = cand & (s == 1), cand & (s == 0)
        if kept.any() and gone.any():
            assert key[kept].max() <= key[gone].min()
            kt = key[kept].max()
            # at the threshold key the kept ones come first in index order
            at = np.nonzero(cand & (key == kt))[0]
            assert np.all(np.diff(s[at].astype(int)) <= 0)
        # a zero-importance candidate goes before any positive one
        if gone.any() and (S[kept] == 0).any():
            assert np.all(S[gone] == 0)


def test_survivor_count_rounds_down(orc):
    # 5 candidates at ratio 0.75: 3.75 -> 3 survivors (the share is rounded down)
    count = np.array([0, 0, 0, 0, 0, 7, 7], np.int32)
    S = np.ones(7, np.float32)
    E = np.arange(1, 8, dtype=np.float32)
    s = orc.prune_select(count, S, 1, E, 0.75)
    np.testing.assert_array_equal(s, [1, 1, 1, 0, 0, 1, 1])


def test_survivor_count_uses_the_fp32_ratio_exactly(orc):
    # the ratio is the FP32 value the caller passes: FP32 0.7 is 0.699999988..., so 10
    # candidates keep floor(6.99999988) = 6, not 7; FP32 0.3 is 0.300000012..., so 10
    # keep 3
    count = np.zeros(10, np.int32)
    S = np.ones(10, np.float32)
    E = np.arange(1, 11, dtype=np.float32)
    assert orc.prune_select(count, S, 1, E, 0.7).sum() == 6
    assert orc.prune_select(count, S, 1, E, 0.3).sum() == 3
    assert orc.prune_select(count, S, 1, E, 1.0).sum() == 10
