"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
bench's CPU-baseline leg, never by the product path.  Nothing here is shared with
the HIP library.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so (plain gcc, FP64, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if force or not os.path.exists(LIB_PATH):
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB_OVERRIDE") or LIB_PATH
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        Lg = ctypes.c_long
        L.orc_project.argtypes = [I, P, P, P, P, P, P, I, I, P, P, P, P, P, P, P, P]
        L.orc_render.argtypes = [I, P, P, P, P, P, P, I, I, I, I, P, P, P, P, P, P, P, P, P]
        L.orc_feature.argtypes = [Lg, I, I, P, P, P, P]
        L.orc_prune_stats.argtypes = [I, P, P, P, P, P, P, I, I, I, P, P]
        L.orc_backward.argtypes = [I, P, P, P, P, P, P, I, I, I, I, P, P, P, P, P,
                                   P, P, P, P, P, P, P, P, P, P, P, P, P, I]
        L.orc_vanilla_feature.argtypes = [I, P, P, P, P, P, P, I, I, I, P, P]
        L.orc_set_threads.argtypes = [I]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_bf16_from_f32.argtypes = [Lg, P, P]
        L.orc_bf16_value.argtypes = [ctypes.c_uint16]
        L.orc_bf16_value.restype = ctypes.c_double
        L.orc_e4m3_value.argtypes = [ctypes.c_uint8]
        L.orc_e4m3_value.restype = ctypes.c_double
        L.orc_fp8_quantize.argtypes = [Lg, I, P, P, P]
        L.orc_e4m3_table.argtypes = [P]
        L.orc_topk_select.argtypes = [I, P, I, P]
        L.orc_feature_backward.argtypes = [Lg, I, I, I, P, P, P, P, P, P]
        for f in (L.orc_project, L.orc_render, L.orc_feature, L.orc_backward,
                  L.orc_bf16_from_f32, L.orc_fp8_quantize, L.orc_e4m3_table, L.orc_num_threads,
                  L.orc_topk_select, L.orc_feature_backward, L.orc_prune_stats, L.orc_vanilla_feature):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def cam_array(cam):
    return np.concatenate([np.asarray(cam.Rt, np.float32).reshape(12),
                           np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32)])


def _geom(g):
    return [_f32(g.means), _f32(g.log_scales), _f32(g.quats), _f32(g.opacity_logits), _f32(g.rgb)]


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    """OpenMP threads of later oracle calls (the bench's CPU baseline times 1 and all)."""
    return lib().orc_set_threads(int(n))


def project(g, cam):
    n = g.means.shape[0]
    geo = _geom(g)
    out = dict(valid=np.zeros(n, np.int32), mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)),
               conic=np.zeros((n, 3)), tview=np.zeros((n, 3)), zkey=np.zeros(n, np.float32),
               opacity=np.zeros(n), rect=np.zeros((n, 4), np.int32))
    c = cam_array(cam)
    rc = lib().orc_project(n, *[_p(a) for a in geo], _p(c), cam.W, cam.H,
                           _p(out["valid"]), _p(out["mean2d"]), _p(out["cov2d"]), _p(out["conic"]),
                           _p(out["tview"]), _p(out["zkey"]), _p(out["opacity"]), _p(out["rect"]))
    if rc:
        raise RuntimeError(f"orc_project failed: {rc}")
    return out


def render(g, cam, K, brute=False):
    """Forward render (Eq. 1 + Eq. 2).  Arrays are pixel-major, row-major images."""
    n = g.means.shape[0]
    W, H = cam.W, cam.H
    P = W * H
    out = dict(C=np.zeros((H, W, 3)), D=np.zeros((H, W)), O=np.zeros((H, W)), T=np.zeros((H, W)),
               nblend=np.zeros((H, W), np.int32), ids=np.zeros((H, W, K), np.int32),
               w=np.zeros((H, W, K)), margins=np.zeros((H, W, 4)), sig=np.zeros((H, W), np.uint64))
    geo = _geom(g)
    c = cam_array(cam)
    rc = lib().orc_render(n, *[_p(a) for a in geo], _p(c), W, H, int(K), int(bool(brute)),
                          _p(out["C"]), _p(out["D"]), _p(out["O"]), _p(out["T"]), _p(out["nblend"]),
                          _p(out["ids"]), _p(out["w"]), _p(out["margins"]), _p(out["sig"]))
    if rc:
        raise RuntimeError(f"orc_render failed: {rc}")
    assert P == out["D"].size
    return out


def prune_stats(g, cam, K, count=None, maxw=None):
    """Sec. 3.3 statistics of one view (Eq. 5), accumulated into count (int32 [n],
    Top-K participation) and maxw (float64 [n], the largest blending weight)."""
    n = g.means.shape[0]
    count = np.zeros(n, np.int32) if count is None else count
    maxw = np.zeros(n) if maxw is None else maxw
    geo = _geom(g)
    rc = lib().orc_prune_stats(n, *[_p(a) for a in geo], _p(cam_array(cam)), cam.W, cam.H, int(K), _p(count),
                               _p(maxw))
    if rc:
        raise RuntimeError(f"orc_prune_stats failed: {rc}")
    return count, maxw


def prune_select(count, maxw, count_below, expo, keep_ratio):
    """Survival draw of the consistency pruning (Sec. 3.3, Eq. 6), from its definition:
    candidates are the Gaussians with count < count_below; m = floor(keep_ratio * c)
    (the exact product of the FP32 ratio and c) of the c candidates survive, drawn
    without replacement with weights S = maxw by exponential keys E / S (E the given
    Exp(1) variates; the quotient correctly rounded to FP32, here an FP64 quotient
    rounded once more, which gives the same bits since 53 >= 2*24 + 2; +inf where
    S = 0), the m smallest keys surviving, ties in index order.
    Returns uint8 [n]: 1 keep, 0 remove."""
    count = np.asarray(count)
    n = count.shape[0]
    cand = count < count_below
    c = int(cand.sum())
    m = int((Fraction(float(np.float32(keep_ratio))) * c).__floor__())
    e = np.asarray(expo, np.float32).astype(np.float64)
    s = np.asarray(maxw, np.float32).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = (e / np.where(s > 0, s, 1.0)).astype(np.float32)
    key = np.where(s > 0, q.view(np.uint32), np.uint32(0x7F800000))
    idx = np.nonzero(cand)[0]
    order = idx[np.lexsort((idx, key[idx]))]
    survive = np.ones(n, np.uint8)
    survive[cand] = 0
    survive[order[:m]] = 1
    return survive


def feature(ids, w, feat64):
    """Eq. 3-4 on Top-K ids/weights [..., K] and FP64 features [N, D]."""
    ids = np.ascontiguousarray(ids, np.int32)
    w = _f64(w)
    K = ids.shape[-1]
    n_pix = ids.size // K
    feat64 = _f64(feat64)
    D = feat64.shape[1]
    F = np.zeros(ids.shape[:-1] + (D,))
    rc = lib().orc_feature(n_pix, K, D, _p(ids), _p(w), _p(feat64), _p(F))
    if rc:
        raise RuntimeError(f"orc_feature failed: {rc}")
    return F


def feature_backward(ids, w, feat64, gF):
    """Adjoint of Eq. 3-4 for given Top-K ids/w [..., K], FP64 features [N, D] and
    upstream gF [..., D]: returns (d_feat [N, D], d_w [..., K])."""
    ids = np.ascontiguousarray(ids, np.int32)
    K = ids.shape[-1]
    n_pix = ids.size // K
    feat64 = _f64(feat64)
    n, D = feat64.shape
    w = _f64(w)
    gF = _f64(gF)
    d_feat = np.zeros((n, D))
    d_w = np.zeros(ids.shape)
    rc = lib().orc_feature_backward(n_pix, K, D, n, _p(ids), _p(w), _p(feat64), _p(gF), _p(d_feat), _p(d_w))
    if rc:
        raise RuntimeError(f"orc_feature_backward failed: {rc}")
    return d_feat, d_w


def backward(g, cam, K, feat64, gC=None, gD=None, gO=None, gF=None, vanilla=False):
    """Exact adjoint of render + feature for the given upstream gradients, including
    the camera-pose gradients d_Rt (the 12 entries of [R|t]) and d_pose (rho, phi of
    a left increment exp(xi^) [R|t], Sec. 4.1's rendering-loss pose refinement).
    vanilla=True: gF is the upstream gradient of the vanilla feature render
    (vanilla_feature) instead of the Top-K one."""
    n = g.means.shape[0]
    W, H = cam.W, cam.H
    P = W * H
    feat64 = _f64(feat64)
    D = feat64.shape[1]
    out = dict(d_mean2d=np.zeros((n, 2)), d_conic=np.zeros((n, 3)), d_opac=np.zeros(n),
               d_rgb=np.zeros((n, 3)), d_z=np.zeros(n), d_topkw=np.zeros((H, W, K)),
               d_means=np.zeros((n, 3)), d_log_scales=np.zeros((n, 3)), d_quats=np.zeros((n, 4)),
               d_opacity_logits=np.zeros(n), d_feat=np.zeros((n, D)), d_Rt=np.zeros(12),
               d_pose=np.zeros(6))
    ups = [_f64(None if a is None else np.asarray(a).reshape(-1)) for a in (gC, gD, gO, gF)]
    for a, m in zip(ups, (3, 1, 1, D)):
        assert a is None or a.size == P * m
    geo = _geom(g)
    c = cam_array(cam)
    rc = lib().orc_backward(n, *[_p(a) for a in geo], _p(c), W, H, int(K), D, _p(feat64),
                            *[_p(a) for a in ups],
                            _p(out["d_mean2d"]), _p(out["d_conic"]), _p(out["d_opac"]),
                            _p(out["d_rgb"]), _p(out["d_z"]), _p(out["d_topkw"]),
                            _p(out["d_means"]), _p(out["d_log_scales"]), _p(out["d_quats"]),
                            _p(out["d_opacity_logits"]), _p(out["d_feat"]), _p(out["d_Rt"]),
                            _p(out["d_pose"]), int(bool(vanilla)))
    if rc:
        raise RuntimeError(f"orc_backward failed: {rc}")
    return out


def vanilla_feature(g, cam, feat64):
    """The vanilla alpha-blended feature map (Eq. 1 with the D-channel feature in place
    of the colour, over every blended Gaussian): [H, W, D] in FP64."""
    n = g.means.shape[0]
    feat64 = _f64(feat64)
    D = feat64.shape[1]
    F = np.zeros((cam.H, cam.W, D))
    rc = lib().orc_vanilla_feature(n, *[_p(a) for a in _geom(g)], _p(cam_array(cam)), cam.W, cam.H, D,
                                   _p(feat64), _p(F))
    if rc:
        raise RuntimeError(f"orc_vanilla_feature failed: {rc}")
    return F


def topk_select(w, R):
    """List positions of the R top-ranked weights of a list given in blend order."""
    w = _f64(np.asarray(w, np.float64).ravel())
    rank = np.zeros(max(R, 1), np.int32)
    m = lib().orc_topk_select(w.size, _p(w), int(R), _p(rank))
    if m < 0:
        raise RuntimeError("orc_topk_select failed")
    return rank[:m]


# ------------------------------------------------------------------ quantizers

def bf16_bits(x):
    x = _f32(x)
    out = np.zeros(x.shape, np.uint16)
    lib().orc_bf16_from_f32(x.size, _p(x), _p(out))
    return out


def bf16_to_f64(bits):
    return (np.asarray(bits, np.uint32) << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3_table():
    t = np.zeros(256)
    lib().orc_e4m3_table(_p(t))
    return t


def fp8_quantize(x):
    x = _f32(x)
    n, D = x.shape
    codes = np.zeros((n, D), np.uint8)
    scale = np.zeros(n, np.float32)
    lib().orc_fp8_quantize(n, D, _p(x), _p(codes), _p(scale))
    return codes, scale


def fp8_dequant(codes, scale):
    return e4m3_table()[codes] * np.asarray(scale, np.float64)[:, None]


# Decision-margin threshold of the parity tests: 4x the largest FP32 relative error
# of a selected blending weight measured at 640x480 (5.2e-5).
FLAG_EPS = 2.5e-4


def flagged(margins, eps_skip=FLAG_EPS, eps_clamp=FLAG_EPS, eps_T=FLAG_EPS, eps_topk=FLAG_EPS):
    """Pixels whose alpha-skip, alpha-clamp, T-floor or Top-K rank decision came within
    the given relative distance of its threshold."""
    m = np.asarray(margins)
    return ((m[..., 0] < eps_skip) | (m[..., 1] < eps_clamp) | (m[..., 2] < eps_T) |
            (m[..., 3] < eps_topk))


def blend_flagged(margins, eps=FLAG_EPS):
    """Pixels where the blend itself (skip, clamp or T-floor) came within eps of a
    threshold, so C, D and O may legitimately differ by one Gaussian's share."""
    m = np.asarray(margins)
    return (m[..., 0] < eps) | (m[..., 1] < eps) | (m[..., 2] < eps)
