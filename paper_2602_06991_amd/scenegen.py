"""Seeded synthetic room scenes: the only module shared by the oracle tests and the
HIP path.  It draws inputs and holds none of the renderer's arithmetic.

A scene stands in for the paper's RGB-D sequences (Replica, TUM-RGBD; Sec. 4.1),
which are not available here.  It is an axis-aligned 6 x 4 x 3 m room (z up)
whose six faces, plus the six faces of every object box inside it, carry surface
Gaussians.  Each face of the room and each object box is its own language-feature
cluster, matching the paper's use of 512-D LSeg features (Sec. 4.1) by shape only.

Every array is float32, C-contiguous.  The random streams are numpy PCG64
sub-streams spawned from one seed in a fixed order, so a (config, seed) pair
always produces the same bytes; `scene_digest` hashes them.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import hashlib
import math
import os

import numpy as np

ROOM_LO = np.array([-3.0, -2.0, -1.5])
ROOM_HI = np.array([3.0, 2.0, 1.5])

# Workloads: image size, views, Gaussian count, feature width, K, objects.
CONFIGS = {
    0: dict(W=160, H=120, views=1, N=10_000, D=512, K=(4,), objects=0,
            spare_clusters=1, cams="centre"),
    1: dict(W=640, H=480, views=1, N=200_000, D=512, K=(4,), objects=20,
            spare_clusters=0, cams="centre"),
    2: dict(W=1200, H=680, views=1, N=500_000, D=512, K=(1, 4, 8), objects=60,
            spare_clusters=0, cams="centre"),
    3: dict(W=640, H=480, views=8, N=1_000_000, D=512, K=(4,), objects=100,
            spare_clusters=0, cams="random"),
    4: dict(W=1200, H=680, views=4, N=3_000_000, D=768, K=(8,), objects=300,
            spare_clusters=0, cams="random"),
}

_STREAMS = ("room", "objects", "surface", "scales", "rotations", "opacity",
            "colour", "clusters", "features", "cameras", "perturbation")

_CHUNK = 1 << 16   # rows per independently seeded block of feature noise


def _chunked_rows(rng, N, fill):
    """Calls fill(s, e, block_rng) for row blocks [s, e) of _CHUNK rows, each block with
    its own generator spawned from `rng` in block order (so the bytes do not depend on
    how many threads run the blocks); blocks run on a thread pool."""
    starts = list(range(0, N, _CHUNK))
    seeds = np.random.SeedSequence(int(rng.integers(0, 2**63))).spawn(len(starts))
    jobs = [(s, min(N, s + _CHUNK), np.random.Generator(np.random.PCG64(q))) for s, q in zip(starts, seeds)]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        list(ex.map(lambda j: fill(*j), jobs))


@dataclasses.dataclass
class Camera:
    """Pinhole camera. Rt is the 3x4 world->camera [R|t], row-major, OpenCV axes
    (x right, y down, z forward)."""
    Rt: np.ndarray   # float32[12]
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int


@dataclasses.dataclass
class Gaussians:
    means: np.ndarray           # f32[N,3]
    log_scales: np.ndarray      # f32[N,3]
    quats: np.ndarray           # f32[N,4]  (w, x, y, z), not necessarily unit
    opacity_logits: np.ndarray  # f32[N]
    rgb: np.ndarray             # f32[N,3]
    feat: np.ndarray            # f32[N,D]

    @property
    def n(self):
        return self.means.shape[0]

    @property
    def d(self):
        return self.feat.shape[1]

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits,
                self.rgb, self.feat)


@dataclasses.dataclass
class Scene:
    config: dict
    seed: int
    gaussians: Gaussians
    target: Gaussians           # noise-perturbed copy (loss target source)
    cameras: list
    cluster: np.ndarray         # i32[N] cluster index of every Gaussian


def _faces_of_box(lo, hi):
    """Six faces of an axis-aligned box as (origin, u, v) with area |u|*|v|."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    ext = hi - lo
    faces = []
    for axis in range(3):
        a, b = [i for i in range(3) if i != axis]
        u = np.zeros(3)
        v = np.zeros(3)
        u[a] = ext[a]
        v[b] = ext[b]
        for side in (lo[axis], hi[axis]):
            o = lo.copy()
            o[axis] = side
            faces.append((o, u.copy(), v.copy()))
    return faces


def _largest_remainder(total, weights):
    w = np.asarray(weights, float)
    exact = total * w / w.sum()
    base = np.floor(exact).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return base


def _point_box_distance(p, lo, hi):
    d = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return float(np.sqrt((d * d).sum()))


def look_camera(pos, yaw, pitch, W, H):
    """World->camera [R|t] for a camera at `pos` looking along yaw/pitch (z up)."""
    f = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch),
                  math.sin(pitch)])
    r = np.array([f[1], -f[0], 0.0])
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    R = np.stack([r, dn, f])
    t = -R @ np.asarray(pos, float)
    Rt = np.concatenate([R, t[:, None]], axis=1).astype(np.float32).reshape(12)
    return Camera(Rt=Rt, fx=float(np.float32(0.8 * W)), fy=float(np.float32(0.8 * W)),
                  cx=float(W) / 2.0, cy=float(H) / 2.0, W=int(W), H=int(H))


def _normalize_rows(x):
    n = np.sqrt(np.einsum("ij,ij->i", x, x, dtype=np.float32)).astype(np.float32)
    n[n == 0] = 1.0
    return x / n[:, None]


def make_scene(config=0, seed=None, **overrides) -> Scene:
    """Build the seeded scene of workload `config` (0..4); `overrides` replace any
    field of the workload (e.g. N=2000, W=64, H=48 for small tests)."""
    cfg = dict(CONFIGS[config])
    cfg.update(overrides)
    cfg["index"] = config
    if seed is None:
        seed = 1000 + config
    streams = dict(zip(_STREAMS, [np.random.Generator(np.random.PCG64(s))
                                  for s in np.random.SeedSequence(seed).spawn(len(_STREAMS))]))
    W, H, N, D = cfg["W"], cfg["H"], cfg["N"], cfg["D"]

    # Camera positions first: object boxes keep clear of them.
    rc = streams["cameras"]
    cam_pose = []
    for _ in range(cfg["views"]):
        if cfg["cams"] == "centre":
            cam_pose.append((np.zeros(3), rc.uniform(0.0, 2 * math.pi), 0.0))
        else:
            pos = rc.uniform(ROOM_LO + 0.5, ROOM_HI - 0.5)
            yaw = rc.uniform(0.0, 2 * math.pi)
            pitch = math.radians(rc.uniform(-15.0, 15.0))
            cam_pose.append((pos, yaw, pitch))

    ro = streams["objects"]
    boxes = []
    tries = 0
    while len(boxes) < cfg["objects"]:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place object boxes clear of the cameras")
        size = ro.uniform(0.2, 1.0, size=3)
        half = size / 2
        c = ro.uniform(ROOM_LO + half, ROOM_HI - half)
        lo, hi = c - half, c + half
        if any(_point_box_distance(p, lo, hi) < 0.3 for p, _, _ in cam_pose):
            continue
        boxes.append((lo, hi))

    faces = []      # (origin, u, v, cluster)
    for o, u, v in _faces_of_box(ROOM_LO, ROOM_HI):
        faces.append((o, u, v, len(faces)))
    n_room_faces = len(faces)
    for bi, (lo, hi) in enumerate(boxes):
        for o, u, v in _faces_of_box(lo, hi):
            faces.append((o, u, v, n_room_faces + bi))
    n_clusters = n_room_faces + len(boxes) + cfg["spare_clusters"]
    areas = [np.linalg.norm(u) * np.linalg.norm(v) for _, u, v, _ in faces]
    counts = _largest_remainder(N, areas)

    rs = streams["surface"]
    means = np.empty((N, 3), np.float64)
    cluster = np.empty(N, np.int32)
    at = 0
    for (o, u, v, cl), c in zip(faces, counts):
        ab = rs.random((int(c), 2))
        means[at:at + c] = o + ab[:, :1] * u + ab[:, 1:] * v
        cluster[at:at + c] = cl
        at += c
    means = means.astype(np.float32)

    eps = streams["scales"].standard_normal((N, 3))
    log_scales = np.log(np.clip(np.exp(math.log(0.02) + 0.5 * eps), 0.002, 0.2)).astype(np.float32)
    q = streams["rotations"].standard_normal((N, 4))
    quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    opacity_logits = (1.0 + streams["opacity"].standard_normal(N)).astype(np.float32)
    rgb = streams["colour"].random((N, 3)).astype(np.float32)

    centres = _normalize_rows(streams["clusters"].standard_normal((n_clusters, D), dtype=np.float32))
    feat = np.empty((N, D), np.float32)

    def fill_feat(s, e, r):
        noise = r.standard_normal((e - s, D), dtype=np.float32)
        feat[s:e] = _normalize_rows(centres[cluster[s:e]] + np.float32(0.1) * noise)

    _chunked_rows(streams["features"], N, fill_feat)

    g = Gaussians(means, log_scales, quats, opacity_logits, rgb, feat)
    target = perturb(g, streams["perturbation"])
    cams = [look_camera(p, y, pi, W, H) for p, y, pi in cam_pose]
    return Scene(config=cfg, seed=seed, gaussians=g, target=target, cameras=cams,
                 cluster=cluster)


def perturb(g: Gaussians, rng) -> Gaussians:
    """Noise-perturbed copy of a scene (the loss target's source)."""
    N, D = g.feat.shape
    means = (g.means + rng.normal(0, 0.005, (N, 3))).astype(np.float32)
    log_scales = (g.log_scales + rng.normal(0, 0.05, (N, 3))).astype(np.float32)
    q = g.quats + rng.normal(0, 0.02, (N, 4))
    quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    opacity_logits = (g.opacity_logits + rng.normal(0, 0.1, N)).astype(np.float32)
    rgb = np.clip(g.rgb + rng.normal(0, 0.02, (N, 3)), 0.0, 1.0).astype(np.float32)
    feat = np.empty_like(g.feat)
    scale = np.float32(0.1 / math.sqrt(D))

    def fill_feat(s, e, r):
        feat[s:e] = _normalize_rows(g.feat[s:e] + scale * r.standard_normal((e - s, D), dtype=np.float32))

    _chunked_rows(rng, N, fill_feat)
    return Gaussians(means, log_scales, quats, opacity_logits, rgb, feat)


def scene_digest(scene: Scene) -> str:
    h = hashlib.sha256()
    for g in (scene.gaussians, scene.target):
        for a in g.arrays():
            h.update(np.ascontiguousarray(a).tobytes())
    for c in scene.cameras:
        h.update(c.Rt.tobytes())
        h.update(np.array([c.fx, c.fy, c.cx, c.cy, c.W, c.H], np.float64).tobytes())
    return h.hexdigest()


def random_upstream(seed, n_pix, d, map_dtype=np.float32):
    """Seeded upstream gradients (dL/dC, dL/dD, dL/dO, dL/dF) of a random linear
    functional of the rendered outputs."""
    r = np.random.Generator(np.random.PCG64(seed))
    gC = r.standard_normal((n_pix, 3)).astype(np.float32)
    gD = r.standard_normal(n_pix).astype(np.float32)
    gO = r.standard_normal(n_pix).astype(np.float32)
    gF = r.standard_normal((n_pix, d), dtype=np.float32)
    return gC, gD, gO, gF


def identity_camera(W, H, f=None):
    """Camera whose frame is the world frame (looking along +z, y down)."""
    f = float(np.float32(0.8 * W if f is None else f))
    Rt = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    return Camera(Rt=Rt, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, W=int(W), H=int(H))


def make_tiny(seed, n=16, W=24, H=20, D=8, scale=(-3.0, 0.6), depth=(1.0, 3.0), opl=(0.5, 1.0),
              spread=(-0.1, 1.1)):
    """Small random scene in front of an identity camera, for brute-force and
    finite-difference checks.  Gaussians land inside the view frustum."""
    r = np.random.Generator(np.random.PCG64(seed))
    cam = identity_camera(W, H)
    z = r.uniform(depth[0], depth[1], n)
    u = r.uniform(spread[0] * W, spread[1] * W, n)
    v = r.uniform(spread[0] * H, spread[1] * H, n)
    means = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], 1).astype(np.float32)
    log_scales = (scale[0] + scale[1] * r.standard_normal((n, 3))).astype(np.float32)
    q = r.standard_normal((n, 4))
    quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    opacity_logits = (opl[0] + opl[1] * r.standard_normal(n)).astype(np.float32)
    rgb = r.random((n, 3)).astype(np.float32)
    feat = _normalize_rows(r.standard_normal((n, D)).astype(np.float32))
    return Gaussians(means, log_scales, quats, opacity_logits, rgb, feat), cam
