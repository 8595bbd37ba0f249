"""Benchmark of the Top-K renderer's forward + backward step on one MI355X.

Workload (default): 1200x680 px single view, 500k Gaussians on a seeded synthetic
room with 60 object boxes, D = 512 language features, K = 4, with the feature
table stored in BF16 (FP32 accumulation) and, for comparison, the plain FP32 form.

One step = one pass of the whole hot path over one frame:
  quantize the FP32 master features to the storage format (BF16 form only),
  project -> bin + sort -> blend with Top-K,
  L1 loss gradients of colour and depth against a target frame,
  zero the gradient buffers,
  feature render + its adjoint under the feature L1 loss, in one pass that stores the
  map and differentiates it (--feature-path separate: the render, then the adjoint
  with the loss gradient formed inside it, as two launches),
  -> blend adjoint -> projection adjoint.
All inputs are resident in HBM before timing starts.

Prints one JSON line (metric, value = BF16 fwd+bwd ms per frame, roofline of the
dominant feature kernel from live HIP-event timings, and the FP64 oracle's CPU time
for one full frame of the same workload).  Per form it also reports: the forward
alone, the render and the L1 adjoint as two separate launches, a geometry-only step
(the hybrid schedule's geometry iterations: no feature passes), the pruning
statistics and the survival draw; and once the achievable copy bandwidth.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--K", type=int, default=4)
    ap.add_argument("--no-sweep", dest="sweep", action="store_false", help="skip the K = 1 and 8 steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="bf16,f32")
    ap.add_argument("--feature-path", choices=("fused", "separate"), default="fused",
                    help="feature render and adjoint in one launch (fused) or two")
    ap.add_argument("--multi-view", default="3,4",
                    help="also time the batched multi-view steps of these workloads ('' for none): "
                         "3 = 8 x 640x480 / 1M / BF16 / K = 4, 4 = 4 x 1200x680 / 3M / D = 768 / FP8 / K = 8")
    ap.add_argument("--quantize", choices=("rows", "dense"), default="rows",
                    help="refresh the BF16/FP8 store in the rows the step's Top-K lists name (rows), "
                         "or convert the whole FP32 table every step (dense)")
    ap.add_argument("--no-vanilla", dest="vanilla", action="store_false",
                    help="skip the vanilla (alpha-blended, every Gaussian) feature step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy three times (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


# The storage form (BF16 or FP8) is read only by the feature kernels, and the Top-K
# feature kernels read only the rows named in the step's Top-K lists, which the step
# stamps for the sparse gradient clearing anyway: so a Top-K step refreshes just those
# rows of the store from the FP32 master table, after the blend (for every row the step
# reads, the same bits as converting the whole table).  The vanilla render reads every
# blended Gaussian's row and converts the whole table, as does `--quantize dense`.
# The clearing of the previous step's gradient rows, and a whole-table conversion,
# depend on nothing the projection, binning and blend compute, so the timed steps run
# them on a second stream (default priority) beside those phases; the main stream
# waits for them after the blend, before it marks rows or anything reads the store.
# The per-phase pass (events after every phase) runs everything in order on one stream.
def _side_init(st, torch, form, n, d, dev, sparse, dense_quantize):
    st.sparse = sparse
    st.dense_q = dense_quantize or not sparse
    st.side = torch.cuda.Stream()
    st.out = None
    if form in ("bf16", "fp8"):
        st.out = (torch.empty(n, d, dtype=torch.bfloat16 if form == "bf16" else torch.uint8, device=dev),
                  torch.empty(n, device=dev) if form == "fp8" else None)


def _side_begin(st):
    """Issues the side work (the previous step's row clearing, a whole-table
    conversion); returns the event the main stream waits for (None in the per-phase
    pass, which runs the work in order)."""
    t, r, P = st.t, st.render, st.P
    def work():
        if st.sparse:
            st.rows.clear()
            st._mark("clear_rows")
        if st.dense_q and st.out is not None:
            r.quantize(P["feat"], st.form, out=st.out)
            st._mark("quantize")
    if st.events is not None:
        work()
        return None
    ready = t.cuda.Event()
    ready.record()                       # the previous step's reads of the store are queued before this
    st.side.wait_event(ready)
    with t.cuda.stream(st.side):
        work()
        done = t.cuda.Event()
        done.record()
    return done


def _side_join(st, done, topk_ids):
    """After the blend: the main stream waits for the side work, stamps the step's Top-K
    rows and refreshes them in the store; returns (store, scale)."""
    if done is not None:
        st.t.cuda.current_stream().wait_event(done)
    if st.sparse:
        st.rows.mark(topk_ids)
        st._mark("mark_rows")
    if st.out is None:
        return st.P["feat"], None
    if not st.dense_q:
        st.rows.quantize(st.P["feat"], st.form, st.out)
        st._mark("quantize")
    return st.out


def _grad_slab(torch, shapes, dev):
    """One allocation holding a step's gradient buffers (each a view at a 256-byte
    offset), so that one fill clears them all."""
    sizes = [int(np.prod(s)) for s in shapes.values()]
    offs, at = [], 0
    for z in sizes:
        offs.append(at)
        at += (z + 63) // 64 * 64
    flat = torch.zeros(at, device=dev)
    return flat, {k: flat[o:o + z].view(*s) for (k, s), o, z in zip(shapes.items(), offs, sizes)}


def _geometry_grads(torch, n, rec, dev):
    """Screen-space gradients of `rec` records (rgb per Gaussian) and parameter
    gradients of n Gaussians, in one slab."""
    flat, b = _grad_slab(torch, dict(mean2d=(rec, 2), conic=(rec, 3), opacity=(rec,), rgb=(n, 3), depth=(rec,),
                                     means=(n, 3), log_scales=(n, 3), quats=(n, 4), opacity_logits=(n,)), dev)
    sg = {k: b[k] for k in ("mean2d", "conic", "opacity", "rgb", "depth")}
    pg = {k: b[k] for k in ("means", "log_scales", "quats", "opacity_logits")}
    return flat, sg, pg


class Step:
    """All buffers of one frame's forward + backward, reused across steps."""

    def __init__(self, torch, render, lgs, scene_dev, target, cam, K, form, fused=True, geometry_only=False,
                 vanilla=False, dense_quantize=False):
        self.t, self.render, self.lgs = torch, render, lgs
        self.fused = fused
        self.vanilla = vanilla   # the dense alpha-blended feature field in place of Top-K (Tab. 4's comparison)
        self.geometry_only = geometry_only   # the hybrid schedule's geometry iterations (Sec. 3.4)
        self.P, self.target, self.cam, self.K, self.form = scene_dev, target, cam, K, form
        self.map = "f32" if form == "f32" else "bf16"
        self.binner = render.Binner(sync=False)   # no host round trip inside the step
        n, d = scene_dev["feat"].shape
        self.n, self.d = n, d
        dev = "cuda"
        self.dfeat = torch.zeros(n, d, device=dev)
        # the Top-K adjoint writes only the rows of the step's Top-K lists: the table is
        # cleared by zeroing the rows the previous step named (the vanilla adjoint writes
        # every blended Gaussian's row and clears the whole table)
        self.rows = None if vanilla else render.SparseGradRows(self.dfeat)
        self.gflat, self.sg, self.pg = _geometry_grads(torch, n, n, dev)
        self.npix = cam.width * cam.height
        self.events = None
        self.order = self.border = None   # the blend's and its adjoint's dispatch orders
        self.kmarks = None
        _side_init(self, torch, None if geometry_only else form, n, d, dev, not geometry_only and not vanilla,
                   dense_quantize)

    def _mark(self, name):
        if self.events is not None:
            e = self.t.cuda.Event(enable_timing=True)
            e.record()
            self.events.append((name, e))

    def __call__(self):
        r, P, c = self.render, self.P, self.cam
        self._mark("start")
        joined = None if self.geometry_only else _side_begin(self)
        proj = r.project(c, P)
        self._mark("project_fwd")
        ids, ranges, m = self.binner(c, self.n, proj["depth"], proj["tile_rect"], proj["tiles_touched"])
        self._mark("bin_sort")
        self.order = order = r.tile_order(c, ranges, out=self.order)
        self._mark("tile_order")
        fw = r.rasterize(c, self.K, proj, P["rgb"], ids, ranges, order)
        self._mark("rasterize_topk_fwd")
        store, scale = (None, None) if self.geometry_only else _side_join(self, joined, fw["ids"])
        F = None
        if self.vanilla:
            F = r.feature_vanilla_fwd(c, proj, ids, ranges, fw, store, scale, self.form)
            self._mark("feature_render_fwd")
        elif not self.fused and not self.geometry_only:
            F = r.feature_fwd(fw["ids"], fw["w"], store, scale, self.form, self.map)
            self._mark("feature_render_fwd")
        tC, tD, tF = self.target
        gC = r.l1_grad(fw["C"], tC, 1.0 / (3 * self.npix))
        gD = r.l1_grad(fw["D"], tD, 1.0 / self.npix)
        self._mark("l1_grad")
        if self.vanilla:
            self.dfeat.zero_()
        self.gflat.zero_()
        self._mark("zero_grads")
        # Eq. 9's L1 feature loss: its gradient is formed inside the feature adjoint
        if self.kmarks is not None:
            ka = self.t.cuda.Event(enable_timing=True)
            ka.record()
        fscale = 1.0 / (self.npix * self.d)
        if self.geometry_only:
            dtw = None
        elif self.vanilla:
            dtw = None
            r.feature_vanilla_bwd(c, proj, ids, ranges, fw, store, scale, self.form, r.l1_grad(F, tF, fscale),
                                  self.dfeat, self.sg)
        elif self.fused:
            F, dtw = r.feature_fwd_bwd_l1(fw["ids"], fw["w"], store, scale, self.form, self.map, tF, fscale,
                                          self.dfeat)
        else:
            dtw = r.feature_bwd_l1(fw["ids"], fw["w"], store, scale, self.form, self.map, tF, fscale,
                                   self.dfeat)
        if self.kmarks is not None:
            kb = self.t.cuda.Event(enable_timing=True)
            kb.record()
            self.kmarks.append((ka, kb))
        if not self.geometry_only:
            self._mark("feature_render_fwd_bwd" if self.fused and not self.vanilla else "feature_render_bwd")
        self.border = border = r.tile_order(c, ranges, n_contrib=fw["n_contrib"], out=self.border)
        self._mark("tile_order_bwd")
        r.rasterize_bwd(c, self.K, proj, P["rgb"], ids, ranges, fw, gC, gD, None, dtw, self.sg, border)
        self._mark("rasterize_topk_bwd")
        r.project_bwd(c, P, self.sg, self.pg)
        self._mark("project_bwd")
        self.last = dict(fw=fw, pairs=m, F=F, store=store, scale=scale, proj=proj, ids=ids, ranges=ranges)


class StepViews:
    """One mapping step over several keyframes (Sec. 3.4), every geometry call batched
    over the views (the view folded into the binning key) and the feature render +
    adjoint over the stacked views in one launch; the step ends with the parameter
    gradients and every view's camera-pose gradient (Sec. 4.1's pose refinement)."""

    def __init__(self, torch, render, lgs, scene_dev, target, cams, K, form, dense_quantize=False):
        self.t, self.render, self.lgs = torch, render, lgs
        self.P, self.target, self.cams, self.K, self.form = scene_dev, target, cams, K, form
        self.V = len(cams)
        self.map = "f32" if form == "f32" else "bf16"
        self.binner = render.Binner(sync=False)
        n, d = scene_dev["feat"].shape
        self.n, self.d = n, d
        dev = "cuda"
        self.dfeat = torch.zeros(n, d, device=dev)
        self.rows = render.SparseGradRows(self.dfeat)   # cleared row by row, as in Step
        self.gflat, self.sg, self.pg = _geometry_grads(torch, n, n * self.V, dev)
        self.dpose = torch.empty(6 * self.V, device=dev)
        self.npix = cams[0].width * cams[0].height * self.V
        self.events = None
        self.order = self.border = None
        self.kmarks = None
        _side_init(self, torch, form, n, d, dev, True, dense_quantize)

    _mark = Step._mark

    def __call__(self):
        r, P, c, V, n = self.render, self.P, self.cams, self.V, self.n
        self._mark("start")
        joined = _side_begin(self)
        proj = r.project_views(c, P)
        self._mark("project_fwd")
        ids, ranges, m = self.binner(c, n, proj["depth"], proj["tile_rect"], proj["tiles_touched"], views=V)
        self._mark("bin_sort")
        self.order = order = r.tile_order(c, ranges, views=V, out=self.order)
        self._mark("tile_order")
        fw = r.rasterize_views(c, self.K, n, proj, P["rgb"], ids, ranges, order)
        self._mark("rasterize_topk_fwd")
        store, scale = _side_join(self, joined, fw["ids"])
        tC, tD, tF = self.target
        gC = r.l1_grad(fw["C"], tC, 1.0 / (3 * self.npix))
        gD = r.l1_grad(fw["D"], tD, 1.0 / self.npix)
        self._mark("l1_grad")
        self.gflat.zero_()
        self.dpose.zero_()
        self._mark("zero_grads")
        if self.kmarks is not None:
            ka = self.t.cuda.Event(enable_timing=True)
            ka.record()
        F, dtw = r.feature_fwd_bwd_l1(fw["ids"], fw["w"], store, scale, self.form, self.map, tF,
                                      1.0 / (self.npix * self.d), self.dfeat, views=V)
        if self.kmarks is not None:
            kb = self.t.cuda.Event(enable_timing=True)
            kb.record()
            self.kmarks.append((ka, kb))
        self._mark("feature_render_fwd_bwd")
        self.border = border = r.tile_order(c, ranges, views=V, n_contrib=fw["n_contrib"], out=self.border)
        self._mark("tile_order_bwd")
        r.rasterize_bwd_views(c, self.K, n, proj, P["rgb"], ids, ranges, fw, gC, gD, None, dtw, self.sg, border)
        self._mark("rasterize_topk_bwd")
        r.project_bwd_views(c, P, self.sg, self.pg, self.dpose)
        self._mark("project_bwd")
        self.last = dict(fw=fw, F=F, store=store, scale=scale)


def multi_view(torch, render, lgs, config, steps, warmup, dense_quantize=False):
    """The batched mapping step of workload `config` for each of its storage forms:
    ms per step, the feature kernel's HBM roofline, and each form's feature-map error
    against the FP32 form's map of the same step."""
    from paper_2602_06991_amd.scenegen import make_scene
    t_gen = time.perf_counter()
    scene = make_scene(config)
    cfg = scene.config
    print(f"# scene {cfg['views']} x {cfg['W']}x{cfg['H']} N={cfg['N']} D={cfg['D']} generated in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    names = ("means", "log_scales", "quats", "opacity_logits", "rgb", "feat")
    P = {k: f(v) for k, v in zip(names, scene.gaussians.arrays())}
    PT = {k: f(v) for k, v in zip(names, scene.target.arrays())}
    cams = lgs.camera_array([lgs.make_camera(c) for c in scene.cameras])
    del scene
    K = cfg["K"][0]
    V, n, D = len(cams), cfg["N"], cfg["D"]
    forms = ("fp8", "bf16", "f32") if config == 4 else ("bf16", "f32")
    out, maps = {}, {}
    # target frames: the perturbed scene rendered by the same path, outside timing
    tproj = render.project_views(cams, PT)
    tids, tranges, _ = render.Binner()(cams, n, tproj["depth"], tproj["tile_rect"], tproj["tiles_touched"], views=V)
    tfw = render.rasterize_views(cams, K, n, tproj, PT["rgb"], tids, tranges)
    del tproj, tids, tranges
    for form in forms:
        mp = "f32" if form == "f32" else "bf16"
        tstore, tscale = render.quantize(PT["feat"], form)
        tF = render.feature_fwd(tfw["ids"], tfw["w"], tstore, tscale, form, mp, views=V)
        del tstore, tscale
        step = StepViews(torch, render, lgs, P, (tfw["C"], tfw["D"], tF), cams, K, form, dense_quantize)
        ms, phases, kern_ms, dist = time_steps(torch, step, steps, warmup)
        pairs, fitted = step.binner.count()
        assert fitted, "pair buffer overflowed during timing"
        fw = step.last["fw"]
        U = render.union_count(fw["ids"], n)
        s_map = 4 if mp == "f32" else 2
        s_f = {"f32": 4, "bf16": 2, "fp8": 1}[form]
        _, _, both = feature_bytes(step.npix, K, D, U, s_map, s_f, form == "fp8")
        gbs = both / (kern_ms * 1e-3) / 1e9
        maps[form] = step.last["F"]
        out[form] = dict(ms_per_step=round(ms, 4), step_ms_percentiles=dist,
                         feature_fwd_bwd_ms=round(kern_ms, 4), feature_GBps=round(gbs, 1),
                         feature_hbm_frac=round(gbs / HBM_PEAK_GBS, 4), algorithmic_bytes=int(both),
                         phases_ms={p: round(x, 4) for p, x in phases.items()}, U=U, pairs=int(pairs))
        print(f"# config {config} {form}: {ms:.3f} ms/step, feature kernel {kern_ms:.3f} ms "
              f"({gbs:.0f} GB/s), pairs {pairs}, U {U}", file=sys.stderr, flush=True)
        del step, tF
        torch.cuda.empty_cache()
    # feature error of each low-precision form against the FP32 form (same Top-K records)
    ref = maps["f32"].float()
    for form in forms:
        if form == "f32":
            continue
        a = maps[form].float()
        nrm = ref.norm(dim=-1).clamp_min(1e-2)
        e = ((a - ref).norm(dim=-1) / nrm)
        out[form]["feature_err_vs_f32"] = dict(max=round(float(e.max()), 5), mean=round(float(e.mean()), 5))
        del a, e
    del maps, ref
    torch.cuda.empty_cache()
    return dict(workload=f"{V} views x {cams[0].width}x{cams[0].height} px, N={n} Gaussians, D={D}, K={K}",
                views=V, N=n, D=D, K=K, forms=out)


def time_steps(torch, step, steps, warmup):
    """Times `steps` steps after `warmup` untimed ones.  Inside the timed steps only
    the feature adjoint (the dominant HBM-bound kernel) is bracketed by HIP events, on
    torch's stream, where it and the main stream's work run (the side stream's work is
    joined into it before the feature kernel and before the end event); a second,
    separate pass runs every phase in order on one stream with an event after each, for
    the per-phase breakdown (each event costs a few us of GPU time, which is why the
    timed pass carries only two per step)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    step.kmarks = []
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    kern = [a.elapsed_time(b) for a, b in step.kmarks]
    step.kmarks = None
    # the per-phase steps run back to back as the timed ones do (a synchronization after
    # each would let the GPU idle and its first kernels start cold), then one wait
    phases, per_step, runs = {}, [], []
    for _ in range(steps):
        step.events = []
        step()
        runs.append(step.events)
    torch.cuda.synchronize()
    for ev in runs:
        for (_, a), (name, b) in zip(ev[:-1], ev[1:]):
            phases.setdefault(name, []).append(a.elapsed_time(b))
        per_step.append(ev[0][1].elapsed_time(ev[-1][1]))
    step.events = None
    # spread of single steps (from the pass with per-phase events, so a few us higher)
    dist = {f"p{q}": round(float(np.percentile(per_step, q)), 4) for q in (10, 50, 90)}
    return total_ms / steps, {k: float(np.median(v)) for k, v in phases.items()}, float(np.mean(kern)), dist


def counter_traffic(kernel, workload_ok):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    summary (already scaled by the copy calibration), or None when the workload
    differs or the kernel source changed since the counters were taken."""
    import hashlib
    if not workload_ok:
        return None
    csrc = os.path.join(ROOT, "paper_2602_06991_amd", "csrc")
    prof = os.path.join(ROOT, "profiles", "hbm_counters_c2_1200x680_K4_bf16.md")
    if not os.path.exists(prof):
        return None
    h = hashlib.sha256()
    for name in ("feature_impl.hpp", "feature_launch.hpp", "lgs_device.hpp"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    sha = h.hexdigest()[:16]
    for line in open(prof):
        if line.startswith("traffic:"):
            f = [x.strip() for x in line[len("traffic:"):].split("|")]
            if f[0] == sha and f[1] == kernel:
                return dict(read=int(f[2]), write=int(f[3]), total=int(f[2]) + int(f[3]))
    return None


def timed(torch, fn, reps=10):
    """Average ms of `fn` over `reps` launches after two warm-ups, by HIP events."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def copy_bandwidth(torch, nbytes):
    """GB/s of a plain device-to-device copy of `nbytes` (nbytes read and nbytes
    written): the achievable streaming rate, reported beside the 8 TB/s peak."""
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(torch, lambda: dst.copy_(src))
    del src, dst
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def tile_union_stats(ids, W, H):
    """Distinct Top-K Gaussians per 16x16 tile (host-side diagnostic)."""
    ids = ids.cpu().numpy()
    K = ids.shape[-1]
    out = []
    for ty in range(0, H, 16):
        for tx in range(0, W, 16):
            t = ids[ty:ty + 16, tx:tx + 16].reshape(-1)
            out.append(len(np.unique(t[t >= 0])))
    out = np.array(out)
    return dict(mean=round(float(out.mean()), 1), p99=int(np.percentile(out, 99)), max=int(out.max()))


def feature_bytes(npix, K, D, U, s_map, s_f, fp8):
    """Algorithmic HBM bytes of the feature render, of its L1 adjoint, and of both in
    one pass (map written and target read; ids and w read once, dL/dw written; the
    union's rows read and their gradient rows written; FP8 row scales)."""
    sc = 4 * U if fp8 else 0
    fwd = npix * D * s_map + 8 * npix * K + U * D * s_f + sc
    bwd = npix * D * s_map + 12 * npix * K + U * D * (s_f + 4) + sc
    both = 2 * npix * D * s_map + 12 * npix * K + U * D * (s_f + 4) + sc
    return fwd, bwd, both


def feature_ms(phases):
    if "feature_render_fwd_bwd" in phases:
        return phases["feature_render_fwd_bwd"]
    return phases["feature_render_fwd"] + phases["feature_render_bwd"]


def separate_feature_ms(torch, render, fw, store, scale, form, mp, target, d, n, reps=10):
    """The render and the L1 adjoint as two launches (for comparison with the one-pass
    kernel), each timed alone with HIP events over `reps` launches."""
    dfeat = torch.zeros(n, d, device="cuda")
    fs = 1.0 / (fw["ids"].shape[0] * fw["ids"].shape[1] * d)
    runs = {"feature_render_fwd": lambda: render.feature_fwd(fw["ids"], fw["w"], store, scale, form, mp),
            "feature_render_bwd_l1": lambda: render.feature_bwd_l1(fw["ids"], fw["w"], store, scale, form, mp,
                                                                   target, fs, dfeat)}
    out = {}
    for name, fn in runs.items():
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = round(a.elapsed_time(b) / reps, 4)
    del dfeat
    return out


def cpu_baseline(scene, K, form, gpu_out=None):
    """The FP64 oracle (test infrastructure, timed as a reported baseline, never tuned)
    rendering and differentiating one full frame of the same workload on the host:
    the median of three runs on every host thread, and one run on a single thread.
    With gpu_out (the GPU's C, D, Top-K ids and map of that frame) it also reports the
    GPU's errors against the oracle under the parity rule of the tests."""
    from oracle import oracle as O
    from paper_2602_06991_amd.scenegen import random_upstream
    cam = scene.cameras[0]
    g = scene.gaussians
    feat64 = g.feat.astype(np.float64)
    gC, gD, gO, gF = random_upstream(1, cam.W * cam.H, g.d)

    def once():
        t0 = time.perf_counter()
        r = O.render(g, cam, K)
        Fo = O.feature(r["ids"], r["w"], feat64)
        t1 = time.perf_counter()
        O.backward(g, cam, K, feat64, gC, gD, None, gF)
        t2 = time.perf_counter()
        return (t1 - t0, t2 - t1), r, Fo

    cores = O.num_threads()
    runs = [once() for _ in range(3)]
    fwd = float(np.median([x[0][0] for x in runs]))
    tot = float(np.median([sum(x[0]) for x in runs]))
    O.set_threads(1)
    (f1, b1), _, _ = once()
    O.set_threads(cores)
    out = dict(value=round(tot * 1e3, 1), unit="ms/frame", cores=cores, kind="oracle",
               sample=f"one full {cam.W}x{cam.H} frame (render, Top-K feature map, full adjoint), FP64 "
                      f"features (storage form {form} not applied); median of 3 runs on {cores} threads: "
                      f"fwd {1e3 * fwd:.0f} ms + bwd {1e3 * (tot - fwd):.0f} ms",
               single_thread_ms_per_frame=round(1e3 * (f1 + b1), 1))
    if gpu_out is not None:
        r, Fo = runs[0][1], runs[0][2]
        fl = O.flagged(r["margins"])
        bl = O.blend_flagged(r["margins"])
        ok, cl = ~fl, ~bl
        rel = lambda a, b, floor: float((np.abs(a - b) / np.maximum(np.abs(b), floor)).max())
        Fg = gpu_out["F"]
        nf = np.linalg.norm(Fg[ok] - Fo[ok], axis=-1) / np.maximum(np.linalg.norm(Fo[ok], axis=-1), 1e-2)
        out["gpu_errors_vs_oracle"] = dict(
            flagged_share=round(float(fl.mean()), 5), blend_flagged_share=round(float(bl.mean()), 5),
            topk_id_mismatch_unflagged=int(np.sum(np.any(gpu_out["ids"] != r["ids"], -1) & ok)),
            color_max_rel=float(f"{rel(gpu_out['C'][cl], r['C'][cl], 1e-2):.3g}"),
            depth_max_rel=float(f"{rel(gpu_out['D'][cl], r['D'][cl], 1e-2):.3g}"),
            feature_normwise_vs_unquantized_fp64=dict(max=float(f"{nf.max():.3g}"), mean=float(f"{nf.mean():.3g}")),
            rule="ids bit-exact on unflagged pixels; C, D on pixels whose blend decisions are clear; F normwise "
                 "on unflagged pixels against the FP64 map of the unquantized features")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this renderer runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)
    multi = [int(x) for x in args.multi_view.split(",") if x.strip()]
    import torch
    from paper_2602_06991_amd import lgs, render
    from paper_2602_06991_amd.scenegen import make_scene
    lgs.load()
    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.copy_calibration:
        src = torch.ones(64 << 20, device="cuda")          # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: 3 x {src.numel() * 4} bytes read and written", file=sys.stderr)
        del src, dst
    t_gen = time.perf_counter()
    scene = make_scene(args.config)
    cfg = scene.config
    print(f"# scene {cfg['W']}x{cfg['H']} N={cfg['N']} D={cfg['D']} generated in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    cam_np = scene.cameras[0]
    cam = lgs.make_camera(cam_np)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = {k: f(v) for k, v in zip(("means", "log_scales", "quats", "opacity_logits", "rgb", "feat"),
                                 scene.gaussians.arrays())}
    PT = {k: f(v) for k, v in zip(("means", "log_scales", "quats", "opacity_logits", "rgb", "feat"),
                                  scene.target.arrays())}
    del scene.target
    K = args.K
    forms = args.forms.split(",")
    results = {}
    gpu_out = None
    for form in forms:
        mp = "f32" if form == "f32" else "bf16"
        # target frame: the perturbed scene rendered by the same path, outside timing
        tproj = render.project(cam, PT)
        tb = render.Binner()
        tids, tranges, _ = tb(cam, PT["means"].shape[0], tproj["depth"], tproj["tile_rect"],
                              tproj["tiles_touched"])
        tfw = render.rasterize(cam, K, tproj, PT["rgb"], tids, tranges)
        tstore, tscale = render.quantize(PT["feat"], form)
        tF = render.feature_fwd(tfw["ids"], tfw["w"], tstore, tscale, form, mp)
        target = (tfw["C"].clone(), tfw["D"].clone(), tF.clone())
        del tproj, tb, tids, tranges, tfw, tstore, tscale, tF
        fused = args.feature_path == "fused"
        step = Step(torch, render, lgs, P, target, cam, K, form, fused, dense_quantize=args.quantize == "dense")
        ms, phases, kern_ms, dist = time_steps(torch, step, args.steps, args.warmup)
        pairs, fitted = step.binner.count()
        assert fitted, "pair buffer overflowed during timing"
        step.last["pairs"] = pairs
        fw = step.last["fw"]
        U = render.union_count(fw["ids"], P["feat"].shape[0])
        npix = cam.width * cam.height
        s_map = 4 if mp == "f32" else 2
        s_f = {"f32": 4, "bf16": 2, "fp8": 1}[form]
        bf, bb, b2 = feature_bytes(npix, K, cfg["D"], U, s_map, s_f, form == "fp8")
        sep = separate_feature_ms(torch, render, fw, step.last["store"], step.last["scale"], form, mp,
                                  target[2], cfg["D"], P["feat"].shape[0])
        # the pruning statistics of Sec. 3.3 (run every few hundred iterations, not per step)
        cnt = torch.zeros(P["feat"].shape[0], dtype=torch.int32, device="cuda")
        mxw = torch.zeros(P["feat"].shape[0], device="cuda")
        st = step.last
        # with the dispatch order of the replay, weighted by the forward's n_contrib
        prune_ms = timed(torch, lambda: render.prune_stats(
            cam, K, st["proj"], st["ids"], st["ranges"], fw, cnt, mxw,
            render.tile_order(cam, st["ranges"], n_contrib=fw["n_contrib"])))
        # the hybrid schedule's geometry-only iterations: no feature passes, no gamma term
        geo = Step(torch, render, lgs, P, target, cam, K, form, fused, geometry_only=True)
        geo_ms, _, _, _ = time_steps(torch, geo, args.steps, args.warmup)
        assert geo.binner.count()[1], "pair buffer overflowed during timing"
        del geo
        # the same step converting the whole FP32 table every step (the other schedule)
        dense_ms = None
        if form != "f32" and args.quantize == "rows":
            dq = Step(torch, render, lgs, P, target, cam, K, form, fused, dense_quantize=True)
            dense_ms, _, _, _ = time_steps(torch, dq, args.steps, args.warmup)
            del dq
        # and the Eq. 6 survival draw over the Gaussians never in a Top-K list, keeping half
        gen = torch.Generator(device="cuda").manual_seed(5)
        expo = torch.empty(P["feat"].shape[0], device="cuda").exponential_(generator=gen)
        select_ms = timed(torch, lambda: render.prune_select(cnt, mxw, 1, expo, 0.5))
        del cnt, mxw, expo
        if form == forms[0] and not args.no_cpu_baseline:
            gpu_out = dict(C=fw["C"].cpu().numpy().astype(np.float64), D=fw["D"].cpu().numpy().astype(np.float64),
                           ids=fw["ids"].cpu().numpy(), F=step.last["F"].float().cpu().numpy().astype(np.float64))
        # (pixel, Gaussian) pairs the blend walks: per pixel, its list up to the last
        # Gaussian it blends (n_contrib), the unit of the blend kernels' rates
        blend_pairs = int(fw["n_contrib"].sum())
        results[form] = dict(ms=ms, phases=phases, kern_ms=kern_ms, U=U, pairs=int(step.last["pairs"]),
                             blend_pairs=blend_pairs,
                             bytes_fwd=bf, bytes_bwd=bb, bytes_both=b2, fused=fused, separate=sep,
                             prune_ms=prune_ms, select_ms=select_ms, geo_ms=geo_ms, dense_ms=dense_ms, dist=dist,
                             tile_union=tile_union_stats(fw["ids"], cam.width, cam.height))
        print(f"# {form}: {ms:.3f} ms/step" + (f" (whole-table quantize {dense_ms:.3f})" if dense_ms else "")
              + f", U={U}, pairs={step.last['pairs']}, phases "
              + ", ".join(f"{k} {v:.3f}" for k, v in phases.items()), file=sys.stderr, flush=True)
        del step, target
        torch.cuda.empty_cache()
    sweep = {}
    if args.sweep:
        for k2 in (1, 8):
            for form in forms:
                mp = "f32" if form == "f32" else "bf16"
                tproj = render.project(cam, PT)
                tb = render.Binner()
                tids, tranges, _ = tb(cam, PT["means"].shape[0], tproj["depth"], tproj["tile_rect"],
                                      tproj["tiles_touched"])
                tfw = render.rasterize(cam, k2, tproj, PT["rgb"], tids, tranges)
                tstore, tscale = render.quantize(PT["feat"], form)
                tF = render.feature_fwd(tfw["ids"], tfw["w"], tstore, tscale, form, mp)
                step = Step(torch, render, lgs, P, (tfw["C"].clone(), tfw["D"].clone(), tF.clone()), cam,
                            k2, form, args.feature_path == "fused", dense_quantize=args.quantize == "dense")
                ms, ph, _, _ = time_steps(torch, step, max(5, args.steps // 2), 2)
                assert step.binner.count()[1], "pair buffer overflowed during timing"
                sweep[f"K{k2}_{form}"] = dict(ms_per_frame=round(ms, 4), feature_fwd_bwd_ms=round(feature_ms(ph), 4))
                del step
                torch.cuda.empty_cache()

    vanilla = {}
    if "bf16" in forms and args.vanilla:
        # Tab. 4's comparison: the dense alpha-blended feature field (every blended
        # Gaussian) in the same step, BF16 storage and map, L1 feature loss
        tproj = render.project(cam, PT)
        tb = render.Binner()
        tids, tranges, _ = tb(cam, PT["means"].shape[0], tproj["depth"], tproj["tile_rect"], tproj["tiles_touched"])
        tfw = render.rasterize(cam, K, tproj, PT["rgb"], tids, tranges)
        tstore, tscale = render.quantize(PT["feat"], "bf16")
        tF = render.feature_vanilla_fwd(cam, tproj, tids, tranges, tfw, tstore, tscale, "bf16")
        step = Step(torch, render, lgs, P, (tfw["C"].clone(), tfw["D"].clone(), tF.clone()), cam, K, "bf16",
                    fused=False, vanilla=True)
        del tproj, tb, tids, tranges, tfw, tstore, tscale, tF
        ms, ph, _, _ = time_steps(torch, step, max(5, args.steps // 2), 2)
        assert step.binner.count()[1], "pair buffer overflowed during timing"
        vanilla = dict(ms_per_frame=round(ms, 4),
                       feature_fwd_ms=round(ph["feature_render_fwd"], 4),
                       feature_bwd_ms=round(ph["feature_render_bwd"], 4),
                       feature_fwd_bwd_ms=round(ph["feature_render_fwd"] + ph["feature_render_bwd"], 4),
                       phases_ms={p_: round(x, 4) for p_, x in ph.items()})
        print(f"# vanilla bf16: {ms:.3f} ms/step, feature fwd {ph['feature_render_fwd']:.3f} + bwd "
              f"{ph['feature_render_bwd']:.3f} ms", file=sys.stderr, flush=True)
        del step
        torch.cuda.empty_cache()

    mv = {}
    for c in multi:
        mv[f"config{c}"] = multi_view(torch, render, lgs, c, max(3, args.steps // 4), 2, args.quantize == "dense")
        torch.cuda.empty_cache()

    main_form = forms[0]
    R = results[main_form]
    ph = R["phases"]
    # dominant kernel of the feature path (HBM-bound): the one-pass render + adjoint (or
    # the adjoint alone with --feature-path separate), timed by the HIP events around it
    # inside the timed steps
    mode = 2 if R["fused"] else 1
    kern = "feature_render_fwd_bwd_l1" if R["fused"] else "feature_render_bwd_l1"
    kbytes = R["bytes_both"] if R["fused"] else R["bytes_bwd"]
    achieved = kbytes / (R["kern_ms"] * 1e-3) / 1e9
    ft = {"bf16": "1, 1", "f32": "0, 0", "fp8": "2, 1"}[main_form]
    # the adjoint kernel's multi-slab variant serves D above one channel slab (512
    # channels with a BF16 map and one-term rows, 256 in the FP32 form)
    multi = cfg["D"] > (256 if main_form == "f32" else 512)
    kname = f"feature_bwd_kernel<{K}, {ft}, {mode}, {'true' if multi else 'false'}>"
    t = counter_traffic(kname, args.config == 2 and K == 4 and main_form == "bf16")
    traffic = None if t is None else t["total"]
    feat_ms = feature_ms(ph)
    feat_gbs = (R["bytes_both"] if R["fused"] else R["bytes_fwd"] + R["bytes_bwd"]) / (feat_ms * 1e-3) / 1e9
    line = {
        "metric": "Top-K feature render fwd+bwd ms/frame + HBM GB/s, BF16 vs FP32, D=512, 1 GPU",
        "value": round(R["ms"], 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 storage, f32 accumulate" if main_form == "bf16" else main_form,
        "data": "synthetic (seeded room scene; Replica/TUM stand-in)",
        "config": {"workload": f"{cfg['W']}x{cfg['H']} px x1 view, N={cfg['N']} Gaussians, "
                               f"D={cfg['D']}, K={K}, features {main_form}",
                   "W": cfg["W"], "H": cfg["H"], "N": cfg["N"], "D": cfg["D"], "K": K,
                   "feature_dtype": main_form},
        "feature_fwd_bwd_ms": round(feat_ms, 4),
        "feature_fwd_bwd_GBps": round(feat_gbs, 1),
        "feature_fwd_bwd_hbm_frac": round(feat_gbs / HBM_PEAK_GBS, 4),
        "feature_path": args.feature_path,
        "achievable_copy_GBps": copy_bandwidth(torch, cfg["W"] * cfg["H"] * cfg["D"] * 2),   # a BF16 map
        "forms": {k: {"ms_per_frame": round(v["ms"], 4),
                      "feature_fwd_bwd_ms": round(feature_ms(v["phases"]), 4),
                      "separate_launches_ms": v["separate"],
                      "fwd_ms_per_frame": round(v["phases"]["project_fwd"] + v["phases"]["bin_sort"] +
                                                v["phases"]["tile_order"] + v["phases"]["rasterize_topk_fwd"] +
                                                v["separate"]["feature_render_fwd"], 4),
                      "step_ms_percentiles": v["dist"],
                      # the render's own fwd+bwd: without the storage quantization of the
                      # master features and the caller's gradient zeroing
                      "ms_per_frame_excl_quantize_zeroing": round(sum(x for p, x in v["phases"].items()
                                                                      if p not in ("quantize", "zero_grads",
                                                                                   "clear_rows", "mark_rows")), 4),
                      "quantize": args.quantize if k != "f32" else None,
                      "dense_quantize_ms_per_frame": v["dense_ms"] and round(v["dense_ms"], 4),
                      "geometry_only_ms_per_frame": round(v["geo_ms"], 4),
                      "prune_stats_ms": round(v["prune_ms"], 4),
                      "prune_select_ms": round(v["select_ms"], 4),
                      "phases_ms": {p: round(x, 4) for p, x in v["phases"].items()},
                      "U": v["U"], "pairs": v["pairs"], "tile_union": v["tile_union"],
                      "blend_pairs": v["blend_pairs"],
                      "blend_fwd_Gpairs_per_s": round(v["blend_pairs"] / v["phases"]["rasterize_topk_fwd"] / 1e6, 2),
                      "blend_bwd_Gpairs_per_s": round(v["blend_pairs"] / v["phases"]["rasterize_topk_bwd"] / 1e6, 2)}
                  for k, v in results.items()},
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_read_write": None if t is None else [t["read"], t["write"]],
                     "algorithmic_bytes": int(kbytes),
                     "avg_ms": round(R["kern_ms"], 4)},
    }
    if sweep:
        line["k_sweep"] = sweep
    if vanilla:
        line["vanilla_bf16"] = vanilla
    if mv:
        line["multi_view"] = mv
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, K, main_form, gpu_out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
