"""Helpers of the GPU parity tests: move seeded inputs to the device, run the HIP
path through the C ABI, and compare with the oracle."""
import numpy as np

# Decision-margin thresholds: 4x the largest FP32 relative error of the blending
# weights measured on the GPU at 640x480 (5.2e-5); no pixel whose Top-K differed had a
# margin above 1.4e-5.
FLAG_EPS = dict(eps_skip=2.5e-4, eps_clamp=2.5e-4, eps_T=2.5e-4, eps_topk=2.5e-4)


def torch_mod():
    import torch
    return torch


def dev_params(g):
    torch = torch_mod()
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    return dict(means=f(g.means), log_scales=f(g.log_scales), quats=f(g.quats),
                opacity_logits=f(g.opacity_logits), rgb=f(g.rgb), feat=f(g.feat))


def gpu_forward(g, cam, K, P=None):
    """project -> bin_sort -> rasterize_topk on the GPU; numpy results + device state."""
    from paper_2602_06991_amd import lgs, render
    torch = torch_mod()
    P = P or dev_params(g)
    c = lgs.make_camera(cam)
    proj = render.project(c, P)
    binner = render.Binner()
    ids, ranges, m = binner(c, g.n, proj["depth"], proj["tile_rect"], proj["tiles_touched"])
    fw = render.rasterize(c, K, proj, P["rgb"], ids, ranges)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in fw.items()}
    state = dict(P=P, cam=c, proj=proj, sorted_ids=ids.clone(), ranges=ranges, fw=fw, pairs=m)
    return out, state


def rel_close(a, b, rtol, floor):
    """|a - b| <= rtol * max(|b|, floor), elementwise."""
    return np.abs(a - b) <= rtol * np.maximum(np.abs(b), floor)


def normwise(a, b, floor):
    """Per-row ||a - b|| / max(||b||, floor) over the last axis."""
    return np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), floor)
