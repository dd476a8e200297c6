"""Helpers for the GPU parity tests: move seeded scenes to the device, run the
HIP path through the C ABI, and build the oracle's ambiguity mask."""
from __future__ import annotations

import numpy as np
import torch

# Ambiguity bands: relative distance of a discrete decision from its
# threshold (FP64 oracle side) within which FP32 may legitimately decide the
# other way.  End to end (GPU projection vs FP64 projection) the splat
# parameters differ by FP32 rounding: oG by up to ~1e-4 relative near the
# skip contour, T' by ~1e-4 after ~100 steps, and the binary32 depth keys by
# up to ~3 ulps (3.6e-7 relative).  Staged (both sides composite the same
# binary32 splats in the same order) only the compositing arithmetic differs.
E2E = dict(skip=1e-4, stop=1e-3, depth=5e-7)
STAGED = dict(skip=1e-5, stop=1e-5, depth=0.0)


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2603_09632_amd as xgs  # fails loudly if libxgs.so is missing
    return xgs


def gaussians(scene, xgs, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return xgs.Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity),
                         t(scene.colors), t(scene.features))


def run_render(xgs, scene, cam, g=None, max_instances=None):
    g = g or gaussians(scene, xgs)
    c = xgs.camera_from(cam)
    p = xgs.xgs_project(g, c)
    m = int(p.tiles_touched.to(torch.int64).sum().item()) if max_instances is None else max_instances
    b = xgs.alloc_binning(g.n, max(m, 1), c)
    xgs.xgs_tile_sort(p, c, g.n, b)
    out, fT, nl = xgs.xgs_render_fwd(g, p, b, c)
    torch.cuda.synchronize()
    return dict(g=g, p=p, b=b, cam=c, out=out, final_T=fT, n_last=nl, m=m)


def ambiguous(r_oracle, bands=E2E):
    a = r_oracle.amb
    return (a[0] < bands["skip"]) | (a[1] < bands["stop"]) | (a[2] < bands["depth"])


def rel_max(gpu, ref, mask=None):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        gpu = gpu[..., ~mask]
        ref = ref[..., ~mask]
    den = np.abs(ref).max()
    return float(np.abs(gpu - ref).max() / (den if den > 0 else 1.0))


def rel_l2(gpu, ref):
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(gpu - ref) / (den if den > 0 else 1.0))


def np_(t):
    return t.detach().cpu().numpy()


def splat_from_oracle(xgs, pr, opacity, n):
    """Projected buffers holding the oracle's projection rounded to binary32."""
    p = xgs.Projected.alloc(n)
    sp = np.zeros((n, 8), np.float32)
    sp[:, 0:2] = pr.mean2d
    sp[:, 2:5] = pr.conic
    sp[:, 5] = opacity
    sp[:, 6] = pr.depth
    vis = pr.visible == 1
    sp[~vis, 0:5] = 0.0
    p.splat.copy_(torch.from_numpy(sp))
    p.tile_rect.copy_(torch.from_numpy(pr.rect.astype(np.uint16).view(np.int16)))
    p.tiles_touched.copy_(torch.from_numpy(pr.touched.astype(np.uint32).view(np.int32)))
    p.radius.copy_(torch.from_numpy(vis.astype(np.int32)))
    return p, sp


def binning_from_oracle(xgs, keys, vals, ranges, n, cam):
    m = len(keys)
    b = xgs.alloc_binning(n, max(m, 1), cam)
    if m:
        b.keys[:m].copy_(torch.from_numpy(keys.view(np.int64)))
        b.vals[:m].copy_(torch.from_numpy(vals.view(np.int32)))
    b.ranges.copy_(torch.from_numpy(np.ascontiguousarray(ranges).view(np.int32)))
    b.num_instances.fill_(m)
    b.tile_order = None  # tiles in id order (the sort kernel writes the table)
    return b
