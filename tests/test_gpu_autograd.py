"""Differentiation form (torch.autograd.Function around xgs_render_bwd):
gradients on all six parameter groups against the FP64 oracle's analytic
gradient and against central finite differences (h = 1e-3), at the tiny size
and at 1,000,000 Gaussians, 1200x680, 3 + 1 + 32 channels."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import E2E, ambiguous, np_, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity", "colors", "features")


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def params(scene, requires_grad=True):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda().requires_grad_(requires_grad)
    return {k: t(getattr(scene, k)) for k in GROUPS}


def tile_pixels(mask, cam):
    hs, ws, ty, tx = oracle.grid_info(cam)
    return np.repeat(np.repeat(mask.reshape(ty, tx), 16, 0), 16, 1)[:hs, :ws].astype(bool)


def autograd_grads(xgs, scene, cam, g):
    from paper_2603_09632_amd.autograd import render
    P = params(scene)
    out, fT, nl = render(*(P[k] for k in GROUPS), xgs.camera_from(cam))
    (out * torch.from_numpy(g).cuda()).sum().backward()
    torch.cuda.synchronize()
    return {k: np_(P[k].grad) for k in GROUPS}, out


def test_autograd_matches_oracle_tiny(xgs):
    scene, cam = synth.tiny_scene(seed=0), synth.tiny_camera().with_grid(2, 1, 0)
    ref = oracle.render(scene, cam)
    hs, ws, _, _ = oracle.grid_info(cam)
    g = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=3)
    g[:, ambiguous(ref, E2E)] = 0.0
    got, out = autograd_grads(xgs, scene, cam, g)
    want = oracle.render_grad(scene, cam, g.astype(np.float64), ref)
    errs = {k: rel_l2(got[k], getattr(want, k)) for k in GROUPS}
    assert all(v <= 1e-3 for v in errs.values()), errs


def test_autograd_chains_through_sigmoid_and_features_only(xgs):
    from paper_2603_09632_amd.autograd import render
    scene, cam = synth.tiny_scene(seed=1), synth.tiny_camera()
    P = params(scene)
    raw = torch.logit(P["opacity"].detach().clone()).requires_grad_(True)
    hs, ws, _, _ = oracle.grid_info(cam)
    g = torch.from_numpy(synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=4)).cuda()
    out, _, _ = render(P["means"], P["log_scales"], P["quats"], torch.sigmoid(raw), P["colors"], P["features"],
                       xgs.camera_from(cam))
    (out * g).sum().backward()
    P2 = params(scene)
    out2, _, _ = render(*(P2[k] for k in GROUPS), xgs.camera_from(cam))
    (out2 * g).sum().backward()
    sig = torch.sigmoid(raw.detach())
    assert rel_l2(np_(raw.grad), np_(P2["opacity"].grad * sig * (1 - sig))) < 1e-5
    P3 = params(scene)
    out3, _, _ = render(*(P3[k] for k in GROUPS), xgs.camera_from(cam), features_only=True)
    (out3 * g).sum().backward()
    assert P3["means"].grad is None and P3["opacity"].grad is None
    assert rel_l2(np_(P3["features"].grad), np_(P2["features"].grad)) < 1e-6


@pytest.fixture(scope="module")
def big():
    scene = synth.room_scene(1_000_000, seed=2, c_sem=32)
    cam = synth.room_camera(1200, 680, 600.0, synth.room_trajectory(100, seed=10)[9])
    hs, ws, ty, tx = oracle.grid_info(cam)
    rng = np.random.default_rng(1)
    mask = np.zeros(tx * ty, np.uint8)
    mask[rng.choice(tx * ty, 100, replace=False)] = 1
    ref = oracle.render(scene, cam, tile_mask=mask)
    sel = tile_pixels(mask, cam) & ~ambiguous(ref, E2E)
    g = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=5)
    g[:, ~sel] = 0.0
    return scene, cam, mask, ref, g


def test_autograd_1m_against_oracle_gradient(xgs, big):
    """All six groups at 1M Gaussians / 1200x680 / 36 channels, the loss taken
    over 100 random tiles (every Gaussian touching them gets a gradient)."""
    scene, cam, mask, ref, g = big
    got, _ = autograd_grads(xgs, scene, cam, g)
    want = oracle.render_grad(scene, cam, g.astype(np.float64), ref, tile_mask=mask)
    errs = {k: rel_l2(got[k], getattr(want, k)) for k in GROUPS}
    touched = int((np.abs(want.opacity) > 0).sum())
    print(f"1M autograd vs oracle rel-L2 {errs} over {touched} Gaussians")
    assert touched > 10_000
    assert all(v <= 1e-3 for v in errs.values()), errs


def test_autograd_1m_against_central_fd(xgs, big):
    """64 random contributing Gaussians of the 1M scene, every parameter.  The
    oracle evaluates each difference on the sub-scene of Gaussians overlapping
    the Gaussian's tiles (nothing else reaches those pixels), restricted to
    pixels whose blending decisions do not change within the steps; the GPU
    gradient is of that same restricted loss.  With these ~3 px splats a 1 mm
    step of a mean moves the splat by ~8% of its width, so the plain central
    difference at h = 1e-3 carries an O(h^2) truncation error of order 1e-3;
    the check uses the Richardson combination (4 D(h/2) - D(h)) / 3 of the
    central differences at h = 1e-3 and 5e-4 (error O(h^4)) and reports the
    plain one beside it."""
    scene, cam, _, _, _ = big
    hs, ws, ty, tx = oracle.grid_info(cam)
    base_pr = oracle.project(scene, cam)
    g0 = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=6).astype(np.float64)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    gs = xgs.Gaussians(*(t(getattr(scene, k)) for k in GROUPS))
    c = xgs.camera_from(cam)
    out, fT, nl, p, b = xgs.render(gs, c)
    grads = xgs.Gaussians.empty_like(gs)
    ws_bwd = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(gs.n)), dtype=torch.uint8, device="cuda")
    gk_dev = torch.empty_like(out)
    rng = np.random.default_rng(20)
    visible = np.nonzero(base_pr.visible)[0]
    rect = base_pr.rect
    h = 1e-3
    got, want, plain = ({k: [] for k in GROUPS} for _ in range(3))
    tried = 0
    chosen = []
    for i in rng.permutation(visible):
        if len(chosen) == 64:
            break
        x0, y0, x1, y1 = rect[i]
        if (x1 - x0) * (y1 - y0) <= 4:
            chosen.append(i)
    for n_done, i in enumerate(chosen):
        x0, y0, x1, y1 = rect[i]
        tiles = [y * tx + x for y in range(y0, y1) for x in range(x0, x1)]
        inside = oracle.tile_view(np.ones((hs, ws)), cam, tiles) == 1
        gt = oracle.tile_view(g0, cam, tiles)
        members = np.nonzero((rect[:, 0] < x1) & (rect[:, 2] > x0) & (rect[:, 1] < y1) & (rect[:, 3] > y0))[0]
        sub = scene.subset(members)
        isub = int(np.searchsorted(members, i))
        _, _, _, amb0 = oracle.render_tiles(sub, cam, tiles)
        stable = inside & ~((amb0[:, 0] < E2E["skip"]) | (amb0[:, 1] < E2E["stop"]) | (amb0[:, 2] < E2E["depth"]))
        base = {k: getattr(sub, k).astype(np.float64) for k in GROUPS}
        for k in GROUPS:
            arr = base[k]
            for j in range(arr.shape[1] if arr.ndim == 2 else 1):
                tried += 1
                rs = {}
                for step in (h, -h, h / 2, -h / 2):
                    a = {kk: vv.copy() for kk, vv in base.items()}
                    if arr.ndim == 2:
                        a[k][isub, j] += step
                    else:
                        a[k][isub] += step
                    rs[step] = oracle.render_tiles(synth.Scene(**a), cam, tiles)
                if any(not np.array_equal(x[0].rect[isub], rect[i]) for x in rs.values()):
                    continue
                keep = stable.copy()
                for x in rs.values():
                    keep &= x[3][:, 3] == amb0[:, 3]
                gk = gt * keep[:, None]
                L = {st: float((x[1] * gk).sum()) for st, x in rs.items()}
                d1 = (L[h] - L[-h]) / (2 * h)
                d2 = (L[h / 2] - L[-h / 2]) / h
                gk_dev.copy_(torch.from_numpy(oracle.untile(gk, cam, tiles).astype(np.float32)))
                xgs.xgs_render_bwd(gs, p, b, c, gk_dev, fT, nl, grads=grads, workspace=ws_bwd)
                row = getattr(grads, k)[int(i)]
                v = row[j] if arr.ndim == 2 else row
                got[k].append(float(v.item()))
                want[k].append((4 * d2 - d1) / 3)
                plain[k].append(d1)
        if n_done % 8 == 7:
            print(f"  FD: {n_done + 1}/64 Gaussians", flush=True)
    errs = {k: rel_l2(got[k], want[k]) for k in GROUPS}
    errs_plain = {k: rel_l2(got[k], plain[k]) for k in GROUPS}
    counts = {k: len(want[k]) for k in GROUPS}
    print(f"1M FD rel-L2 (Richardson) {errs}; plain central h=1e-3 {errs_plain}; counts {counts} of {tried}")
    assert sum(counts.values()) >= 0.9 * tried
    assert all(v <= 1e-3 for v in errs.values()), errs
