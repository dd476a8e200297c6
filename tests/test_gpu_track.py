"""Tracking on the GPU (f2, Eq. (tracking) / Eq. (loss_track)): the L1
photometric + depth loss and the camera-pose gradient against the FP64
oracle."""
import numpy as np
import pytest
import torch
from dataclasses import replace

import oracle
import synth
from gpu_util import gaussians, np_, rel_max, require_gpu, run_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("C,hs,ws,depth", [(4, 5, 7, True), (12, 37, 53, True), (36, 64, 65, False)])
def test_tracking_loss_matches_oracle(xgs, C, hs, ws, depth):
    rng = np.random.default_rng(C + hs)
    out = rng.random((C, hs, ws)).astype(np.float32)
    img = rng.random((3, hs, ws)).astype(np.float32)
    dep = (rng.random((hs, ws)) * 3).astype(np.float32)
    dep[rng.random((hs, ws)) < 0.3] = 0.0
    lam = 0.3
    loss, d = xgs.xgs_tracking_loss(t(out), t(img), t(dep) if depth else None, lam)
    torch.cuda.synchronize()
    ref, dref = oracle.track_loss(out, img, dep if depth else None, lam)
    assert abs(float(np_(loss)[0]) - ref) <= 1e-5 * ref
    assert rel_max(np_(d), dref) < 1e-6


def posed_camera(cam):
    return replace(cam, viewmat=oracle.se3_exp(np.r_[0.05, -0.03, 0.1, 0.04, -0.06, 0.02]).astype(np.float32))


def test_pose_gradient_tiny_end_to_end(xgs):
    """Tiny scene at a posed camera: the GPU's own projection, binning,
    backward and pose reduction under a seeded upstream gradient; the pose
    gradient matches the oracle's within 1e-3 of its largest component."""
    scene = synth.tiny_scene(seed=3)
    cam = posed_camera(synth.tiny_camera())
    hs, ws, _, _ = oracle.grid_info(cam)
    g = np.random.default_rng(4).standard_normal((4 + scene.c_sem, hs, ws))
    ref = oracle.pose_grad(scene, cam, g)
    r = run_render(xgs, scene, cam)
    ws_ = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(scene.n)), dtype=torch.uint8, device="cuda")
    xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], t(g), r["final_T"], r["n_last"], workspace=ws_)
    d = xgs.xgs_pose_grad(r["g"], r["p"], r["cam"], ws_)
    torch.cuda.synchronize()
    d = np_(d)
    assert np.abs(d - ref).max() <= 1e-3 * np.abs(ref).max(), (d, ref)


def test_pose_gradient_room_300k(xgs):
    """300k-Gaussian room at 640x480, random upstream gradient on all 20
    channels: the GPU's pose gradient against the oracle's over the whole
    frame (relative max error <= 1e-3 of the largest component)."""
    scene = synth.room_scene(300_000, seed=2, c_sem=16)
    cam = synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[12])
    hs, ws, _, _ = oracle.grid_info(cam)
    g = np.random.default_rng(13).standard_normal((20, hs, ws))
    ref = oracle.pose_grad(scene, cam, g)
    r = run_render(xgs, scene, cam)
    ws_ = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(scene.n)), dtype=torch.uint8, device="cuda")
    xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], t(g), r["final_T"], r["n_last"], workspace=ws_)
    d = np_(xgs.xgs_pose_grad(r["g"], r["p"], r["cam"], ws_))
    torch.cuda.synchronize()
    print("pose gradient gpu", d, "oracle", ref)
    assert np.abs(d - ref).max() <= 1e-3 * np.abs(ref).max()


def test_tracking_step_against_a_perturbed_target(xgs):
    """Target = the oracle's render at a pose moved by a small twist; the
    tracking step at the original pose: its loss equals the oracle's tracking
    loss of the oracle's render at that pose (relative 1e-4), and the pose
    gradient points downhill (a small step along -grad lowers the loss)."""
    scene = synth.tiny_scene(seed=5)
    cam = posed_camera(synth.tiny_camera())
    xi = np.r_[0.01, 0.0, -0.01, 0.0, 0.01, 0.0]
    cam_t = replace(cam, viewmat=(oracle.se3_exp(xi) @ cam.viewmat).astype(np.float32))
    tgt = oracle.render(scene, cam_t).out
    img_np, dep_np = tgt[:3].astype(np.float32), tgt[3].astype(np.float32)
    img, dep = t(img_np), t(dep_np)
    r = run_render(xgs, scene, cam)
    loss, d_pose, out = xgs.tracking_step(r["g"], r["p"], r["b"], r["cam"], img, dep, 0.5)
    torch.cuda.synchronize()
    ref, _ = oracle.track_loss(oracle.render(scene, cam).out, img_np, dep_np, 0.5)
    assert abs(float(np_(loss)[0]) - ref) <= 1e-4 * ref
    d = np_(d_pose).astype(np.float64)
    step = -1e-3 * d / np.linalg.norm(d)
    cam_s = replace(cam, viewmat=(oracle.se3_exp(step) @ cam.viewmat).astype(np.float32))
    r2 = run_render(xgs, scene, cam_s)
    l2, _ = xgs.xgs_tracking_loss(r2["out"], img, dep, 0.5)
    torch.cuda.synchronize()
    assert float(np_(l2)[0]) < float(np_(loss)[0])
