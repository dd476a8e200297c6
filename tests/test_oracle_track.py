"""Pins of the oracle's tracking pieces (Eq. (tracking), Eq. (loss_track)):
the L1 photometric + depth loss and the camera-pose gradient, against finite
differences, the library matrix exponential, closed forms and a rigid-motion
invariance."""
from dataclasses import replace

import numpy as np
import pytest
import scipy.linalg

import oracle
from synth import Camera, Scene

CAM = Camera(width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0)


def small_scene(seed, n=24):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(-0.5, 0.5, (n, 2)), rng.uniform(2.0, 3.0, n)]
    ls = rng.normal(-2.6, 0.3, (n, 3))
    q = rng.standard_normal((n, 4))
    o = rng.uniform(0.2, 0.95, n)
    c = rng.uniform(0, 1, (n, 3))
    f = rng.standard_normal((n, 2))
    return Scene(means, ls, q, o, c, f)


def twist(xi):
    rho, phi = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    X[:3, 3] = rho
    return X


def test_se3_exp_matches_library_expm():
    rng = np.random.default_rng(0)
    for _ in range(5):
        xi = rng.standard_normal(6) * 0.7
        assert np.abs(oracle.se3_exp(xi) - scipy.linalg.expm(twist(xi))).max() < 1e-13
    assert np.abs(oracle.se3_exp(np.r_[1.0, 2.0, 3.0, 0, 0, 0]) - scipy.linalg.expm(twist(np.r_[1.0, 2, 3, 0, 0, 0]))).max() < 1e-15


def test_track_loss_gradient_and_closed_forms():
    rng = np.random.default_rng(1)
    C, H, W = 6, 5, 7
    out = rng.random((C, H, W))
    img = rng.random((3, H, W))
    dep = rng.random((H, W)) * 3
    dep[rng.random((H, W)) < 0.3] = 0.0          # pixels without depth
    lam = 0.4
    val, d = oracle.track_loss(out, img, dep, lam)
    assert np.all(d[4:] == 0)
    h = 1e-7
    for idx in [(0, 1, 2), (2, 4, 6), (3, 0, 0), (3, 2, 3), (1, 3, 1)]:
        a = out.copy(); a[idx] += h
        b = out.copy(); b[idx] -= h
        num = (oracle.track_loss(a, img, dep, lam)[0] - oracle.track_loss(b, img, dep, lam)[0]) / (2 * h)
        assert num == pytest.approx(d[idx], abs=1e-9)
    # perfect prediction: zero loss
    perfect = out.copy(); perfect[:3] = img; perfect[3] = dep
    assert oracle.track_loss(perfect, img, dep, lam)[0] == 0.0
    # depth term: mean over the pixels that have depth
    has = dep > 0
    only_depth = perfect.copy(); only_depth[3] += 0.5
    assert oracle.track_loss(only_depth, img, dep, lam)[0] == pytest.approx(lam * 0.5 * has.sum() / has.sum())
    # no depth anywhere: photometric term only
    v0, d0 = oracle.track_loss(out, img, np.zeros((H, W)), lam)
    assert v0 == pytest.approx(np.abs(out[:3] - img).mean()) and np.all(d0[3] == 0)


def trace(r):
    return (r.n_last.copy(), r.amb[3].copy(), r.proj.rect.copy())


def base_view():
    T = oracle.se3_exp(np.r_[0.05, -0.03, 0.1, 0.04, -0.06, 0.02])
    return T


@pytest.mark.parametrize("seed", [0, 1])
def test_pose_gradient_matches_central_fd(seed):
    s = small_scene(seed)
    cam = replace(CAM, viewmat=base_view())
    hs, ws, _, _ = oracle.grid_info(cam)
    g = np.random.default_rng(50 + seed).standard_normal((4 + s.c_sem, hs, ws))
    r0 = oracle.render(s, cam)
    ana = oracle.pose_grad(s, cam, g, r0)
    h = 1e-6
    checked = 0
    for k in range(6):
        e = np.zeros(6); e[k] = h
        cp = replace(cam, viewmat=oracle.se3_exp(e) @ cam.viewmat)
        cm = replace(cam, viewmat=oracle.se3_exp(-e) @ cam.viewmat)
        rp, rm = oracle.render(s, cp), oracle.render(s, cm)
        if not all(np.array_equal(a, b) for a, b in zip(trace(rp), trace(r0))) or \
           not all(np.array_equal(a, b) for a, b in zip(trace(rm), trace(r0))):
            continue
        fd = (oracle.loss(rp.out, g) - oracle.loss(rm.out, g)) / (2 * h)
        assert fd == pytest.approx(ana[k], rel=1e-5, abs=1e-7), (k, fd, ana[k])
        checked += 1
    assert checked >= 5


def test_pose_translation_part_is_the_summed_mean_gradient():
    """dL/drho = sum_i dL/dp_i = Rv sum_i dL/dmu_i."""
    s = small_scene(2)
    cam = replace(CAM, viewmat=base_view())
    hs, ws, _, _ = oracle.grid_info(cam)
    g = np.random.default_rng(9).standard_normal((4 + s.c_sem, hs, ws))
    r = oracle.render(s, cam)
    d_pose = oracle.pose_grad(s, cam, g, r)
    gr = oracle.render_grad(s, cam, g, r)
    Rv = np.asarray(cam.viewmat, np.float64)[:3, :3]
    assert np.abs(d_pose[:3] - Rv @ gr.means.sum(0)).max() < 1e-10 * max(1.0, np.abs(d_pose[:3]).max())


def test_pose_gradient_is_invariant_to_a_shared_rigid_motion():
    """Moving the world and the camera by the same rigid motion leaves every
    camera-frame quantity, hence the left-perturbation gradient, unchanged."""
    s = small_scene(3)
    cam = replace(CAM, viewmat=base_view())
    hs, ws, _, _ = oracle.grid_info(cam)
    g = np.random.default_rng(10).standard_normal((4 + s.c_sem, hs, ws))
    A = oracle.se3_exp(np.r_[0.3, -0.2, 0.5, 0.2, 0.1, -0.3])
    Ra, ta = A[:3, :3], A[:3, 3]
    means2 = s.means @ Ra.T + ta
    # rotate each Gaussian's orientation with the world: q2 = qa * q
    w = np.sqrt(max(0.0, 1 + np.trace(Ra))) / 2
    qa = np.array([w, (Ra[2, 1] - Ra[1, 2]) / (4 * w), (Ra[0, 2] - Ra[2, 0]) / (4 * w), (Ra[1, 0] - Ra[0, 1]) / (4 * w)])
    q = s.quats / np.linalg.norm(s.quats, axis=1, keepdims=True)
    q2 = np.c_[qa[0] * q[:, 0] - qa[1:] @ q[:, 1:].T,
               qa[0] * q[:, 1:] + q[:, :1] * qa[1:] + np.cross(np.broadcast_to(qa[1:], q[:, 1:].shape), q[:, 1:])]
    s2 = Scene(means2, s.log_scales, q2, s.opacity, s.colors, s.features)
    cam2 = replace(cam, viewmat=cam.viewmat @ np.linalg.inv(A))
    d1 = oracle.pose_grad(s, cam, g)
    d2 = oracle.pose_grad(s2, cam2, g)
    assert np.abs(d1 - d2).max() < 1e-8 * max(1.0, np.abs(d1).max())
