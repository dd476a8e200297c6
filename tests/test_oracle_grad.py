"""Pins of the oracle's analytic gradient (no GPU): central finite differences of
its own forward in FP64, exact closed forms for the linear channels, the
single-Gaussian opacity derivative and a mirror symmetry.

Passage: the derivative of Eq. (rendering) / Eq. (discrete_render) through the
EWA projection of App. A.
"""
import math

import numpy as np
import pytest

import synth
from synth import Camera, Scene

CAM = Camera(width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0)


def small_scene(seed, n=24):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(-0.5, 0.5, (n, 2)), rng.uniform(2.0, 3.0, n)]
    ls = rng.normal(-2.6, 0.3, (n, 3))
    q = rng.standard_normal((n, 4))
    o = rng.uniform(0.2, 0.95, n)
    c = rng.uniform(0, 1, (n, 3))
    f = rng.standard_normal((n, 3))
    return Scene(means, ls, q, o, c, f)  # float64 on purpose: FD on exact values


def fields(s):
    return {"means": s.means, "log_scales": s.log_scales, "quats": s.quats, "opacity": s.opacity,
            "colors": s.colors, "features": s.features}


def with_field(s, name, arr):
    d = fields(s)
    d[name] = arr
    return Scene(d["means"], d["log_scales"], d["quats"], d["opacity"], d["colors"], d["features"])


def trace(r):
    return (r.n_last.copy(), r.amb[3].copy(), r.proj.rect.copy())


@pytest.mark.parametrize("seed", [0, 1])
def test_analytic_gradient_matches_central_fd(orc, seed):
    s = small_scene(seed)
    cam = CAM
    hs, ws, _, _ = orc.grid_info(cam)
    g = np.random.default_rng(100 + seed).standard_normal((4 + s.c_sem, hs, ws))
    r0 = orc.render(s, cam)
    gr = orc.render_grad(s, cam, g, r0)
    h = 1e-6
    checked = 0
    for name in ("means", "log_scales", "quats", "opacity", "colors", "features"):
        base = np.asarray(fields(s)[name], np.float64)
        ana = getattr(gr, name)
        for flat in range(base.size):
            ep = base.copy().reshape(-1); ep[flat] += h
            em = base.copy().reshape(-1); em[flat] -= h
            rp = orc.render(with_field(s, name, ep.reshape(base.shape)), cam)
            rm = orc.render(with_field(s, name, em.reshape(base.shape)), cam)
            # a discrete decision (skip / stop / clamp / tile set / order) that
            # flips inside [-h, h] makes the difference quotient meaningless
            if not all(np.array_equal(a, b) for a, b in zip(trace(rp), trace(r0))) or \
               not all(np.array_equal(a, b) for a, b in zip(trace(rm), trace(r0))):
                continue
            fd = (orc.loss(rp.out, g) - orc.loss(rm.out, g)) / (2 * h)
            a = ana.reshape(-1)[flat]
            assert abs(fd - a) <= 1e-5 * max(1.0, abs(a)), (name, flat, fd, a)
            checked += 1
    assert checked > 0.9 * sum(np.asarray(v).size for v in fields(s).values())


def test_channel_gradients_are_exact_weight_sums(orc):
    """dL/dc_i = sum_x w_i(x) g(x): L is linear in colours and features, so the
    unit-step difference is exact."""
    s = small_scene(3)
    hs, ws, _, _ = orc.grid_info(CAM)
    g = np.random.default_rng(5).standard_normal((4 + s.c_sem, hs, ws))
    r0 = orc.render(s, CAM)
    gr = orc.render_grad(s, CAM, g, r0)
    L0 = orc.loss(r0.out, g)
    for i in (0, 5, 11):
        for c in range(3):
            col = s.colors.copy(); col[i, c] += 1.0
            assert orc.loss(orc.render(with_field(s, "colors", col), CAM).out, g) - L0 == pytest.approx(gr.colors[i, c], abs=1e-9)
        fe = s.features.copy(); fe[i, 1] += 1.0
        assert orc.loss(orc.render(with_field(s, "features", fe), CAM).out, g) - L0 == pytest.approx(gr.features[i, 1], abs=1e-9)


def test_single_gaussian_opacity_derivative(orc):
    """One Gaussian, no clamp: dC/do = c G summed over covered pixels."""
    z, sig, o = 3.0, 0.06, 0.5
    s = Scene(np.array([[0.0, 0.0, z]]), np.full((1, 3), math.log(sig)), np.array([[1.0, 0, 0, 0]]),
              np.array([o]), np.array([[1.0, 0.0, 0.0]]), np.zeros((1, 1)))
    hs, ws, _, _ = orc.grid_info(CAM)
    g = np.zeros((5, hs, ws)); g[0] = 1.0
    r = orc.render(s, CAM)
    gr = orc.render_grad(s, CAM, g, r)
    s2 = (CAM.fx * sig / z) ** 2 + 0.3
    yy, xx = np.mgrid[0:hs, 0:ws] + 0.5
    G = np.exp(-((xx - CAM.cx) ** 2 + (yy - CAM.cy) ** 2) / (2 * s2))
    covered = o * G >= 1 / 255
    assert gr.opacity[0] == pytest.approx(G[covered].sum(), rel=1e-12)


def test_mirror_symmetry_zero_lateral_gradient(orc):
    """Centred isotropic Gaussian, upstream gradient mirror-symmetric in x:
    no force along x."""
    s = Scene(np.array([[0.0, 0.0, 3.0]]), np.full((1, 3), math.log(0.07)), np.array([[1.0, 0, 0, 0]]),
              np.array([0.8]), np.array([[0.3, 0.6, 0.9]]), np.zeros((1, 1)))
    hs, ws, _, _ = orc.grid_info(CAM)
    g = np.random.default_rng(0).standard_normal((5, hs, ws))
    g = g + g[:, :, ::-1]
    gr = orc.render_grad(s, CAM, g)
    assert abs(gr.means[0, 0]) < 1e-12 * max(1.0, np.abs(gr.means).max())
    assert abs(gr.mean2d[0, 0]) < 1e-12 * max(1.0, np.abs(gr.mean2d).max())


def test_tile_mask_restricts_gradient(orc):
    """Rendering only some tiles gives the gradient of the loss restricted to
    them (used to check large frames on a subset of tiles)."""
    s = synth.tiny_scene(seed=21, n=600)
    cam = synth.tiny_camera()
    hs, ws, ty, tx = orc.grid_info(cam)
    g = synth.upstream_grad(4 + s.c_sem, hs, ws, seed=3).astype(np.float64)
    mask = np.zeros(tx * ty, np.uint8); mask[[1, 5, 9, 14]] = 1
    pix = np.repeat(np.repeat(mask.reshape(ty, tx), 16, 0), 16, 1)[:hs, :ws]
    full = orc.render_grad(s, cam, g * pix[None])
    part = orc.render_grad(s, cam, g, tile_mask=mask)
    np.testing.assert_allclose(part.means, full.means, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(part.features, full.features, rtol=1e-12, atol=1e-12)
