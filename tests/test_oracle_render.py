"""Pins of the FP64 oracle's projection, binning and compositing against facts
fixed by the paper and by mathematics (no GPU).

Passages: App. A (Sigma = R S S^T R^T, Sigma' = J W Sigma W^T J^T), Sec. 3.1
Eq. (rendering) and App. B Eq. (discrete_render) (front-to-back blending; depth
and feature maps by substitution), App. D Eq. (sampled_loc) (sampled grid).
"""
import itertools
import math

import numpy as np
import pytest

import synth
from synth import Camera, Scene


def one_scene(means, log_scales, quats=None, opac=None, colors=None, feats=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    ls = np.asarray(log_scales, np.float32).reshape(n, 3)
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None else np.asarray(quats, np.float32).reshape(n, 4)
    o = np.full(n, 0.8, np.float32) if opac is None else np.asarray(opac, np.float32).reshape(n)
    c = np.ones((n, 3), np.float32) if colors is None else np.asarray(colors, np.float32).reshape(n, 3)
    f = np.zeros((n, 2), np.float32) if feats is None else np.asarray(feats, np.float32).reshape(n, -1)
    return Scene(means, ls, q, o, c, f)


CAM = Camera(width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0)


# ----------------------------------------------------------------- projection
def test_isotropic_on_axis_closed_form(orc):
    """Sigma' = ((f sigma / z)^2 + 0.3) I and mean2d = principal point."""
    z, ls = 3.0, math.log(0.05)
    pr = orc.project(one_scene([0, 0, z], [ls] * 3), CAM)
    s2 = (CAM.fx * math.exp(np.float32(ls)) / z) ** 2 + 0.3
    np.testing.assert_allclose(pr.cov2d[0], [s2, 0, s2], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(pr.mean2d[0], [CAM.cx, CAM.cy], rtol=0, atol=1e-12)
    np.testing.assert_allclose(pr.conic[0], [1 / s2, 0, 1 / s2], rtol=1e-12, atol=1e-14)
    tau = 2 * math.log(255 * float(np.float32(0.8)))
    np.testing.assert_allclose(pr.ext[0], [math.sqrt(tau * s2)] * 2, rtol=1e-12)
    assert pr.depth[0] == pytest.approx(z)


def test_axis_aligned_off_axis_hand_derived(orc):
    """Sigma = diag(sx^2, sy^2, sz^2); J = [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]]."""
    x, y, z = 0.3, -0.2, 2.5
    sx, sy, sz = 0.04, 0.07, 0.1
    pr = orc.project(one_scene([x, y, z], np.log([sx, sy, sz])), CAM)
    sx, sy, sz = (math.exp(float(np.float32(math.log(v)))) for v in (sx, sy, sz))
    x, y, z = (float(np.float32(v)) for v in (x, y, z))
    f = CAM.fx
    a = (f / z) ** 2 * sx ** 2 + (f * x / z ** 2) ** 2 * sz ** 2 + 0.3
    b = (f * x / z ** 2) * (f * y / z ** 2) * sz ** 2
    c = (f / z) ** 2 * sy ** 2 + (f * y / z ** 2) ** 2 * sz ** 2 + 0.3
    np.testing.assert_allclose(pr.cov2d[0], [a, b, c], rtol=1e-12)
    np.testing.assert_allclose(pr.mean2d[0], [f * x / z + CAM.cx, f * y / z + CAM.cy], rtol=1e-14)


def test_frustum_guard_clamps_jacobian(orc):
    """Far off-axis: J is evaluated at x/z clamped to 1.3 (W/2)/fx."""
    x, y, z = 4.0, 0.0, 2.0
    s = 0.05
    pr = orc.project(one_scene([x, y, z], [math.log(s)] * 3), CAM)
    s = math.exp(float(np.float32(math.log(s))))
    lim = 1.3 * (CAM.width / 2) / CAM.fx
    tx = lim * z
    f = CAM.fx
    a = (f / z) ** 2 * s ** 2 + (f * tx / z ** 2) ** 2 * s ** 2 + 0.3
    np.testing.assert_allclose(pr.cov2d[0, 0], a, rtol=1e-12)
    assert pr.mean2d[0, 0] == pytest.approx(f * x / z + CAM.cx)


def test_conic_inverse_and_min_eigenvalue(orc):
    s = synth.tiny_scene(seed=4, n=500)
    pr = orc.project(s, synth.tiny_camera())
    a, b, c = pr.cov2d.T
    A, B, C = pr.conic.T
    np.testing.assert_allclose(a * A + b * B, 1, atol=1e-10)
    np.testing.assert_allclose(a * B + b * C, 0, atol=1e-10)
    np.testing.assert_allclose(b * B + c * C, 1, atol=1e-10)
    lam_min = (a + c) / 2 - np.sqrt(((a - c) / 2) ** 2 + b ** 2)
    assert (lam_min >= 0.3 - 1e-9).all()


def test_quaternion_sign_and_scale_invariance(orc):
    s = synth.tiny_scene(seed=5, n=200)
    cam = synth.tiny_camera()
    p0 = orc.project(s, cam)
    for k in (-1.0, 2.5, 0.125):
        s2 = Scene(s.means, s.log_scales, s.quats.astype(np.float64) * k, s.opacity, s.colors, s.features)
        p1 = orc.project(s2, cam)
        np.testing.assert_allclose(p1.cov2d, p0.cov2d, rtol=1e-9, atol=1e-12)
        np.testing.assert_array_equal(p1.rect, p0.rect)


def test_rigid_motion_invariance(orc):
    """Moving world and camera by the same rigid motion leaves the splats unchanged."""
    s = synth.tiny_scene(seed=6, n=300)
    cam = synth.tiny_camera()
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    t = np.array([0.5, -1.0, 2.0])
    means = s.means.astype(np.float64) @ R.T + t
    # rotate each Gaussian's frame: q' = q_R * q (Hamilton product with R's quaternion)
    qr = np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)])
    def qmul(a, b):
        w1, x1, y1, z1 = a; w2, x2, y2, z2 = b.T
        return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    q = qmul(qr, s.quats.astype(np.float64))
    view = np.eye(4); view[:3, :3] = R.T; view[:3, 3] = -R.T @ t
    # The oracle reads binary32-valued scenes through float64, so feed float64 directly.
    s2 = Scene(means, s.log_scales.astype(np.float64), q, s.opacity.astype(np.float64), s.colors, s.features)
    cam2 = Camera(**{**cam.__dict__, "viewmat": view})
    p0 = orc.project(Scene(*(a.astype(np.float64) for a in (s.means, s.log_scales, s.quats, s.opacity)), s.colors, s.features), cam)
    p1 = orc.project(s2, cam2)
    np.testing.assert_allclose(p1.mean2d, p0.mean2d, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(p1.cov2d, p0.cov2d, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(p1.depth, p0.depth, rtol=1e-12)


def test_near_plane_and_low_opacity_cull(orc):
    sc = one_scene([[0, 0, 0.1], [0, 0, 3.0], [0, 0, 3.0]], [[-3] * 3] * 3, opac=[0.8, 0.8, 0.5 / 255])
    pr = orc.project(sc, CAM)
    assert list(pr.visible) == [0, 1, 0]
    assert list(pr.touched) == [0, 2, 0]  # centre (32, 24): tile columns 1-2, tile row 1


def test_rect_is_the_set_of_pixel_centres_in_the_box(orc):
    """Brute force over sampled pixels: the tile rectangle covers exactly the
    tiles holding a pixel centre within the opacity-aware box (Eq. sampled_loc)."""
    rng = np.random.default_rng(7)
    for stride, oy, ox in ((1, 0, 0), (2, 1, 0), (3, 2, 1)):
        cam = synth.tiny_camera().with_grid(stride, oy, ox)
        s = synth.tiny_scene(seed=8, n=300)
        pr = orc.project(s, cam)
        hs, ws, ty, tx = orc.grid_info(cam)
        cx = ox + np.arange(ws) * stride + 0.5
        cy = oy + np.arange(hs) * stride + 0.5
        for i in rng.choice(s.n, 60, replace=False):
            if not pr.visible[i]:
                continue
            cols = np.nonzero(np.abs(cx - pr.mean2d[i, 0]) <= pr.ext[i, 0])[0]
            rows = np.nonzero(np.abs(cy - pr.mean2d[i, 1]) <= pr.ext[i, 1])[0]
            assert len(cols) and len(rows)
            assert list(pr.rect[i]) == [cols.min() // 16, rows.min() // 16, cols.max() // 16 + 1, rows.max() // 16 + 1]


# -------------------------------------------------------------------- binning
def brute_lists(pr, tiles_x, tiles_y):
    dbits = pr.depth.astype(np.float32).view(np.uint32)
    lists = []
    for t in range(tiles_x * tiles_y):
        x, y = t % tiles_x, t // tiles_x
        members = [i for i in range(len(pr.depth))
                   if pr.rect[i, 0] <= x < pr.rect[i, 2] and pr.rect[i, 1] <= y < pr.rect[i, 3]]
        lists.append(sorted(members, key=lambda i: (int(dbits[i]), i)))
    return lists


def test_binning_matches_brute_force_and_sorted(orc):
    s = synth.tiny_scene(seed=9, n=400)
    cam = synth.tiny_camera()
    pr = orc.project(s, cam)
    hs, ws, ty, tx = orc.grid_info(cam)
    keys, vals, ranges = orc.bin_instances(pr.rect, orc.depth_bits(pr.depth), tx, ty)
    want = brute_lists(pr, tx, ty)
    for t in range(tx * ty):
        b, e = ranges[t]
        assert list(vals[b:e]) == want[t]
        if e == b:
            assert b == 0
    # keys are the packed (tile, depth bits) and ascending as tuples with the index
    tup = [(int(k), int(v)) for k, v in zip(keys, vals)]
    assert tup == sorted(tup)
    dbits = orc.depth_bits(pr.depth)
    assert all(int(k) & 0xFFFFFFFF == int(dbits[v]) for k, v in zip(keys, vals))


def test_binning_permutation_invariance(orc):
    """Relabelling the input order of <= 6 Gaussians relabels the sorted lists
    and nothing else (every permutation)."""
    rng = np.random.default_rng(11)
    means = np.c_[rng.uniform(-0.2, 0.2, (6, 2)), rng.uniform(2.0, 2.2, 6)]
    means[3, 2] = means[1, 2]  # an exact depth tie, broken by index
    s = one_scene(means, np.full((6, 3), -2.5))
    cam = Camera(width=48, height=48, fx=60.0, fy=60.0, cx=24.0, cy=24.0)
    hs, ws, ty, tx = orc.grid_info(cam)
    base = orc.project(s, cam)
    _, v0, r0 = orc.bin_instances(base.rect, orc.depth_bits(base.depth), tx, ty)
    for perm in itertools.permutations(range(6)):
        perm = np.array(perm)
        pr = orc.project(s.subset(perm), cam)
        _, v1, r1 = orc.bin_instances(pr.rect, orc.depth_bits(pr.depth), tx, ty)
        np.testing.assert_array_equal(r1, r0)
        for t in range(tx * ty):
            b, e = r0[t]
            new = [int(i) for i in v1[b:e]]
            got = [int(perm[i]) for i in new]
            ref = [int(i) for i in v0[b:e]]
            depth = lambda i: float(np.float32(means[i, 2]))
            assert sorted(got) == sorted(ref)
            assert [depth(i) for i in got] == [depth(i) for i in ref]
            # equal depths are ordered by the (new) input index
            for k in range(len(new) - 1):
                if depth(got[k]) == depth(got[k + 1]):
                    assert new[k] < new[k + 1]


# ---------------------------------------------------------------- compositing
def test_single_isotropic_gaussian_analytic(orc):
    z, sig, o = 3.0, 0.06, 0.7
    s = one_scene([0, 0, z], [math.log(sig)] * 3, opac=[o], colors=[[0.2, 0.5, 0.9]], feats=[[1.5, -2.0]])
    r = orc.render(s, CAM)
    sig = math.exp(float(np.float32(math.log(sig))))
    o = float(np.float32(o))
    s2 = (CAM.fx * sig / z) ** 2 + 0.3
    hs, ws, _, _ = orc.grid_info(CAM)
    yy, xx = np.mgrid[0:hs, 0:ws] + 0.5
    d2 = (xx - CAM.cx) ** 2 + (yy - CAM.cy) ** 2
    a = np.minimum(0.99, o * np.exp(-d2 / (2 * s2)))
    a = np.where(a >= 1 / 255, a, 0.0)
    col = np.array([0.2, 0.5, 0.9], np.float32).astype(np.float64)
    for c in range(3):
        np.testing.assert_allclose(r.out[c], col[c] * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.out[3], z * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.out[4], 1.5 * a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.final_T, 1 - a, rtol=1e-12)
    # symmetric image about the principal point
    np.testing.assert_allclose(r.out[0], r.out[0][::-1, :], rtol=1e-12)
    np.testing.assert_allclose(r.out[0], r.out[0][:, ::-1], rtol=1e-12)


def test_two_gaussians_closed_form(orc):
    """C = c1 a1 + c2 a2 (1 - a1) for a front and a back Gaussian."""
    s = one_scene([[0, 0, 2.0], [0.05, 0, 3.0]], [[math.log(0.05)] * 3, [math.log(0.08)] * 3],
                  opac=[0.6, 0.9], colors=[[1, 0, 0], [0, 1, 0]])
    r = orc.render(s, CAM)
    pr = r.proj
    hs, ws, _, _ = orc.grid_info(CAM)
    yy, xx = np.mgrid[0:hs, 0:ws] + 0.5
    def alpha(i):
        dx, dy = xx - pr.mean2d[i, 0], yy - pr.mean2d[i, 1]
        A, B, C = pr.conic[i]
        a = np.minimum(0.99, float(np.float32([0.6, 0.9][i])) * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy)))
        return np.where(a >= 1 / 255, a, 0.0)
    a1, a2 = alpha(0), alpha(1)
    np.testing.assert_allclose(r.out[0], a1, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.out[1], a2 * (1 - a1), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.final_T, (1 - a1) * (1 - a2), rtol=1e-12)


def test_weights_plus_T_is_one_and_T_bounds(orc):
    """Constant colour 1: out = sum_i w_i = 1 - T_final (the product telescopes);
    T never drops below the stop threshold."""
    s = synth.tiny_scene(seed=12)
    s = Scene(s.means, s.log_scales, s.quats, s.opacity, np.ones_like(s.colors), s.features)
    r = orc.render(s, synth.tiny_camera())
    np.testing.assert_allclose(r.out[0] + r.final_T, 1.0, rtol=0, atol=1e-12)
    assert (r.final_T >= 1e-4).all() and (r.final_T <= 1).all()
    assert (r.final_T < 1e-3).any()  # the stop threshold is actually exercised


def test_linear_in_features(orc):
    s = synth.tiny_scene(seed=13)
    cam = synth.tiny_camera()
    f2 = np.random.default_rng(1).standard_normal(s.features.shape).astype(np.float32)
    r1 = orc.render(s, cam)
    r2 = orc.render(Scene(s.means, s.log_scales, s.quats, s.opacity, s.colors, f2), cam)
    r3 = orc.render(Scene(s.means, s.log_scales, s.quats, s.opacity, s.colors,
                          (2 * s.features.astype(np.float64) - 3 * f2.astype(np.float64))), cam)
    np.testing.assert_allclose(r3.out[4:], 2 * r1.out[4:] - 3 * r2.out[4:], atol=1e-10)


@pytest.mark.parametrize("stride,oy,ox", [(1, 0, 0), (2, 1, 1), (4, 3, 0)])
def test_tiled_equals_untiled_brute_force(orc, stride, oy, ox):
    """Every pixel walking all visible Gaussians in (depth, index) order gives
    the same image as the tiled walk: the opacity-aware box drops only pairs
    with alpha < 1/255."""
    s = synth.tiny_scene(seed=14, n=1500)
    cam = synth.tiny_camera().with_grid(stride, oy, ox)
    r = orc.render(s, cam)
    vis = np.nonzero(r.proj.visible)[0]
    db = r.proj.depth.astype(np.float32).view(np.uint32)
    order = np.array(sorted(vis, key=lambda i: (int(db[i]), i)), np.uint32)
    out, fT = orc.composite_list(r.proj, s.opacity, r.chan, order, cam)
    np.testing.assert_allclose(out, r.out, rtol=0, atol=1e-12)
    np.testing.assert_allclose(fT, r.final_T, rtol=0, atol=1e-12)


def test_sampled_grid_picks_dense_pixels(orc):
    """Rendering at stride s and offset o gives the dense image's pixels
    (o_h + m s, o_w + n s) (Eq. sampled_loc)."""
    s = synth.tiny_scene(seed=15, n=800)
    dense = orc.render(s, synth.tiny_camera()).out
    for stride, oy, ox in ((2, 0, 1), (3, 2, 2), (5, 4, 3)):
        sp = orc.render(s, synth.tiny_camera().with_grid(stride, oy, ox)).out
        ref = dense[:, oy::stride, ox::stride]
        np.testing.assert_allclose(sp[:, :ref.shape[1], :ref.shape[2]], ref, rtol=0, atol=1e-12)


def test_tile_list_composite_equals_full_frame(orc):
    """The compact per-tile walk writes the same values as the full frame."""
    s = synth.tiny_scene(seed=16, n=900)
    cam = synth.tiny_camera().with_grid(2, 1, 0)
    hs, ws, ty, tx = orc.grid_info(cam)
    r = orc.render(s, cam)
    tiles = [0, 3, tx * ty - 1, tx]
    pr, out, fT, amb = orc.render_tiles(s, cam, tiles)
    np.testing.assert_array_equal(out, orc.tile_view(r.out, cam, tiles))
    np.testing.assert_array_equal(amb[:, 3], orc.tile_view(r.amb[3], cam, tiles))
    np.testing.assert_array_equal(orc.untile(out, cam, tiles), r.out * orc.untile(np.ones((len(tiles), 16, 16)), cam, tiles)[None])
    ft = orc.tile_view(r.final_T, cam, tiles)
    inside = orc.tile_view(np.ones((hs, ws)), cam, tiles) == 1
    np.testing.assert_array_equal(fT[inside], ft[inside])
