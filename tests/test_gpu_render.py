"""GPU parity of the rasterizer (a1-a4) against the FP64 oracle, through the
C ABI.  Bars: keys/order/ranges bit-exact; images and features within 1e-4
relative max error over pixels with no ambiguous discrete decision; gradients
within 1e-3 relative L2 against the oracle's analytic gradient and its
central finite differences (h = 1e-3)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (E2E, STAGED, ambiguous, binning_from_oracle, gaussians, np_, rel_l2, rel_max,
                      require_gpu, run_render, splat_from_oracle)

pytestmark = pytest.mark.gpu

GRID_CASES = [(1, 0, 0), (2, 1, 0), (3, 2, 1)]


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


@pytest.fixture(scope="module")
def room300k():
    return synth.room_scene(300_000, seed=1, c_sem=16)


def room_cam(width=640, height=480, f=525.0, frame=5):
    return synth.room_camera(width, height, f, synth.room_trajectory(100, seed=10)[frame])


# ------------------------------------------------------------------ a1
@pytest.mark.parametrize("case", ["tiny", "tiny_grid", "room"])
def test_project_matches_oracle(xgs, room300k, case):
    if case == "room":
        scene, cam = room300k, room_cam()
    else:
        scene, cam = synth.tiny_scene(seed=0), synth.tiny_camera()
        if case == "tiny_grid":
            cam = cam.with_grid(3, 2, 1)
    g = gaussians(scene, xgs)
    p = xgs.xgs_project(g, xgs.camera_from(cam))
    torch.cuda.synchronize()
    ref = oracle.project(scene, cam)
    sp = np_(p.splat)
    vis_g = np_(p.radius) > 0
    vis_o = ref.visible == 1
    both = vis_g & vis_o
    assert both.sum() > 0.2 * scene.n if case != "room" else both.sum() > 1000
    assert rel_max(sp[both, 0:2], ref.mean2d[both]) < 1e-6
    assert rel_max(sp[both, 2:5], ref.conic[both]) < 1e-5
    assert rel_max(sp[both, 6], ref.depth[both]) < 1e-6
    # rectangles: identical except where the FP64 pixel-range boundary sits
    # within a hair of a pixel centre
    rect_g = np_(p.tile_rect).astype(np.int64) & 0xFFFF
    diff = np.nonzero((vis_g != vis_o) | (both & (rect_g != ref.rect).any(1)))[0]
    s = cam.stride
    for i in diff:
        e = []
        for ax, o in ((0, cam.off_x), (1, cam.off_y)):
            for sign in (-1, 1):
                v = (ref.mean2d[i, ax] + sign * ref.ext[i, ax] - o - 0.5) / s
                e.append(abs(v - round(v)))
        assert min(e) < 1e-3, (i, e)
    assert len(diff) <= max(3, 1e-3 * scene.n)


# ------------------------------------------------------------------ a2
def projected_from_oracle(xgs, pr, n):
    p = xgs.Projected.alloc(n)
    splat = np.zeros((n, 8), np.float32)
    splat[:, 6] = pr.depth.astype(np.float32)
    p.splat.copy_(torch.from_numpy(splat))
    p.tile_rect.copy_(torch.from_numpy(pr.rect.astype(np.uint16).view(np.int16)))
    p.tiles_touched.copy_(torch.from_numpy(pr.touched.astype(np.uint32).view(np.int32)))
    p.radius.copy_(torch.from_numpy(pr.visible.astype(np.int32)))
    return p


def check_sort(xgs, pr, cam, n, extra_cap=0):
    hs, ws, ty, tx = oracle.grid_info(cam)
    keys, vals, ranges = oracle.bin_instances(pr.rect, oracle.depth_bits(pr.depth), tx, ty)
    m = len(keys)
    p = projected_from_oracle(xgs, pr, n)
    b = xgs.alloc_binning(n, m + extra_cap, xgs.camera_from(cam))
    xgs.xgs_tile_sort(p, xgs.camera_from(cam), n, b)
    torch.cuda.synchronize()
    assert int(b.status.item()) == 0
    assert int(b.num_instances.item()) == m
    np.testing.assert_array_equal(np_(b.keys)[:m].view(np.uint64), keys)
    np.testing.assert_array_equal(np_(b.vals)[:m].view(np.uint32), vals)
    np.testing.assert_array_equal(np_(b.ranges).view(np.uint32), ranges)
    # scheduling table: a permutation of the tiles, longest lists first in
    # buckets of 16 instances, ties by tile id (identity above 16384 tiles)
    r = np.asarray(ranges, np.int64).reshape(-1, 2)
    T = len(r)
    if T <= 16384:
        bucket = np.minimum((r[:, 1] - r[:, 0]) >> 4, 255)
        want = np.argsort(((255 - bucket) << 16) | np.arange(T), kind="stable")
    else:
        want = np.arange(T)
    np.testing.assert_array_equal(np_(b.tile_order).view(np.uint32), want.astype(np.uint32))
    return m


@pytest.mark.parametrize("stride", [1, 3])
def test_tile_sort_bitexact_tiny(xgs, stride):
    scene, cam = synth.tiny_scene(seed=0), synth.tiny_camera().with_grid(stride, stride - 1, 0)
    check_sort(xgs, oracle.project(scene, cam), cam, scene.n, extra_cap=777)


@pytest.mark.parametrize("extra_cap", [0, 1_600_000])
def test_tile_sort_bitexact_room(xgs, room300k, extra_cap):
    """43-bit keys: five 9-bit radix passes at the exact capacity, six 8-bit
    passes when the capacity needs more than 768 sort blocks; both bit-exact."""
    cam = room_cam()
    m = check_sort(xgs, oracle.project(room300k, cam), cam, room300k.n, extra_cap=extra_cap)
    assert m > 100_000  # spans many sort blocks and all tile bits


def test_tile_sort_bitexact_large_rects_and_ties(xgs):
    """Synthetic rectangles: big ones (thousands of instances per Gaussian),
    exact depth ties broken by index, a ragged tile count."""
    rng = np.random.default_rng(3)
    cam = synth.Camera(width=1000, height=700, fx=500.0, fy=500.0, cx=500.0, cy=350.0)
    hs, ws, ty, tx = oracle.grid_info(cam)
    n = 20_000
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    w = np.where(rng.random(n) < 0.01, rng.integers(1, tx + 1, n), rng.integers(1, 4, n))
    h = np.where(rng.random(n) < 0.01, rng.integers(1, ty + 1, n), rng.integers(1, 4, n))
    x1 = np.minimum(x0 + w, tx); y1 = np.minimum(y0 + h, ty)
    culled = rng.random(n) < 0.1
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    rect[culled] = 0
    depth = rng.choice(np.linspace(0.5, 9.0, 500), n)  # many exact ties
    pr = oracle.Projection(None, None, depth, None, None, rect,
                           ((x1 - x0) * (y1 - y0) * ~culled).astype(np.int64), (~culled).astype(np.int32))
    check_sort(xgs, pr, cam, n)


def test_tile_sort_long_tile_lists(xgs):
    """Four tiles with 10,000+ instances each (sorted as 4,096-key chunks and
    merged), many exact depth ties, plus scattered small rectangles."""
    rng = np.random.default_rng(6)
    cam = synth.Camera(width=640, height=480, fx=500.0, fy=500.0, cx=320.0, cy=240.0)
    hs, ws, ty, tx = oracle.grid_info(cam)
    n = 14_000
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    x1 = np.minimum(x0 + rng.integers(1, 4, n), tx); y1 = np.minimum(y0 + rng.integers(1, 4, n), ty)
    big = np.arange(n) < 10_500
    x0[big], y0[big], x1[big], y1[big] = 3, 2, 5, 4
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    depth = rng.choice(np.linspace(0.5, 9.0, 300), n)
    pr = oracle.Projection(None, None, depth, None, None, rect, ((x1 - x0) * (y1 - y0)).astype(np.int64),
                           np.ones(n, np.int32))
    check_sort(xgs, pr, cam, n)


def test_tile_sort_above_order_table_limit(xgs):
    """17,424 tiles (2100 x 2100): above the 16,384 tiles the order kernel
    sorts, so the table is the identity; keys and ranges stay bit-exact."""
    rng = np.random.default_rng(4)
    cam = synth.Camera(width=2100, height=2100, fx=900.0, fy=900.0, cx=1050.0, cy=1050.0)
    hs, ws, ty, tx = oracle.grid_info(cam)
    assert tx * ty > 16384
    n = 6000
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    x1 = np.minimum(x0 + rng.integers(1, 5, n), tx); y1 = np.minimum(y0 + rng.integers(1, 5, n), ty)
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    depth = rng.uniform(0.5, 9.0, n)
    pr = oracle.Projection(None, None, depth, None, None, rect, ((x1 - x0) * (y1 - y0)).astype(np.int64),
                           np.ones(n, np.int32))
    check_sort(xgs, pr, cam, n)


@pytest.mark.parametrize("m", [1, 63, 64, 2048, 4097])
def test_tile_sort_block_and_wave_boundaries(xgs, m):
    """Instance counts at the radix scatter's boundaries: a lone key, a
    partial and a full first wavefront, one full 2,048-key block, and a block
    more by one key (the last block's later wavefronts hold nothing); every
    Gaussian touches one tile, depths with exact ties."""
    rng = np.random.default_rng(9 + m)
    cam = synth.Camera(width=640, height=480, fx=500.0, fy=500.0, cx=320.0, cy=240.0)
    hs, ws, ty, tx = oracle.grid_info(cam)
    x0 = rng.integers(0, tx, m); y0 = rng.integers(0, ty, m)
    rect = np.stack([x0, y0, x0 + 1, y0 + 1], 1).astype(np.int32)
    depth = rng.choice(np.linspace(0.5, 9.0, 40), m)
    pr = oracle.Projection(None, None, depth, None, None, rect, np.ones(m, np.int64), np.ones(m, np.int32))
    assert check_sort(xgs, pr, cam, m, extra_cap=3000) == m


@pytest.mark.parametrize("size", [(2048, 2048), (2030, 2040)])
def test_tile_sort_order_table_at_its_limit(xgs, size):
    """16,384 and 16,256 tiles: each of the order kernel's 16 wavefronts
    ranks 1,024 (1,016, the last step ragged) tiles; large rectangles crowded
    towards one corner spread the list lengths over 8-10 buckets."""
    rng = np.random.default_rng(8)
    w_px, h_px = size
    cam = synth.Camera(width=w_px, height=h_px, fx=900.0, fy=900.0, cx=w_px / 2, cy=h_px / 2)
    hs, ws, ty, tx = oracle.grid_info(cam)
    assert 16_000 < tx * ty <= 16384
    n = 30_000
    big = rng.random(n) < 0.03
    x0 = np.where(big, (tx * rng.random(n) ** 3).astype(np.int64), rng.integers(0, tx, n))
    y0 = np.where(big, (ty * rng.random(n) ** 3).astype(np.int64), rng.integers(0, ty, n))
    w = np.where(big, rng.integers(1, 41, n), rng.integers(1, 4, n))
    h = np.where(big, rng.integers(1, 41, n), rng.integers(1, 4, n))
    x1 = np.minimum(x0 + w, tx); y1 = np.minimum(y0 + h, ty)
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    depth = rng.uniform(0.5, 9.0, n)
    pr = oracle.Projection(None, None, depth, None, None, rect, ((x1 - x0) * (y1 - y0)).astype(np.int64),
                           np.ones(n, np.int32))
    m = check_sort(xgs, pr, cam, n)
    assert m > 200_000


def test_tile_sort_empty_and_overflow(xgs):
    cam = synth.tiny_camera()
    c = xgs.camera_from(cam)
    p = xgs.Projected.alloc(0)
    b = xgs.alloc_binning(0, 16, c)
    xgs.xgs_tile_sort(p, c, 0, b)
    torch.cuda.synchronize()
    assert int(b.num_instances.item()) == 0 and int(b.status.item()) == 0
    assert not np_(b.ranges).any()
    scene = synth.tiny_scene(seed=0)
    pr = oracle.project(scene, cam)
    p = projected_from_oracle(xgs, pr, scene.n)
    b = xgs.alloc_binning(scene.n, int(pr.touched.sum()) - 1, c)
    xgs.xgs_tile_sort(p, c, scene.n, b)
    torch.cuda.synchronize()
    assert int(b.status.item()) == 1 and int(b.num_instances.item()) == 0
    assert not np_(b.ranges).any()


# ------------------------------------------------------------------ a3
GROUPS = ("means", "log_scales", "quats", "opacity", "colors", "features")


def tile_pixels(mask, cam):
    hs, ws, ty, tx = oracle.grid_info(cam)
    return np.repeat(np.repeat(mask.reshape(ty, tx), 16, 0), 16, 1)[:hs, :ws].astype(bool)


def staged(xgs, scene, cam, tile_mask=None):
    """Both sides composite the oracle's projection rounded to binary32, in the
    oracle's (tile, depth, index) order: only compositing arithmetic differs."""
    n = scene.n
    pr = oracle.project(scene, cam)
    p, sp = splat_from_oracle(xgs, pr, scene.opacity, n)
    hs, ws, ty, tx = oracle.grid_info(cam)
    keys, vals, ranges = oracle.bin_instances(pr.rect, oracle.depth_bits(sp[:, 6]), tx, ty)
    c = xgs.camera_from(cam)
    b = binning_from_oracle(xgs, keys, vals, ranges, n, c)
    g = gaussians(scene, xgs)
    out, fT, nl = xgs.xgs_render_fwd(g, p, b, c)
    torch.cuda.synchronize()
    f64 = lambda a: np.asarray(a, np.float64)
    pr32 = oracle.Projection(f64(sp[:, 0:2]), f64(sp[:, 2:5]), f64(sp[:, 6]), pr.cov2d, pr.ext, pr.rect,
                             pr.touched, pr.visible)
    chan = oracle.channels(scene, pr32.depth)
    ro, rT, rnl, ramb = oracle.composite_fwd(pr32, scene.opacity, chan, vals, ranges, cam, tile_mask)
    ref = oracle.Render(pr32, keys, vals, ranges, ro, rT, rnl, ramb, chan)
    amb = ambiguous(ref, STAGED)
    if tile_mask is not None:
        amb = amb | ~tile_pixels(tile_mask, cam)
    gpu = dict(g=g, p=p, b=b, cam=c, out=out, final_T=fT, n_last=nl)
    return gpu, ref, amb


def check_forward(r, ref, amb, max_masked):
    out = np_(r["out"])
    frac = float(amb.mean())
    errs = {
        "rgb": rel_max(out[:3], ref.out[:3], amb),
        "depth": rel_max(out[3], ref.out[3], amb),
        "sem": rel_max(out[4:], ref.out[4:], amb) if out.shape[0] > 4 else 0.0,
        "T": rel_max(np_(r["final_T"]), ref.final_T, amb),
    }
    print(f"forward rel-max errors {errs}, masked {frac:.5f}")
    for k, v in errs.items():
        assert v <= 1e-4, (k, errs)
    return frac


def compare_forward(xgs, scene, cam, tile_mask=None):
    """End to end: the GPU projects, sorts and composites; the oracle does all
    three in FP64.  Pixels with a decision inside the E2E bands are masked."""
    r = run_render(xgs, scene, cam)
    ref = oracle.render(scene, cam, tile_mask=tile_mask)
    amb = ambiguous(ref, E2E)
    sel = np.ones_like(amb) if tile_mask is None else tile_pixels(tile_mask, cam)
    frac = float((amb & sel).sum() / sel.sum())
    assert frac < 0.05, frac
    check_forward(r, ref, amb | ~sel, 1.0)
    return r, ref, amb | ~sel


@pytest.mark.parametrize("stride,oy,ox", GRID_CASES)
def test_render_fwd_tiny(xgs, stride, oy, ox):
    cam = synth.tiny_camera().with_grid(stride, oy, ox)
    compare_forward(xgs, synth.tiny_scene(seed=0), cam)
    r, ref, amb = staged(xgs, synth.tiny_scene(seed=0), cam)
    assert check_forward(r, ref, amb, 0.01) < 0.01
    np.testing.assert_array_equal(np_(r["n_last"])[~amb], ref.n_last[~amb])


def test_render_fwd_room_300k(xgs, room300k):
    cam = room_cam()
    compare_forward(xgs, room300k, cam)
    r, ref, amb = staged(xgs, room300k, cam)
    assert amb.mean() < 0.01
    check_forward(r, ref, amb, 0.01)
    np.testing.assert_array_equal(np_(r["n_last"])[~amb], ref.n_last[~amb])


def test_render_fwd_room_1m_sampled_tiles(xgs):
    """1M Gaussians, 1200x680, 32 semantic channels: every output pixel of 120
    random tiles (including the ragged last row and column) against the oracle."""
    scene = synth.room_scene(1_000_000, seed=2, c_sem=32)
    cam = room_cam(1200, 680, 600.0, frame=7)
    hs, ws, ty, tx = oracle.grid_info(cam)
    rng = np.random.default_rng(0)
    mask = np.zeros(tx * ty, np.uint8)
    mask[rng.choice(tx * ty, 120, replace=False)] = 1
    mask[tx * ty - 1] = mask[tx - 1] = mask[(ty - 1) * tx] = 1
    compare_forward(xgs, scene, cam, tile_mask=mask)
    r, ref, amb = staged(xgs, scene, cam, tile_mask=mask)
    check_forward(r, ref, amb, 1.0)


def test_render_fwd_empty_scene(xgs):
    scene = synth.tiny_scene(seed=0).subset(np.arange(0))
    r = run_render(xgs, scene, synth.tiny_camera(), max_instances=1)
    assert not np_(r["out"]).any()
    assert (np_(r["final_T"]) == 1).all() and not np_(r["n_last"]).any()


def test_render_tile_order_is_only_a_schedule(xgs, room300k):
    """Compositing in the sorted (longest list first) tile order and in tile id
    order gives bit-identical images; gradients differ only by the order of
    their atomic sums."""
    cam = room_cam()
    r = run_render(xgs, room300k, cam)
    b = r["b"]
    order = np_(b.tile_order).view(np.uint32)
    assert np.array_equal(np.sort(order), np.arange(len(order)))
    ids = xgs.Binning(b.keys, b.vals, b.ranges, b.num_instances, b.status, b.workspace, b.max_instances, None)
    out, fT, nl = xgs.xgs_render_fwd(r["g"], r["p"], ids, r["cam"])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(out), np_(r["out"]))
    np.testing.assert_array_equal(np_(fT), np_(r["final_T"]))
    np.testing.assert_array_equal(np_(nl), np_(r["n_last"]))
    hs, ws, _, _ = oracle.grid_info(cam)
    g = torch.from_numpy(synth.upstream_grad(4 + room300k.c_sem, hs, ws, seed=9)).cuda()
    a = xgs.xgs_render_bwd(r["g"], r["p"], b, r["cam"], g, r["final_T"], r["n_last"])
    c = xgs.xgs_render_bwd(r["g"], r["p"], ids, r["cam"], g, r["final_T"], r["n_last"])
    torch.cuda.synchronize()
    for k in GROUPS:
        assert rel_l2(np_(getattr(a, k)), np_(getattr(c, k))) < 1e-5, k


# ------------------------------------------------------------------ a4
def backward_errors(xgs, r, ref, amb, scene, cam, seed, tile_mask=None, flags=0):
    hs, ws, _, _ = oracle.grid_info(cam)
    g = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=seed)
    g[:, amb] = 0.0
    gr = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], torch.from_numpy(g).cuda(), r["final_T"],
                            r["n_last"], flags=flags)
    torch.cuda.synchronize()
    ref_g = oracle.render_grad(scene, cam, g.astype(np.float64), ref, tile_mask=tile_mask)
    errs = {k: rel_l2(np_(getattr(gr, k)), getattr(ref_g, k)) for k in GROUPS}
    print(f"gradient rel-L2 errors {errs}")
    return errs


@pytest.mark.parametrize("stride,oy,ox", GRID_CASES)
@pytest.mark.parametrize("mode", ["staged", "end_to_end"])
def test_render_bwd_tiny(xgs, stride, oy, ox, mode):
    scene, cam = synth.tiny_scene(seed=3), synth.tiny_camera().with_grid(stride, oy, ox)
    r, ref, amb = staged(xgs, scene, cam) if mode == "staged" else compare_forward(xgs, scene, cam)
    errs = backward_errors(xgs, r, ref, amb, scene, cam, seed=2)
    assert all(v <= 1e-3 for v in errs.values()), errs


@pytest.mark.parametrize("mode", ["staged", "end_to_end"])
def test_render_bwd_room_300k(xgs, room300k, mode):
    cam = room_cam()
    r, ref, amb = staged(xgs, room300k, cam) if mode == "staged" else compare_forward(xgs, room300k, cam)
    errs = backward_errors(xgs, r, ref, amb, room300k, cam, seed=4)
    assert all(v <= 1e-3 for v in errs.values()), errs


def quadrant_boundary_scene(cam, seed, per_quadrant=4, c_sem=8):
    """Splats placed so that their alpha = 1/255 contour just reaches one pixel
    centre of a chosen 8x8 quadrant: the closest centre has q = t (1 - eps),
    t = 2 ln(255 o), eps in [0.002, 0.01], so that pixel takes the splat while
    every other pixel of the quadrant may not.  Flat Gaussians turned about the
    optical axis (identity view) give any 2D covariance A + 0.3 I, independent
    of where the mean sits; directions, anisotropy and angles are random."""
    rng = np.random.default_rng(seed)
    hs, ws, ty, tx = oracle.grid_info(cam)
    s = cam.stride
    quads = [(x, y, qx, qy) for y in range(ty) for x in range(tx) for qy in range(2) for qx in range(2)
             if (y * 16 + qy * 8) < hs and (x * 16 + qx * 8) < ws]
    means, ls, quats, opac = [], [], [], []
    for (x, y, qx, qy) in quads:
        cols = cam.off_x + (x * 16 + qx * 8 + np.arange(8)) * s + 0.5
        rows = cam.off_y + (y * 16 + qy * 8 + np.arange(8)) * s + 0.5
        px, py = np.meshgrid(cols, rows)
        centre = np.array([cols.mean(), rows.mean()])
        k = 0
        while k < per_quadrant:
            a1, a2 = np.exp(rng.uniform(np.log(0.4), np.log(6.0), 2)) * s
            th = rng.uniform(0.0, np.pi)
            R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
            A = R @ np.diag([a1 * a1, a2 * a2]) @ R.T
            conic = np.linalg.inv(A + 0.3 * np.eye(2))
            o = rng.uniform(0.02, 0.99)
            target = 2.0 * np.log(255.0 * o) * (1.0 - rng.uniform(0.002, 0.01))
            phi = rng.uniform(0.0, 2.0 * np.pi)
            d = np.array([np.cos(phi), np.sin(phi)])

            def qmin(r):
                dx, dy = px - centre[0] - r * d[0], py - centre[1] - r * d[1]
                return float((conic[0, 0] * dx * dx + 2 * conic[0, 1] * dx * dy + conic[1, 1] * dy * dy).min())

            lo, hi = 0.0, 400.0 * s
            if not (qmin(lo) < target < qmin(hi)):
                continue
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if qmin(mid) < target else (lo, mid)
            u, v = centre + lo * d
            z = rng.uniform(2.0, 4.0)
            means.append([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z])
            ls.append(np.log([a1 * z / cam.fx, a2 * z / cam.fy, 1e-4 * min(a1, a2) * z / cam.fx]))
            quats.append([np.cos(th / 2), 0.0, 0.0, np.sin(th / 2)])
            opac.append(o)
            k += 1
    n = len(means)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return synth.Scene(f32(means), f32(ls), f32(quats), f32(opac), f32(rng.uniform(0, 1, (n, 3))),
                       f32(rng.standard_normal((n, c_sem))))


@pytest.mark.parametrize("stride,oy,ox", GRID_CASES)
def test_render_quadrant_culling_boundary(xgs, stride, oy, ox):
    """Each wavefront drops the splats that cannot reach alpha >= 1/255 at any
    pixel centre of its 8x8 quadrant.  Splats whose contour only just reaches
    one centre of a quadrant must still be composited there, in the forward
    and the backward pass: a wrongly dropped one changes that pixel by about
    (1/255) T c, far above the 1e-4 bar."""
    cam = synth.tiny_camera().with_grid(stride, oy, ox)
    scene = quadrant_boundary_scene(cam, seed=40 + stride)
    r, ref, amb = staged(xgs, scene, cam)
    assert check_forward(r, ref, amb, 0.01) < 0.01
    np.testing.assert_array_equal(np_(r["n_last"])[~amb], ref.n_last[~amb])
    errs = backward_errors(xgs, r, ref, amb, scene, cam, seed=41)
    assert all(v <= 1e-3 for v in errs.values()), errs



@pytest.mark.parametrize("c_sem", [0, 1, 3, 5, 20, 40, 54])
def test_render_channel_counts(xgs, c_sem):
    """Channel counts outside the common ones: none (RGB + depth only), exact
    widths whose channel rows are padded to whole float4s in the backward
    (1, 3), counts that run on a wider compiled width with the rest masked (5,
    20, 40) and the largest the geometric backward takes (54).  Staged forward
    and backward against the oracle, and the feature-only backward against the
    full one."""
    scene = synth.tiny_scene(seed=11, n=1500, c_sem=c_sem)
    cam = synth.tiny_camera().with_grid(2, 1, 0) if c_sem % 2 else synth.tiny_camera()
    r, ref, amb = staged(xgs, scene, cam)
    assert check_forward(r, ref, amb, 0.01) < 0.01
    errs = backward_errors(xgs, r, ref, amb, scene, cam, seed=12)
    assert all(v <= 1e-3 for v in errs.values()), errs
    if c_sem > 0:
        hs, ws, _, _ = oracle.grid_info(cam)
        g = torch.from_numpy(synth.upstream_grad(4 + c_sem, hs, ws, seed=13)).cuda()
        full = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], g, r["final_T"], r["n_last"])
        feat = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], g, r["final_T"], r["n_last"],
                                  flags=xgs.BWD_FEATURES_ONLY)
        torch.cuda.synchronize()
        assert rel_l2(np_(feat.features), np_(full.features)) < 1e-6

def test_render_bwd_features_only_matches_full(xgs):
    scene, cam = synth.tiny_scene(seed=5), synth.tiny_camera().with_grid(2, 1, 1)
    r = run_render(xgs, scene, cam)
    hs, ws, _, _ = oracle.grid_info(cam)
    g = torch.from_numpy(synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=7)).cuda()
    full = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], g, r["final_T"], r["n_last"])
    feat = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], g, r["final_T"], r["n_last"],
                              flags=xgs.BWD_FEATURES_ONLY)
    torch.cuda.synchronize()
    assert rel_l2(np_(feat.features), np_(full.features)) < 1e-6


def test_render_bwd_against_central_fd(xgs):
    """64 contributing Gaussians of the tiny scene: the GPU gradient against the
    oracle's central differences with h = 1e-3 on every parameter.  A +-h step
    flips alpha-skip decisions on the rim of a splat (a jump of ~T/255 per
    pixel), so the loss is restricted to the pixels whose sequence of blending
    decisions is identical at -h, 0 and +h; the GPU gradient is taken of that
    same restricted loss (upstream gradient zero elsewhere)."""
    scene, cam = synth.tiny_scene(seed=0), synth.tiny_camera()
    hs, ws, ty, tx = oracle.grid_info(cam)
    r = run_render(xgs, scene, cam)
    ref = oracle.render(scene, cam)
    amb = ambiguous(ref, E2E)
    g = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=20)
    g[:, amb] = 0.0
    g64 = g.astype(np.float64)
    gt = torch.from_numpy(g).cuda()
    full = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], gt, r["final_T"], r["n_last"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(20)
    contributing = np.nonzero(np.abs(np_(full.opacity)) > 0)[0]
    chosen = rng.choice(contributing, 64, replace=False)
    h = 1e-3
    base = {k: getattr(scene, k).astype(np.float64) for k in GROUPS}
    got, want = {k: [] for k in base}, {k: [] for k in base}
    for i in chosen:
        x0, y0, x1, y1 = ref.proj.rect[i]
        mask = np.zeros(tx * ty, np.uint8)
        for yy in range(y0, y1):
            mask[yy * tx + x0: yy * tx + x1] = 1
        r0 = oracle.render(scene, cam, tile_mask=mask)
        for k, arr in base.items():
            for j in range(arr.shape[1] if arr.ndim == 2 else 1):
                rs = []
                for sgn in (1, -1):
                    a = {kk: vv.copy() for kk, vv in base.items()}
                    if arr.ndim == 2:
                        a[k][i, j] += sgn * h
                    else:
                        a[k][i] += sgn * h
                    rs.append(oracle.render(synth.Scene(**a), cam, tile_mask=mask))
                if any(not np.array_equal(x.proj.rect[i], ref.proj.rect[i]) for x in rs):
                    continue
                keep = (rs[0].amb[3] == r0.amb[3]) & (rs[1].amb[3] == r0.amb[3]) & tile_pixels(mask, cam)
                gk = g64 * keep[None]
                fd = (oracle.loss(rs[0].out, gk) - oracle.loss(rs[1].out, gk)) / (2 * h)
                gr = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], torch.from_numpy(gk.astype(np.float32)).cuda(),
                                        r["final_T"], r["n_last"])
                gg = np_(getattr(gr, k))
                got[k].append(gg[i, j] if arr.ndim == 2 else gg[i])
                want[k].append(fd)
    errs = {k: rel_l2(got[k], want[k]) for k in base}
    counts = {k: len(want[k]) for k in base}
    print(f"FD rel-L2 errors {errs}, counts {counts}")
    assert all(counts[k] >= 0.9 * 64 * (base[k].shape[1] if base[k].ndim == 2 else 1) for k in base), counts
    assert all(v <= 1e-3 for v in errs.values()), errs


def test_backward_zeroing_as_a_separate_call(xgs):
    """xgs_render_bwd_zero on another stream, then xgs_render_bwd with
    BWD_PREZEROED, gives the gradients of the plain call (the arrays start
    out full of garbage; only the order of the gradient atomics differs)."""
    scene = synth.tiny_scene(seed=3)
    cam = synth.tiny_camera()
    r = run_render(xgs, scene, cam)
    hs, ws, _, _ = oracle.grid_info(cam)
    d_out = torch.from_numpy(synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=5)).cuda()
    for flags in (xgs.BWD_ALL, xgs.BWD_FEATURES_ONLY):
        ref = xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], d_out, r["final_T"], r["n_last"], flags=flags)
        grads = xgs.Gaussians(*(torch.full_like(t, 7.0) for t in (r["g"].means, r["g"].log_scales, r["g"].quats,
                                                                   r["g"].opacity, r["g"].colors, r["g"].features)))
        ws_ = torch.full((int(xgs.lib.xgs_render_bwd_workspace(scene.n)),), 3, dtype=torch.uint8, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        xgs.xgs_render_bwd_zero(r["g"], grads, ws_, flags=flags, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        xgs.xgs_render_bwd(r["g"], r["p"], r["b"], r["cam"], d_out, r["final_T"], r["n_last"],
                           flags=flags | xgs.BWD_PREZEROED, grads=grads, workspace=ws_)
        torch.cuda.synchronize()
        groups = ("features",) if flags == xgs.BWD_FEATURES_ONLY else GROUPS
        for k in groups:
            assert rel_max(np_(getattr(grads, k)), np_(getattr(ref, k))) < 1e-5, (flags, k)
