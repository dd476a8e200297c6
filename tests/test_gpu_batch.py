"""Batched render requests (the serving form's launches keyed by (slot,
tile, depth)): one projection, one tile sort and one compositing launch for
several requests of different scenes, poses and resolutions.  Each request's
image, final transmittance and n_last must equal, bit for bit, what it gets
rendered alone; one batched request is also checked against the FP64
oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import E2E, ambiguous, gaussians, np_, rel_max, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def alone(xgs, g, cam):
    c = xgs.camera_from(cam)
    p = xgs.xgs_project(g, c)
    m = int(p.tiles_touched.to(torch.int64).sum().item())
    b = xgs.alloc_binning(g.n, max(m, 1), c)
    xgs.xgs_tile_sort(p, c, g.n, b)
    out, fT, nl = xgs.xgs_render_fwd(g, p, b, c)
    return out, fT, nl


def test_batch_equals_each_request_alone(xgs):
    poses = synth.room_trajectory(100, seed=10)
    rooms = [synth.room_scene(n, seed=40 + k, c_sem=16) for k, n in enumerate((100_000, 250_000))]
    gs = [gaussians(s, xgs) for s in rooms]
    reqs = [
        (gs[0], synth.room_camera(640, 480, 525.0, poses[3])),
        (gs[1], synth.room_camera(1200, 680, 600.0, poses[40])),
        (gs[0], synth.room_camera(320, 240, 262.5, poses[77])),          # same scene again, other pose
        (gs[1], synth.room_camera(640, 480, 525.0, poses[12]).with_grid(3, 2, 1)),  # sampled grid
    ]
    print(f"batch of {len(reqs)} requests", flush=True)
    outs, b = xgs.render_batch(reqs, tiles_x=75, tile_rows=160, cap_gaussians=800_000)
    torch.cuda.synchronize()
    assert int(np_(b.status)[0]) == 0
    for k, (g, cam) in enumerate(reqs):
        ref = alone(xgs, g, cam)
        torch.cuda.synchronize()
        for a, r in zip(outs[k], ref):
            np.testing.assert_array_equal(np_(a), np_(r), err_msg=f"request {k}")


def test_eight_slot_batch_equals_each_request_alone(xgs):
    """Eight requests (three scenes, the three serving resolutions, two grid
    strides) in one batch: a 75 x 179 virtual grid whose narrower slots leave
    runs of empty tiles (the order kernel's one-key steps); every request
    bitwise as rendered alone."""
    poses = synth.room_trajectory(100, seed=10)
    rooms = [synth.room_scene(n, seed=50 + k, c_sem=16) for k, n in enumerate((60_000, 150_000, 300_000))]
    gs = [gaussians(s, xgs) for s in rooms]
    res = [(320, 240, 262.5), (640, 480, 525.0), (1200, 680, 600.0)]
    reqs = []
    for k in range(8):
        w, h, f = res[k % 3]
        cam = synth.room_camera(w, h, f, poses[(11 * k + 3) % 100])
        if k in (2, 5):
            cam = cam.with_grid(2, k % 2, 1)
        reqs.append((gs[k % 3], cam))
    print(f"batch of {len(reqs)} requests", flush=True)
    outs, b = xgs.render_batch(reqs, tiles_x=75)
    torch.cuda.synchronize()
    assert int(np_(b.status)[0]) == 0
    assert int(b.ranges.shape[0]) == 75 * 179
    for k, (g, cam) in enumerate(reqs):
        ref = alone(xgs, g, cam)
        torch.cuda.synchronize()
        for a, r in zip(outs[k], ref):
            np.testing.assert_array_equal(np_(a), np_(r), err_msg=f"request {k}")


def test_batch_with_an_empty_slot_and_unused_capacity(xgs):
    s = synth.tiny_scene(seed=0, n=2000)
    g = gaussians(s, xgs)
    empty = xgs.Gaussians(g.means[:0], g.log_scales[:0], g.quats[:0], g.opacity[:0], g.colors[:0],
                          g.features[:0])
    cam = synth.tiny_camera()
    outs, b = xgs.render_batch([(empty, cam), (g, cam)], tiles_x=9, tile_rows=20, cap_gaussians=5000)
    torch.cuda.synchronize()
    assert float(np_(outs[0][0]).max()) == 0.0 and np.all(np_(outs[0][1]) == 1.0) and np.all(np_(outs[0][2]) == 0)
    ref = alone(xgs, g, cam)
    torch.cuda.synchronize()
    for a, r in zip(outs[1], ref):
        np.testing.assert_array_equal(np_(a), np_(r))


def test_batched_request_matches_oracle(xgs):
    """The tiny scene in slot 1 of a batch (after a room request): image
    within 1e-4 relative max of the FP64 oracle outside the ambiguity bands,
    n_last equal there."""
    s = synth.tiny_scene(seed=0)
    room = synth.room_scene(100_000, seed=40, c_sem=8)
    cam = synth.tiny_camera()
    reqs = [(gaussians(room, xgs), synth.room_camera(320, 240, 262.5, synth.room_trajectory(100, seed=10)[5])),
            (gaussians(s, xgs), cam)]
    outs, _ = xgs.render_batch(reqs, tiles_x=20, tile_rows=21, cap_gaussians=102_000)
    torch.cuda.synchronize()
    ref = oracle.render(s, cam)
    amb = ambiguous(ref, E2E)
    out = np_(outs[1][0])
    err = rel_max(out, ref.out, amb)
    print(f"batched tiny request vs oracle: rel max {err:.2e}, {amb.mean():.4f} masked")
    assert err < 1e-4
    np.testing.assert_array_equal(np_(outs[1][2])[~amb], ref.n_last[~amb])
