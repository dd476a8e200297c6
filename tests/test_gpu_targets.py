"""Region-indexed grid targets and occluder pruning on the GPU (f4) against
the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import np_, require_gpu, run_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("H,W,R,D,s,oy,ox", [(7, 9, 4, 3, 3, 2, 1), (48, 64, 10, 16, 1, 0, 0),
                                            (480, 640, 100, 512, 1, 0, 0), (481, 643, 37, 20, 4, 3, 1)])
def test_region_targets_bitexact(xgs, H, W, R, D, s, oy, ox):
    rng = np.random.default_rng(H + R)
    S = rng.integers(-1, R + 2, (H, W)).astype(np.int32)   # includes labels >= R
    Phi = rng.standard_normal((R, D)).astype(np.float32)
    G, V = xgs.xgs_region_targets(t(S, np.int32), t(Phi), s, oy, ox)
    torch.cuda.synchronize()
    Gr, Vr = oracle.region_targets(S, Phi, s, oy, ox)
    np.testing.assert_array_equal(np_(V), Vr)
    np.testing.assert_array_equal(np_(G), Gr.astype(np.float32))


def test_occluder_mask_matches_the_rule_on_the_oracles_projection(xgs):
    """Staged: both sides apply the rule in binary32 to the oracle's projection
    rounded to binary32 (the decision is an integer function of those
    values), against a depth map made from the oracle's render pushed back by
    15% on a band."""
    from gpu_util import splat_from_oracle
    scene = synth.room_scene(300_000, seed=2, c_sem=1)
    cam = synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[20])
    pr = oracle.project(scene, cam)
    p, sp = splat_from_oracle(xgs, pr, scene.opacity, scene.n)
    tiles = np.zeros(oracle.grid_info(cam)[2] * oracle.grid_info(cam)[3], np.uint8)
    tiles[::3] = 1
    dm = oracle.render(scene, cam, tiles).out[3].astype(np.float32)
    dm[100:200] *= np.float32(1.15)
    prune, count = xgs.xgs_occluder_mask(p, scene.n, t(dm), 0.1)
    torch.cuda.synchronize()
    vis = pr.visible == 1
    ref = oracle.occluder_mask(sp[:, 0:2], sp[:, 6], vis, dm, np.float32(0.1))
    got = np_(prune)
    np.testing.assert_array_equal(got, ref)
    assert int(np_(count)[0]) == int(ref.sum()) and ref.sum() > 0


def test_occluders_in_front_of_a_wall(xgs):
    from synth import Scene
    cam = synth.tiny_camera()
    rng = np.random.default_rng(2)
    n = 200
    means = np.c_[rng.uniform(-1.5, 1.5, (n, 2)), np.full(n, 4.0)]
    means[:10, 2] = 1.0
    means[:10, :2] *= 0.2
    sc = Scene(means.astype(np.float32), np.full((n, 3), -3.0, np.float32),
               np.tile(np.array([1.0, 0, 0, 0], np.float32), (n, 1)), np.full(n, 0.8, np.float32),
               np.zeros((n, 3), np.float32), np.zeros((n, 1), np.float32))
    r = run_render(xgs, sc, cam)
    prune, count = xgs.xgs_occluder_mask(r["p"], n, t(np.full((cam.height, cam.width), 4.0)), 0.1)
    torch.cuda.synchronize()
    got = np_(prune)
    assert got[:10].all() and not got[10:].any() and int(np_(count)[0]) == 10
