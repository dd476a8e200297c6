"""Semantic phase on the GPU (f1): mixture-weight softmax, the fused decode +
masked cosine/L1 loss, and dL/dz through the feature-only backward, against
the FP64 oracle (Sec. 3.2.2, App. D, App. E)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gaussians, np_, rel_l2, rel_max, require_gpu, run_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("L", [4, 16, 64])
def test_softmax_and_backward(xgs, L):
    rng = np.random.default_rng(L)
    z = (rng.standard_normal((1000 + 37, L)) * 4).astype(np.float32)
    dw = rng.standard_normal(z.shape).astype(np.float32)
    w = xgs.xgs_semantic_softmax(t(z))
    dz = xgs.xgs_semantic_softmax_bwd(w, t(dw))
    torch.cuda.synchronize()
    wr = oracle.semantic_softmax(z)
    assert rel_max(np_(w), wr) < 2e-6
    assert rel_max(np_(dz), oracle.semantic_softmax_bwd(np_(w), dw)) < 2e-5


@pytest.mark.parametrize("L,D,hs,ws,frac", [(4, 8, 5, 7, 0.6), (16, 512, 37, 53, 0.8), (64, 96, 64, 65, 1.0),
                                            (32, 128, 9, 11, 0.0)])
def test_loss_matches_oracle_on_the_same_map(xgs, L, D, hs, ws, frac):
    """Staged: the kernel and the oracle see the same FP32 map."""
    rng = np.random.default_rng(L + D)
    wmap = rng.random((4 + L, hs, ws)).astype(np.float32)
    E = rng.standard_normal((L, D)).astype(np.float32)
    Gs = rng.standard_normal((D, hs, ws)).astype(np.float32)
    V = (rng.random((hs, ws)) < frac).astype(np.uint8)
    lam = 0.75
    loss, d_out = xgs.xgs_semantic_loss(t(wmap), t(E), t(Gs), t(V, np.uint8), lam)
    torch.cuda.synchronize()
    ref, dref = oracle.semantic_loss(wmap[4:], E, Gs, V, lam)
    d = np_(d_out)
    assert np.all(d[:4] == 0)
    if V.sum() == 0:
        assert float(np_(loss)[0]) == 0.0 and np.all(d == 0)
        return
    assert abs(float(np_(loss)[0]) - ref) <= 1e-5 * abs(ref)
    assert rel_max(d[4:], dref) < 1e-4
    assert np.all(d[4:, V == 0] == 0)


def test_loss_all_valid_when_mask_is_null(xgs):
    rng = np.random.default_rng(5)
    L, D, hs, ws = 8, 64, 20, 30
    wmap = rng.random((4 + L, hs, ws)).astype(np.float32)
    E = rng.standard_normal((L, D)).astype(np.float32)
    Gs = rng.standard_normal((D, hs, ws)).astype(np.float32)
    l0, d0 = xgs.xgs_semantic_loss(t(wmap), t(E), t(Gs), None, 1.0)
    l1, d1 = xgs.xgs_semantic_loss(t(wmap), t(E), t(Gs), t(np.ones((hs, ws)), np.uint8), 1.0)
    torch.cuda.synchronize()
    assert float(np_(l0)[0]) == float(np_(l1)[0])
    np.testing.assert_array_equal(np_(d0), np_(d1))


def test_semantic_phase_end_to_end_tiny(xgs):
    """softmax -> render -> decode + loss -> feature-only backward -> softmax
    backward on the GPU against the oracle's FP64 phase (relative L2 <= 1e-3
    on dL/dz, loss within 1e-4)."""
    scene = synth.tiny_scene(seed=7, n=2000, c_sem=1)
    cam = synth.tiny_camera()
    rng = np.random.default_rng(8)
    L, D = 16, 64
    z = (rng.standard_normal((scene.n, L)) * 2).astype(np.float32)
    E = rng.standard_normal((L, D)).astype(np.float32)
    hs, ws, _, _ = oracle.grid_info(cam)
    Gs = rng.standard_normal((D, hs, ws)).astype(np.float32)
    V = (rng.random((hs, ws)) < 0.85).astype(np.uint8)
    ref, dz_ref, wmap_ref = oracle.semantic_phase(scene, cam, z, E, Gs, V, 0.5)
    sc = scene.__class__(**{**scene.__dict__, "features": np.zeros((scene.n, L), np.float32)})
    r = run_render(xgs, sc, cam)
    loss, dz, out = xgs.semantic_step(r["g"], r["p"], r["b"], r["cam"], t(z), t(E), t(Gs), t(V, np.uint8), 0.5)
    torch.cuda.synchronize()
    assert rel_max(np_(out)[4:], wmap_ref) < 1e-4
    assert abs(float(np_(loss)[0]) - ref) <= 1e-4 * abs(ref)
    assert rel_l2(np_(dz), dz_ref) < 1e-3


def test_semantic_loss_full_grid_640x480(xgs):
    """300k-Gaussian room at 640x480, L = 16 mixture weights, D = 512 targets
    from the bilinear grid sample of a 512x30x40 map, a region-shaped validity
    mask: the kernel's loss and sampled gradient rows against the oracle on
    the same rendered map."""
    scene = synth.room_scene(300_000, seed=2, c_sem=16)
    cam = synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[7])
    rng = np.random.default_rng(9)
    L, D = 16, 512
    z = (rng.standard_normal((scene.n, L)) * 2).astype(np.float32)
    E = rng.standard_normal((L, D)).astype(np.float32)
    P = t(synth.feature_map(D, 30, 40, seed=5))
    Gs, _ = xgs.xgs_grid_sample(P, 480, 640)
    yy, xx = np.mgrid[0:480, 0:640]
    V = (((yy // 60) + (xx // 80)) % 3 != 0).astype(np.uint8)   # blocky "annotated regions"
    g = gaussians(scene, xgs)
    r = run_render(xgs, scene, cam, g=g)
    loss, dz, out = xgs.semantic_step(g, r["p"], r["b"], r["cam"], t(z), t(E), Gs, t(V, np.uint8), 1.0)
    torch.cuda.synchronize()
    _, d_out = xgs.xgs_semantic_loss(out, t(E), Gs, t(V, np.uint8), 1.0)
    torch.cuda.synchronize()
    wmap = np_(out)[4:]
    ref, dref = oracle.semantic_loss(wmap, E, np_(Gs), V, 1.0)
    assert abs(float(np_(loss)[0]) - ref) <= 2e-5 * abs(ref)
    rows = np.random.default_rng(10).choice(480, 24, replace=False)
    assert rel_max(np_(d_out)[4:, rows], dref[:, rows]) < 1e-4
    assert np.isfinite(np_(dz)).all() and np.abs(np_(dz)).max() > 0
