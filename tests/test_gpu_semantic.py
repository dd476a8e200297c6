"""Semantic phase on the GPU (f1): mixture-weight softmax, the fused decode +
masked cosine/L1 loss, and dL/dz through the feature-only backward, against
the FP64 oracle (Sec. 3.2.2, App. D, App. E)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import ambiguous, gaussians, np_, rel_l2, rel_max, require_gpu, run_render

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
    assert rel_max(np_(dz), oracle.semantic_softmax_bwd(wr, dw)) < 2e-5


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
    """The decode + loss kernel at the mapping-scale grid (640x480, L = 16
    mixture weights, D = 512 targets from the FP64 bilinear sample of a
    512x30x40 map, a blocky validity mask): loss and every gradient row
    against the oracle on the same seeded map."""
    rng = np.random.default_rng(9)
    L, D, H, W = 16, 512, 480, 640
    wmap = rng.dirichlet(np.ones(L), H * W).T.reshape(L, H, W).astype(np.float32)
    wmap = np.concatenate([rng.random((4, H, W)).astype(np.float32), wmap])
    E = rng.standard_normal((L, D)).astype(np.float32)
    Gs, _ = oracle.grid_sample(synth.feature_map(D, 30, 40, seed=5), H, W)
    Gs = Gs.astype(np.float32)
    yy, xx = np.mgrid[0:H, 0:W]
    V = (((yy // 60) + (xx // 80)) % 3 != 0).astype(np.uint8)   # blocky "annotated regions"
    loss, d_out = xgs.xgs_semantic_loss(t(wmap), t(E), t(Gs), t(V, np.uint8), 1.0)
    torch.cuda.synchronize()
    ref, dref = oracle.semantic_loss(wmap[4:], E, Gs, V, 1.0)
    assert abs(float(np_(loss)[0]) - ref) <= 2e-5 * abs(ref)
    d = np_(d_out)
    assert np.all(d[:4] == 0)
    # The L1 term's derivative sign(a - b) jumps at a = b: a pixel with a
    # component whose decoded value is within FP32 rounding of its target may
    # take either sign (both are correct), so such pixels are left out.
    amb = np.zeros((H, W), bool)
    for y0 in range(0, H, 60):
        a = E.T.astype(np.float64) @ wmap[4:, y0:y0 + 60].reshape(L, -1).astype(np.float64)
        b = Gs[:, y0:y0 + 60].reshape(D, -1).astype(np.float64)
        amb[y0:y0 + 60] = (np.abs(a - b) <= 4e-6 * (np.abs(a) + np.abs(b) + 1.0)).any(0).reshape(-1, W)
    print(f"decode + loss 640x480: {int(amb.sum())} pixels with a near-zero L1 difference left out")
    assert amb.mean() < 0.01
    assert rel_max(d[4:], dref, amb) < 1e-4


def test_semantic_phase_640x480_dz_matches_oracle(xgs):
    """The whole phase on the 300k room at 640x480 (softmax -> render ->
    decode + loss -> feature-only backward -> softmax backward) against the
    oracle's FP64 phase on 96 random tiles: the validity mask keeps those
    tiles' pixels whose compositing decisions are not within the FP32
    ambiguity bands, so both sides evaluate the same loss; dL/dz of all
    300,000 Gaussians within 1e-3 relative L2."""
    scene = synth.room_scene(300_000, seed=2, c_sem=16)
    cam = synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[7])
    hs, ws, ty, tx = oracle.grid_info(cam)
    rng = np.random.default_rng(9)
    L, D = 16, 512
    z = (rng.standard_normal((scene.n, L)) * 2).astype(np.float32)
    E = rng.standard_normal((L, D)).astype(np.float32)
    Gs = oracle.grid_sample(synth.feature_map(D, 30, 40, seed=5), 480, 640)[0].astype(np.float32)
    tile_mask = np.zeros(ty * tx, np.uint8)
    tile_mask[np.random.default_rng(11).choice(ty * tx, 96, replace=False)] = 1
    # oracle phase, written out so that the mask can drop ambiguous pixels
    w = oracle.semantic_softmax(z)
    sc = scene.__class__(**{**scene.__dict__, "features": w})
    r = oracle.render(sc, cam, tile_mask)
    yy, xx = np.mgrid[0:hs, 0:ws]
    in_tiles = tile_mask[(yy // 16) * tx + xx // 16] == 1
    V = (in_tiles & ~ambiguous(r) & ((((yy // 60) + (xx // 80)) % 3) != 0)).astype(np.uint8)
    ref, dwmap = oracle.semantic_loss(r.out[4:], E, Gs, V, 1.0)
    gr = oracle.render_grad(sc, cam, np.concatenate([np.zeros((4, hs, ws)), dwmap]), r, tile_mask=tile_mask)
    dz_ref = oracle.semantic_softmax_bwd(w, gr.features)
    g = gaussians(scene, xgs)
    rg = run_render(xgs, scene, cam, g=g)
    loss, dz, out = xgs.semantic_step(g, rg["p"], rg["b"], rg["cam"], t(z), t(E), t(Gs), t(V, np.uint8), 1.0)
    torch.cuda.synchronize()
    e_map = rel_max(np_(out)[4:][:, V == 1], r.out[4:][:, V == 1])
    e_loss = abs(float(np_(loss)[0]) - ref) / abs(ref)
    e_dz = rel_l2(np_(dz), dz_ref)
    print(f"semantic phase 640x480: {int(V.sum())} valid px, map {e_map:.2e}, loss {e_loss:.2e}, dL/dz {e_dz:.2e}")
    assert e_map < 1e-4 and e_loss < 1e-4 and e_dz < 1e-3
    assert np.count_nonzero(dz_ref) > 10_000
