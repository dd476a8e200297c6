"""Pins of the oracle's semantic phase (Sec. 3.2.2 online VQ mixture weights,
App. D masked loss, App. E per-pixel decode) against closed forms, invariants
and finite differences."""
import numpy as np
import pytest

import oracle
import synth


def small_case(seed=0, L=5, D=7, H=4, W=6, frac=0.7):
    rng = np.random.default_rng(seed)
    wm = rng.random((L, H, W))
    E = rng.standard_normal((L, D))
    Gs = rng.standard_normal((D, H, W))
    V = rng.random((H, W)) < frac
    return wm, E, Gs, V


def test_loss_gradient_matches_central_differences():
    wm, E, Gs, V = small_case()
    lam = 0.7
    _, dw = oracle.semantic_loss(wm, E, Gs, V, lam)
    h = 1e-6
    num = np.zeros_like(wm)
    for idx in np.ndindex(wm.shape):
        a = wm.copy(); a[idx] += h
        b = wm.copy(); b[idx] -= h
        num[idx] = (oracle.semantic_loss(a, E, Gs, V, lam)[0] - oracle.semantic_loss(b, E, Gs, V, lam)[0]) / (2 * h)
    assert np.abs(num - dw).max() < 1e-8 * max(1.0, np.abs(dw).max())
    # pixels outside the mask get no gradient
    assert np.all(dw[:, ~V] == 0)


def test_exact_targets_give_zero_loss_and_gradient():
    # dyadic weights and integer codewords: the decode is exact in binary64,
    # so the targets equal it bit for bit (L1 has no gradient at 0 only then)
    wm, E, _, V = small_case(1)
    wm = np.round(wm * 4) / 4
    E = np.round(E * 3)
    Gs = np.einsum("ld,lhw->dhw", E, wm)  # the decoded map itself
    val, dw = oracle.semantic_loss(wm, E, Gs, V, 1.0)
    assert abs(val) < 1e-12
    assert np.abs(dw).max() < 1e-12


def test_positive_multiple_target_closed_form():
    # cos = 1 exactly, so only L1 remains: mean |G^ - 2 G^| = mean |G^|
    wm, E, _, V = small_case(2)
    A = np.einsum("ld,lhw->dhw", E, wm)
    val, _ = oracle.semantic_loss(wm, E, 2.0 * A, V, 0.5)
    n, D = V.sum(), E.shape[1]
    assert val == pytest.approx(0.5 * np.abs(A[:, V]).sum() / (n * D), rel=1e-12)


def test_orthogonal_equal_norm_target():
    # one valid pixel, G* orthogonal to G^ with the same norm: cos = 0
    E = np.eye(2)
    wm = np.array([[[1.0]], [[0.0]]])            # G^ = (1, 0)
    Gs = np.array([[[0.0]], [[1.0]]])            # G* = (0, 1)
    val, _ = oracle.semantic_loss(wm, E, Gs, np.ones((1, 1), bool), 1.0)
    assert val == pytest.approx(1.0 + (1.0 + 1.0) / 2.0, rel=1e-15)


def test_mask_semantics():
    wm, E, Gs, V = small_case(3)
    val0, dw0 = oracle.semantic_loss(wm, E, Gs, np.zeros_like(V), 1.0)
    assert val0 == 0.0 and np.all(dw0 == 0)
    # targets under the mask do not matter
    Gs2 = Gs.copy()
    Gs2[:, ~V] = 1e3
    assert oracle.semantic_loss(wm, E, Gs2, V, 1.0)[0] == oracle.semantic_loss(wm, E, Gs, V, 1.0)[0]


def test_softmax_and_its_backward():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((6, 5)) * 3
    w = oracle.semantic_softmax(z)
    assert np.allclose(w.sum(1), 1.0, atol=1e-15) and np.all(w > 0)
    assert np.allclose(oracle.semantic_softmax(z + 7.0), w, atol=1e-15)  # shift invariance
    dw = rng.standard_normal(w.shape)
    dz = oracle.semantic_softmax_bwd(w, dw)
    h = 1e-6
    for i, j in [(0, 0), (2, 3), (5, 4)]:
        a = z.copy(); a[i, j] += h
        b = z.copy(); b[i, j] -= h
        num = ((oracle.semantic_softmax(a) - oracle.semantic_softmax(b)) * dw).sum() / (2 * h)
        assert num == pytest.approx(dz[i, j], abs=1e-8)


@pytest.fixture(scope="module")
def phase_case():
    scene = synth.tiny_scene(seed=5, n=300, c_sem=1)
    cam = synth.tiny_camera()
    rng = np.random.default_rng(6)
    L, D = 6, 9
    z = rng.standard_normal((scene.n, L)) * 2
    E = rng.standard_normal((L, D))
    hs, ws, _, _ = oracle.grid_info(cam)
    Gs = rng.standard_normal((D, hs, ws))
    V = rng.random((hs, ws)) < 0.8
    return scene, cam, z, E, Gs, V


def test_rendered_weights_sum_to_coverage(phase_case):
    scene, cam, z, E, Gs, V = phase_case
    _, _, wmap = oracle.semantic_phase(scene, cam, z, E, Gs, V)
    sc = scene.__class__(**{**scene.__dict__, "features": oracle.semantic_softmax(z)})
    r = oracle.render(sc, cam)
    assert np.abs(wmap.sum(0) - (1.0 - r.final_T)).max() < 1e-12


def test_phase_gradient_matches_central_differences(phase_case):
    """Geometry is frozen, so the rendered map is linear in the features and
    no skip/stop decision depends on z: central differences are exact up to
    rounding."""
    scene, cam, z, E, Gs, V = phase_case
    val, dz, _ = oracle.semantic_phase(scene, cam, z, E, Gs, V, 0.8)
    big = np.argsort(-np.abs(dz).sum(1))[:4]
    h = 1e-5
    for i in big:
        for j in (0, 3):
            a = z.copy(); a[i, j] += h
            b = z.copy(); b[i, j] -= h
            num = (oracle.semantic_phase(scene, cam, a, E, Gs, V, 0.8)[0] -
                   oracle.semantic_phase(scene, cam, b, E, Gs, V, 0.8)[0]) / (2 * h)
            assert num == pytest.approx(dz[i, j], rel=1e-5, abs=1e-9)
