"""Pins of the oracle's grid-sampled targets, VQ assignment and EMA update
(no GPU).

Passages: App. D Eq. (sampled_loc), Eq. (target_continuous) and the mask
paragraph; Sec. 3.2.2 nearest-codeword assignment and Eq. (ema_update).
"""
import os

import numpy as np
import pytest
import torch

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# --------------------------------------------------------------- grid sample
def torch_ref(P, H, W, stride, oy, ox, mode):
    D, Hf, Wf = P.shape
    Hs, Ws = -(-H // stride), -(-W // stride)
    u = oy + np.arange(Hs) * stride
    v = ox + np.arange(Ws) * stride
    uu = u * (Hf - 1) / max(H - 1, 1)
    vv = v * (Wf - 1) / max(W - 1, 1)
    gy = 2 * uu / (Hf - 1) - 1 if Hf > 1 else np.zeros_like(uu, dtype=np.float64)
    gx = 2 * vv / (Wf - 1) - 1 if Wf > 1 else np.zeros_like(vv, dtype=np.float64)
    grid = np.stack(np.broadcast_arrays(gx[None, :], gy[:, None]), -1)[None]
    out = torch.nn.functional.grid_sample(torch.from_numpy(P.astype(np.float64))[None],
                                          torch.from_numpy(grid), mode=mode, align_corners=True)
    valid = (u[:, None] < H) & (v[None, :] < W)
    return np.where(valid[None], out[0].numpy(), 0.0), valid


@pytest.mark.parametrize("H,W,Hf,Wf,stride,oy,ox", [
    (480, 640, 30, 40, 1, 0, 0), (96, 128, 7, 9, 3, 2, 1), (50, 70, 13, 5, 4, 3, 3), (17, 1, 4, 1, 2, 1, 0)])
def test_bilinear_matches_torch_grid_sample(orc, H, W, Hf, Wf, stride, oy, ox):
    P = synth.feature_map(6, Hf, Wf, seed=H)
    G, V = orc.grid_sample(P, H, W, stride, oy, ox, orc.BILINEAR)
    ref, valid = torch_ref(P, H, W, stride, oy, ox, "bilinear")
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(V, valid)


def test_nearest_matches_golden_table_and_torch(orc):
    """Eq. (target_continuous) for 640x480 and a 40x30 map: the stored index
    table (exact rationals) and torch's nearest mode away from exact halves."""
    with open(os.path.join(GOLDEN, "nearest_index_table.txt")) as f:
        lines = [l for l in f if not l.startswith("#")]
    rows = np.array(lines[0].split(), int)
    cols = np.array(lines[1].split(), int)
    D, Hf, Wf = 3, 30, 40
    P = np.arange(D * Hf * Wf, dtype=np.float32).reshape(D, Hf, Wf)
    G, V = orc.grid_sample(P, 480, 640, 1, 0, 0, orc.NEAREST)
    np.testing.assert_array_equal(G, P[:, rows[:, None], cols[None, :]])
    assert V.all()
    ref, _ = torch_ref(P, 480, 640, 1, 0, 0, "nearest")
    np.testing.assert_array_equal(G, ref)


def test_same_size_is_a_copy_and_corners(orc):
    P = synth.feature_map(4, 9, 11, seed=2)
    for mode in (orc.BILINEAR, orc.NEAREST):
        G, V = orc.grid_sample(P, 9, 11, 1, 0, 0, mode)
        np.testing.assert_array_equal(G, P)
        G, _ = orc.grid_sample(P, 95, 131, 1, 0, 0, mode)
        for (a, b), (c, d) in (((0, 0), (0, 0)), ((-1, -1), (-1, -1)), ((0, -1), (0, -1)), ((-1, 0), (-1, 0))):
            np.testing.assert_array_equal(G[:, a, b], P[:, c, d])


def test_constant_and_affine_maps_exact(orc):
    P = synth.affine_feature_map(5, 9, 17)
    # H-1 = 8*(Hf-1) and W-1 = 4*(Wf-1): coordinates are dyadic, so exact
    G, _ = orc.grid_sample(P, 65, 65, 1, 0, 0, orc.BILINEAR)
    a, b, c = (np.random.default_rng(6).integers(-4, 5, (3, 5))).astype(np.float64)
    u = np.arange(65) * 8 / 64
    v = np.arange(65) * 16 / 64
    want = a[:, None, None] + b[:, None, None] * u[None, :, None] + c[:, None, None] * v[None, None, :]
    np.testing.assert_array_equal(G, want)
    K = np.full((2, 5, 6), 3.25, np.float32)
    G, V = orc.grid_sample(K, 37, 41, 3, 1, 2, orc.BILINEAR)
    # constant map: weights sum to one, so only rounding separates G from 3.25
    np.testing.assert_allclose(G, np.broadcast_to(np.where(V[None] == 1, 3.25, 0.0), G.shape), rtol=4e-16, atol=0)
    assert V.sum() == 12 * 13


def test_out_of_bounds_mask(orc):
    """Fixed H_s x W_s = ceil(H/s) x ceil(W/s); grid points past the image are
    padded: V = 0 and G = 0 (App. D, mask paragraph)."""
    P = synth.feature_map(2, 5, 5, seed=1)
    G, V = orc.grid_sample(P, 10, 10, 4, 3, 2, orc.BILINEAR)
    assert G.shape == (2, 3, 3)
    # rows u = 3, 7, 11 ; cols v = 2, 6, 10
    np.testing.assert_array_equal(V, [[1, 1, 0], [1, 1, 0], [0, 0, 0]])
    assert not G[:, 2, :].any() and not G[:, :, 2].any()


# ------------------------------------------------------------------------ VQ
def test_vq_matches_cdist_and_brute_force(orc):
    X = synth.vq_mixture(3000, 64, 16, seed=2)
    E = synth.vq_codebook(128, 64, 16, seed=3, centre_seed=2)
    idx, d1, d2 = orc.vq_assign(X, E)
    dist = torch.cdist(torch.from_numpy(X.astype(np.float64)), torch.from_numpy(E.astype(np.float64))) ** 2
    ref = dist.argmin(1).numpy()
    gap = (d2 - d1) / np.maximum(d1, 1e-300)
    agree = (idx == ref) | (gap < 1e-9)
    assert agree.all()
    np.testing.assert_allclose(d1, dist.min(1).values.numpy(), rtol=1e-10)
    # tiny brute force with Python loops
    Xs, Es = X[:20, :8], E[:9, :8]
    i2, _, _ = orc.vq_assign(Xs, Es)
    for n in range(20):
        ds = [sum((float(Xs[n, d]) - float(Es[l, d])) ** 2 for d in range(8)) for l in range(9)]
        assert i2[n] == min(range(9), key=lambda l: (ds[l], l))


def test_vq_ties_go_to_lowest_index(orc):
    E = np.array([[1, 0], [0, 1], [1, 0], [0, 1]], np.float32)
    X = np.array([[1, 0], [0, 1], [0.5, 0.5]], np.float32)
    idx, _, _ = orc.vq_assign(X, E)
    assert list(idx) == [0, 1, 0]


# ----------------------------------------------------------------------- EMA
def test_ema_constant_input_closed_form(orc):
    """Repeating the same assignment t times: N_t = l^t N_0 + (1 - l^t) c and
    (paper mode) a never-assigned code keeps E = l^t E_0 / (l^t + eps)."""
    rng = np.random.default_rng(0)
    K, D = 6, 4
    E0 = rng.standard_normal((K, D))
    X = rng.standard_normal((30, D))
    idx = rng.integers(0, K - 1, 30)  # code K-1 never assigned
    lam, eps = 0.9, 1e-3
    N, M = orc.ema_init(E0)
    c = np.bincount(idx, minlength=K).astype(float)
    for t in range(1, 8):
        N, M, E, cnt, _ = orc.ema_update(X, idx, N, M, lam, eps, orc.PAPER)
        np.testing.assert_allclose(N, lam ** t * 1.0 + (1 - lam ** t) * c, rtol=1e-12)
        np.testing.assert_allclose(E[K - 1], lam ** t * E0[K - 1] / (lam ** t + eps), rtol=1e-12)


def test_ema_hand_computed_two_codes(orc):
    """K = 2, D = 2, three rows, decay 0.5, eps 0.1, worked by hand from
    Eq. (ema_update): c = (2, 1), s = ((8, 2), (0, 4)), N = (1.5, 1.0),
    M = ((4.5, 1), (0, 3)).  PAPER: E = M / (N + eps).  LAPLACE: n = 2.5,
    Ntilde = (N + eps) / (n + 2 eps) n = (1.6, 1.1) * 2.5 / 2.7."""
    E0 = np.array([[1.0, 0.0], [0.0, 2.0]])
    X = np.array([[3.0, 1.0], [5.0, 1.0], [0.0, 4.0]])
    idx = np.array([0, 0, 1])
    N, M = orc.ema_init(E0)
    Np, Mp, Ep, cnt, sums = orc.ema_update(X, idx, N, M, 0.5, 0.1, orc.PAPER)
    np.testing.assert_array_equal(cnt, [2.0, 1.0])
    np.testing.assert_array_equal(sums, [[8.0, 2.0], [0.0, 4.0]])
    np.testing.assert_array_equal(Np, [1.5, 1.0])
    np.testing.assert_array_equal(Mp, [[4.5, 1.0], [0.0, 3.0]])
    np.testing.assert_allclose(Ep, [[2.8125, 0.625], [0.0, 3.0 / 1.1]], rtol=1e-15)
    _, _, El, _, _ = orc.ema_update(X, idx, N, M, 0.5, 0.1, orc.LAPLACE)
    # E_0 = (4.5, 1) * 2.7 / (1.6 * 2.5) = (3.0375, 0.675); E_1 = (0, 3) * 2.7 / (1.1 * 2.5)
    np.testing.assert_allclose(El, [[3.0375, 0.675], [0.0, 8.1 / 2.75]], rtol=1e-15)


def test_ema_conservation_and_laplace_mass(orc):
    X = synth.vq_mixture(2000, 16, 8, seed=4)
    E0 = synth.vq_codebook(32, 16, 8, seed=5, centre_seed=4)
    idx, _, _ = orc.vq_assign(X, E0)
    N, M = orc.ema_init(E0)
    N1, M1, E1, cnt, sums = orc.ema_update(X, idx, N, M, 0.99, 1e-5, orc.LAPLACE)
    assert cnt.sum() == len(X)
    np.testing.assert_allclose(sums.sum(0), X.astype(np.float64).sum(0), rtol=1e-12, atol=1e-12)
    # Laplace smoothing redistributes the counts without changing their total:
    # the per-code divisors M_l / E_l sum to sum_l N_l, and each divisor is
    # N_l shifted towards the mean by eps
    div = (M1 / E1)[:, 0]
    np.testing.assert_allclose(M1 / E1, np.repeat(div[:, None], 16, 1), rtol=1e-12)
    assert div.sum() == pytest.approx(N1.sum(), rel=1e-13)
    assert np.all(np.sign(div - N1) == np.sign(N1.mean() - N1))
    # with no samples the EMA only decays
    N2, M2, _, _, _ = orc.ema_update(X[:0], idx[:0], N, M, 0.99, 1e-5, orc.LAPLACE)
    np.testing.assert_allclose(N2, 0.99 * N)
