"""Pins of the region-indexed targets (App. D Eq. (target_discrete)) and the
occluder pruning rule (Sec. 3.2.1 mapping, 10% margin)."""
import numpy as np

import oracle


def test_region_targets_hand_case():
    S = np.array([[0, -1, 2], [1, 1, -1]])
    Phi = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    G, V = oracle.region_targets(S, Phi)
    np.testing.assert_array_equal(V, [[1, 0, 1], [1, 1, 0]])
    np.testing.assert_array_equal(G[:, 0, 0], [1, 2])
    np.testing.assert_array_equal(G[:, 0, 2], [5, 6])
    np.testing.assert_array_equal(G[:, 1, 0], [3, 4])
    np.testing.assert_array_equal(G[:, 0, 1], [0, 0])


def test_region_targets_stride_offset_and_padding():
    rng = np.random.default_rng(0)
    S = rng.integers(-1, 4, (7, 9))
    Phi = rng.standard_normal((4, 3))
    G, V = oracle.region_targets(S, Phi, stride=3, off_y=2, off_x=1)
    assert G.shape == (3, 3, 3) and V.shape == (3, 3)
    # grid row 2 sits at image row 8 >= 7: padding, no target
    assert np.all(V[2] == 0) and np.all(G[:, 2] == 0)
    for m in range(2):
        for n in range(3):
            lab = S[2 + 3 * m, 1 + 3 * n]
            assert V[m, n] == (lab >= 0)
            if lab >= 0:
                np.testing.assert_array_equal(G[:, m, n], Phi[lab])
    # labels outside [0, R) count as unannotated
    S2 = S.copy(); S2[S2 == 3] = 7
    _, V2 = oracle.region_targets(S2, Phi[:3])
    assert np.all(V2[S2 == 7] == 0)


def test_region_targets_full_mask_is_a_table_lookup():
    rng = np.random.default_rng(1)
    S = rng.integers(0, 5, (6, 8))
    Phi = rng.standard_normal((5, 4))
    G, V = oracle.region_targets(S, Phi)
    assert V.all()
    np.testing.assert_array_equal(G, Phi[S].transpose(2, 0, 1))


def test_occluder_rule():
    mean2d = np.array([[1.5, 1.5], [1.5, 1.5], [1.5, 1.5], [9.0, 0.0], [-0.5, 1.0], [2.2, 0.7], [0.1, 0.1]])
    depth = np.array([0.85, 0.95, 0.5, 0.1, 0.1, 0.1, 0.1])
    visible = np.array([1, 1, 0, 1, 1, 1, 1], bool)
    Dm = np.ones((3, 4))
    Dm[0, 2] = 0.0        # no depth where Gaussian 5 lands
    got = oracle.occluder_mask(mean2d, depth, visible, Dm, 0.1)
    # 0: 0.85 < 0.9 -> occluder; 1: 0.95 not; 2: culled; 3: outside (x = 9);
    # 4: outside (x < 0); 5: no depth; 6: occluder
    np.testing.assert_array_equal(got, [1, 0, 0, 0, 0, 0, 1])


def test_occluders_of_a_scene_in_front_of_a_wall():
    """Gaussians on a wall at z = 4 plus a few floaters at z = 1: against the
    wall's depth map only the floaters are pruned."""
    import synth
    from synth import Scene
    cam = synth.tiny_camera()
    rng = np.random.default_rng(2)
    n = 200
    means = np.c_[rng.uniform(-1.5, 1.5, (n, 2)), np.full(n, 4.0)]
    means[:10, 2] = 1.0
    means[:10, :2] *= 0.2
    sc = Scene(means, np.full((n, 3), -3.0), np.tile([1.0, 0, 0, 0], (n, 1)), np.full(n, 0.8),
               np.zeros((n, 3)), np.zeros((n, 1)))
    pr = oracle.project(sc, cam)
    Dm = np.full((cam.height, cam.width), 4.0)
    got = oracle.occluder_mask(pr.mean2d, pr.depth, pr.visible, Dm, 0.1)
    assert got[:10].all() and not got[10:].any()
