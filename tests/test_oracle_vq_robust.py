"""Pins of the robust online VQ pieces of App. C: the confidence score, the
confidence mask on the EMA statistics, and dead-code reinitialisation."""
import numpy as np
import pytest

import oracle
import synth


def test_confidence_closed_forms():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [3.0, 4.0]], np.float32)
    E = np.array([[1.0, 0.0], [-1.0, 0.0]], np.float32)
    tau = 0.7
    c = oracle.vq_confidence(X, E, tau)
    assert c[0] == pytest.approx(0.5, abs=1e-15)              # equidistant
    assert c[1] == pytest.approx(1.0 / (1.0 + np.exp(-2.0 / tau)), rel=1e-14)
    d0, d1 = np.hypot(2.0, 4.0), np.hypot(4.0, 4.0)
    assert c[2] == pytest.approx(1.0 / (1.0 + np.exp(-(d1 - d0) / tau)), rel=1e-14)
    assert np.all(oracle.vq_confidence(X, E[:1], tau) == 1.0)  # one codeword


def test_confidence_equals_the_softmax_definition():
    X = synth.vq_mixture(200, 16, 8, seed=4)
    E = synth.vq_codebook(33, 16, 8, seed=5, centre_seed=4)
    tau = 0.7
    d = np.sqrt(((X.astype(np.float64)[:, None, :] - E.astype(np.float64)[None]) ** 2).sum(-1))
    z = -d / tau
    p = np.exp(z - z.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    assert np.abs(oracle.vq_confidence(X, E, tau) - p.max(1)).max() < 1e-14
    # invariant under a permutation of the codewords
    perm = np.random.default_rng(0).permutation(33)
    assert np.abs(oracle.vq_confidence(X, E[perm], tau) - p.max(1)).max() < 1e-14


def test_masked_update_limits():
    X = synth.vq_mixture(500, 8, 4, seed=6)
    E = synth.vq_codebook(16, 8, 4, seed=7, centre_seed=6)
    idx, _, _ = oracle.vq_assign(X, E)
    conf = oracle.vq_confidence(X, E, 0.7)
    N0, M0 = oracle.ema_init(E)
    res = synth.vq_mixture(5, 8, 4, seed=8)
    # gamma = 0, delta = 0: exactly the plain EMA step
    Nr, Mr, Er, cr, _ = oracle.ema_update(X, idx, N0, M0, 0.9, 1e-5, oracle.LAPLACE)
    Nm, Mm, Em, cm, dead = oracle.ema_update_robust(X, idx, conf, 0.0, N0, M0, 0.9, 1e-5, oracle.LAPLACE, 0.0, res)
    assert not dead.any()
    np.testing.assert_array_equal(cm, cr)
    assert np.abs(Em - Er).max() == 0.0
    # gamma above every confidence: pure decay, no counts
    Nd, Md, _, cd, _ = oracle.ema_update_robust(X, idx, conf, 1.1, N0, M0, 0.9, 1e-5, oracle.PAPER, 0.0, res)
    assert cd.sum() == 0 and np.allclose(Nd, 0.9 * N0) and np.allclose(Md, 0.9 * M0)
    # the mask keeps exactly the confident samples
    g = float(np.median(conf))
    _, _, _, cg, _ = oracle.ema_update_robust(X, idx, conf, g, N0, M0, 0.9, 1e-5, oracle.PAPER, 0.0, res)
    assert cg.sum() == (conf >= g).sum()


def test_dead_codes_take_reservoir_rows_in_order():
    K, D = 6, 3
    N0 = np.array([5.0, 0.01, 3.0, 0.02, 0.0, 2.0])
    M0 = np.arange(K * D, dtype=np.float64).reshape(K, D)
    X = np.zeros((0, D), np.float32)
    res = np.array([[10.0, 11, 12], [20, 21, 22], [30, 31, 32]])
    N, M, E, c, dead = oracle.ema_update_robust(X, np.zeros(0, np.int64), None, 0.0, N0, M0, 1.0, 1e-5,
                                                oracle.PAPER, 0.5, res, offset=2)
    np.testing.assert_array_equal(dead, [0, 1, 0, 1, 1, 0])
    np.testing.assert_array_equal(M[1], res[2])   # first dead code: row (2 + 0) mod 3
    np.testing.assert_array_equal(M[3], res[0])   # second: (2 + 1) mod 3
    np.testing.assert_array_equal(M[4], res[1])   # third: (2 + 2) mod 3
    assert N[1] == N[3] == N[4] == 1.0 + 1e-5
    np.testing.assert_array_equal(M[[0, 2, 5]], M0[[0, 2, 5]])
    np.testing.assert_allclose(E[1], res[2] / (1.0 + 2e-5), rtol=1e-15)


def test_warm_start_is_the_masked_pass_with_zero_decay():
    X = synth.vq_mixture(400, 8, 4, seed=9)
    E = synth.vq_codebook(12, 8, 4, seed=10, centre_seed=9)
    idx, _, _ = oracle.vq_assign(X, E)
    conf = oracle.vq_confidence(X, E, 0.7)
    g = 0.3
    N, M, _, c, _ = oracle.ema_update_robust(X, idx, conf, g, np.ones(12), E.astype(np.float64), 0.0, 1e-5,
                                             oracle.PAPER, 0.0, X[:2])
    use = conf >= g
    for k in range(12):
        sel = use & (idx == k)
        assert N[k] == sel.sum()
        np.testing.assert_allclose(M[k], X[sel].astype(np.float64).sum(0), atol=1e-12)
