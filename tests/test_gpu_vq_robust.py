"""Robust online VQ on the GPU (f3, App. C): the confidence score fused in the
BF16 sweep, the confidence-masked EMA step and the dead-code reset, against
the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import np_, rel_max, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("n,d,k", [(12_288, 64, 128), (1000, 48, 77), (3000, 72, 5000)])
def test_confidence_matches_oracle(xgs, n, d, k):
    X = synth.vq_mixture(n, d, 16, seed=2)
    E = synth.vq_codebook(k, d, 16, seed=3, centre_seed=2)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    idx, dist, conf = xgs.xgs_vq_assign_conf(t(X), t(E), Eb, en, 0.7)
    idx0, dist0 = xgs.xgs_vq_assign(t(X), t(E), Eb, en, xgs.VQ_BF16_RESCORE4)
    torch.cuda.synchronize()
    # the assignment is the plain BF16 form's
    np.testing.assert_array_equal(np_(idx), np_(idx0))
    np.testing.assert_array_equal(np_(dist), np_(dist0))
    ref = oracle.vq_confidence(X, E, 0.7)
    err = np.abs(np_(conf) - ref)
    print(f"confidence: max abs err {err.max():.2e}, mean {err.mean():.2e}")
    assert err.max() < 5e-3
    assert np.all(np_(conf) > 0) and np.all(np_(conf) <= 1.0 + 1e-6)


def test_confidence_full_size_sampled(xgs):
    X, E = synth.vq_mixture(816_000, 768, 256, seed=30), synth.vq_codebook(4096, 768, 256, seed=31, centre_seed=30)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    _, _, conf = xgs.xgs_vq_assign_conf(t(X), t(E), Eb, en, 0.7)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(32).choice(len(X), 512, replace=False))
    ref = oracle.vq_confidence(X[rows], E, 0.7)
    err = np.abs(np_(conf)[rows] - ref)
    print(f"confidence 816000x768 K=4096: max abs err {err.max():.2e}")
    assert err.max() < 5e-3


@pytest.mark.parametrize("mode", ["paper", "laplace"])
def test_masked_ema_with_dead_codes(xgs, mode):
    """Warm-start configuration (decay 0): codes without a confident sample
    die and take reservoir rows in order."""
    m = xgs.EMA_PAPER if mode == "paper" else xgs.EMA_LAPLACE
    X = synth.vq_mixture(6000, 32, 8, seed=40)
    E = synth.vq_codebook(64, 32, 8, seed=41, centre_seed=40)
    ri, _, _ = oracle.vq_assign(X, E)
    conf = oracle.vq_confidence(X, E, 0.7).astype(np.float32)
    gamma = float(np.quantile(conf, 0.4))
    res = synth.vq_mixture(7, 32, 8, seed=42)
    N0, M0 = oracle.ema_init(E)
    for decay, delta in ((0.0, 0.5), (0.9, 0.95)):
        Nr, Mr, Er, cr, dead = oracle.ema_update_robust(X, ri, conf, gamma, N0, M0, decay, 1e-5, m, delta, res, 3)
        Ng, Mg, Eg = t(N0), t(M0), t(E)
        Eb, en = xgs.xgs_vq_prepare(Eg)
        counts, n_dead = xgs.xgs_vq_ema_update_robust(t(X), t(ri, np.int32), t(conf), gamma, Ng, Mg, Eg, Eb, en,
                                                      decay=decay, eps=1e-5, mode=m, delta=delta, reservoir=t(res),
                                                      offset=3)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(np_(counts), cr)
        assert int(np_(n_dead)[0]) == int(dead.sum())
        assert rel_max(np_(Ng), Nr) < 1e-6
        assert rel_max(np_(Mg), Mr) < 1e-5
        assert rel_max(np_(Eg), Er) < 1e-5
        assert dead.sum() > 0


def test_robust_update_without_mask_or_reset_is_the_plain_update(xgs):
    X = synth.vq_mixture(3000, 16, 8, seed=50)
    E = synth.vq_codebook(40, 16, 8, seed=51, centre_seed=50)
    ri, _, _ = oracle.vq_assign(X, E)
    outs = []
    for robust in (False, True):
        N0, M0 = oracle.ema_init(E)
        Ng, Mg, Eg = t(N0), t(M0), t(E)
        Eb, en = xgs.xgs_vq_prepare(Eg)
        if robust:
            xgs.xgs_vq_ema_update_robust(t(X), t(ri, np.int32), None, 0.0, Ng, Mg, Eg, Eb, en, decay=0.99, eps=1e-5,
                                         mode=xgs.EMA_LAPLACE)
        else:
            xgs.xgs_vq_ema_update(t(X), t(ri, np.int32), Ng, Mg, Eg, Eb, en, 0.99, 1e-5, xgs.EMA_LAPLACE)
        torch.cuda.synchronize()
        outs.append([np_(a) for a in (Ng, Mg, Eg, Eb, en)])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)
