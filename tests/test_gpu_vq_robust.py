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


# Relative bound on the confidence of the BF16 form.  Its distances are
# exact for the bf16-rounded operands (the squared norms ride along as three
# bf16 pieces), so the error is that of rounding x and e to bf16: a relative
# 2^-9 per element, averaging to about 2^-9 ||x|| ||e|| / sqrt(D) in the dot
# product, divided by tau in the exponent.  Emulated in FP64 on these
# distributions (round the operands, recompute the confidence) that gives at
# most 1.8e-3 at D = 48..72 and 4.9e-4 at D = 768; the bounds below leave 2x.
CONF_REL = {"small_d": 4e-3, "d768": 1.5e-3}


def conf_rel_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / ref


@pytest.mark.parametrize("n,d,k", [(12_288, 64, 128), (1000, 48, 77), (3000, 72, 5000), (4000, 64, 1100)])
def test_confidence_matches_oracle(xgs, n, d, k):
    """K = 5000 runs 4 codebook parts of 5 tiles, K = 1100 runs 3 parts of 2
    tiles (the last one ragged): the per-part log-sum-exp terms are merged in
    the rescore."""
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
    err = conf_rel_err(np_(conf), ref)
    print(f"confidence K={k}: range [{ref.min():.3e}, {ref.max():.3e}], max rel err {err.max():.2e}")
    assert err.max() < CONF_REL["small_d"]
    assert np.all(np_(conf) <= 1.0 + 1e-6)


def exact_bf16_mixture(n, d, centres, sigma, seed):
    """Rows of a mixture rounded to multiples of 1/8 with |v| < 16: every value
    is a bf16 number and every product, norm and distance of two rows is exact
    in FP32, so the BF16 form's distances are exact."""
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, len(centres), n)
    v = centres[lab] + rng.normal(0.0, sigma, (n, d))
    return np.clip(np.round(v * 8) / 8, -15.875, 15.875).astype(np.float32)


def test_confidence_exact_operands_three_parts(xgs):
    """Operands exactly representable in bf16, K = 1100 (3 codebook parts),
    tau = 0.3: the confidence spans 0.05 .. 0.9 and only the FP32 evaluation
    of the softmax terms separates the kernel from the FP64 oracle, so the
    cross-part merge is checked to 2e-5 relative.  The rows include exact
    distance ties (lowest index wins on both sides)."""
    rng = np.random.default_rng(60)
    d, k = 64, 1100
    centres = rng.integers(-8, 9, (16, d)).astype(np.float64)
    X = exact_bf16_mixture(4000, d, centres, 0.6, seed=61)
    E = exact_bf16_mixture(k, d, centres, 0.6, seed=62)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    idx, dist, conf = xgs.xgs_vq_assign_conf(t(X), t(E), Eb, en, 0.3)
    torch.cuda.synchronize()
    ri, d1, d2 = oracle.vq_assign(X, E)
    assert (d1 == d2).sum() > 0
    np.testing.assert_array_equal(np_(idx), ri)
    np.testing.assert_array_equal(np_(dist).astype(np.float64), d1)
    ref = oracle.vq_confidence(X, E, 0.3)
    assert ref.min() < 0.1 and ref.max() > 0.8
    err = conf_rel_err(np_(conf), ref)
    print(f"confidence exact operands: max rel err {err.max():.2e}")
    assert err.max() < 2e-5


def test_confidence_full_size_sampled(xgs):
    X, E = synth.vq_mixture(816_000, 768, 256, seed=30), synth.vq_codebook(4096, 768, 256, seed=31, centre_seed=30)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    _, _, conf = xgs.xgs_vq_assign_conf(t(X), t(E), Eb, en, 0.7)
    torch.cuda.synchronize()
    c = np_(conf)
    assert np.all(c > 0) and np.all(c <= 1.0 + 1e-6)
    rows = np.sort(np.random.default_rng(32).choice(len(X), 512, replace=False))
    ref = oracle.vq_confidence(X[rows], E, 0.7)
    err = conf_rel_err(c[rows], ref)
    print(f"confidence 816000x768 K=4096: max rel err {err.max():.2e}")
    assert err.max() < CONF_REL["d768"]


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


@pytest.mark.parametrize("mode", ["paper", "laplace"])
def test_masked_ema_with_dead_codes_workload_shape(xgs, mode):
    """K = 4096, D = 768 on 65,536 rows with Zipf-popular codes and a seeded
    confidence mask: the dead-code ranking (4 codes per thread), the ordered
    reservoir reset and the masked sums against the FP64 oracle."""
    K, D, n = 4096, 768, 65_536
    m = xgs.EMA_PAPER if mode == "paper" else xgs.EMA_LAPLACE
    X = synth.vq_mixture(n, D, 256, seed=33)
    E = synth.vq_codebook(K, D, 256, seed=31, centre_seed=30)
    rng = np.random.default_rng(35)
    p = 1.0 / np.arange(1, K + 1)
    idx = rng.permutation(K)[rng.choice(K, n, p=p / p.sum())].astype(np.int32)
    conf = rng.random(n).astype(np.float32)
    gamma = 0.3
    res = synth.vq_mixture(300, D, 256, seed=36)
    N0, M0 = oracle.ema_init(E)
    Nr, Mr, Er, cr, dead = oracle.ema_update_robust(X, idx, conf, gamma, N0, M0, 0.99, 1e-5, m, 0.995, res, 7)
    assert dead.sum() > len(res)   # more dead codes than reservoir rows: the reset wraps around
    Ng, Mg, Eg = t(N0), t(M0), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    counts, n_dead = xgs.xgs_vq_ema_update_robust(t(X), t(idx, np.int32), t(conf), gamma, Ng, Mg, Eg, Eb, en,
                                                  decay=0.99, eps=1e-5, mode=m, delta=0.995, reservoir=t(res),
                                                  offset=7)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(counts), cr)
    assert int(np_(n_dead)[0]) == int(dead.sum())
    assert rel_max(np_(Ng), Nr) < 1e-6
    assert rel_max(np_(Mg), Mr) < 1e-5
    assert rel_max(np_(Eg), Er) < 1e-5


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
