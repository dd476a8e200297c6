"""GPU parity of grid-sampled targets (a5), VQ assignment (a6) and the EMA
update (a7) against the FP64 oracle, through the C ABI."""
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


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------ a5
@pytest.mark.parametrize("H,W,Hf,Wf,D,stride,oy,ox", [
    (480, 640, 30, 40, 512, 1, 0, 0),     # the mapping-scale target map
    (96, 128, 7, 9, 13, 3, 2, 1),         # ragged: H_s*W_s not a multiple of 4
    (50, 70, 13, 5, 6, 4, 3, 3),          # padded rows/columns at a large offset
    (17, 1, 4, 1, 3, 2, 1, 0),            # degenerate width
])
def test_grid_sample(xgs, H, W, Hf, Wf, D, stride, oy, ox):
    P = synth.feature_map(D, Hf, Wf, seed=H + W)
    for mode in (xgs.GRID_BILINEAR, xgs.GRID_NEAREST):
        G, V = xgs.xgs_grid_sample(t(P), H, W, stride, oy, ox, mode)
        torch.cuda.synchronize()
        Gr, Vr = oracle.grid_sample(P, H, W, stride, oy, ox, mode)
        np.testing.assert_array_equal(np_(V), Vr)
        if mode == xgs.GRID_NEAREST:
            np.testing.assert_array_equal(np_(G), Gr)  # a copy: bit-exact
        else:
            assert rel_max(np_(G), Gr) < 1e-6


@pytest.mark.parametrize("H,W,Hf,Wf,D,stride,mode", [
    (480, 640, 30, 40, 64, 2, 0),        # the mapping-scale map, four offsets
    (96, 128, 7, 9, 13, 3, 0),           # ragged grids (H_s W_s not a multiple of 4)
    (50, 70, 13, 5, 6, 4, 1),            # nearest, padded rows and columns
    (17, 1, 4, 1, 3, 2, 0),              # degenerate width
    (33, 41, 5, 6, 3, 1, 0),             # stride 1: the one offset is the plain call
    (40, 56, 6, 7, 2, 8, 1),             # 64 offsets, nearest
    (5, 70, 3, 9, 2, 8, 0),              # H < stride: offsets past the last row are all padding
])
def test_grid_sample_all_offsets(xgs, H, W, Hf, Wf, D, stride, mode):
    """Every offset's grid in one launch is bitwise the per-offset call, and
    matches the oracle for each offset."""
    P = synth.feature_map(D, Hf, Wf, seed=7)
    Pg = t(P)
    G, V = xgs.xgs_grid_sample_offsets(Pg, H, W, stride, mode)
    torch.cuda.synchronize()
    G, V = np_(G), np_(V)
    for oy in range(stride):
        for ox in range(stride):
            o = oy * stride + ox
            g1, v1 = xgs.xgs_grid_sample(Pg, H, W, stride, oy, ox, mode)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(G[o], np_(g1))
            np.testing.assert_array_equal(V[o], np_(v1))
            ref, vref = oracle.grid_sample(P, H, W, stride, oy, ox, mode)
            np.testing.assert_array_equal(V[o], vref)
            if mode == xgs.GRID_NEAREST:
                np.testing.assert_array_equal(G[o], ref)
            else:
                assert rel_max(G[o], ref) < 1e-6


def test_grid_sample_affine_exact(xgs):
    P = synth.affine_feature_map(5, 9, 17)
    G, _ = xgs.xgs_grid_sample(t(P), 65, 65)
    Gr, _ = oracle.grid_sample(P, 65, 65)
    np.testing.assert_array_equal(np_(G), Gr)


# ------------------------------------------------------------------ a6
def agreement(idx, ref_idx, d1, d2, tie_rel=1e-6):
    raw = float((idx == ref_idx).mean())
    tie = (d2 - d1) <= tie_rel * np.maximum(d1, 1e-30)
    adj = float(((idx == ref_idx) | tie).mean())
    return raw, adj


def vq_case(n, d, k, clusters, seed=2):
    X = synth.vq_mixture(n, d, clusters, seed=seed)
    E = synth.vq_codebook(k, d, clusters, seed=seed + 1, centre_seed=seed)
    return X, E


@pytest.mark.parametrize("n,d,k", [(12_288, 64, 128), (1000, 48, 77), (65, 16, 5), (3000, 72, 5000), (300, 8, 1),
                                   (4500, 32, 700)])
def test_vq_assign_small(xgs, n, d, k):
    X, E = vq_case(n, d, k, 16)
    ri, d1, d2 = oracle.vq_assign(X, E)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    for prec in (xgs.VQ_FP32, xgs.VQ_BF16_RESCORE4):
        idx, dist = xgs.xgs_vq_assign(t(X), t(E), Eb, en, prec)
        torch.cuda.synchronize()
        idx = np_(idx)
        raw, adj = agreement(idx, ri, d1, d2)
        assert adj >= 0.999, (prec, raw, adj)
        # the reported distance is the FP32 squared distance of the chosen codeword
        chosen = ((X.astype(np.float64) - E[idx].astype(np.float64)) ** 2).sum(1)
        assert rel_max(np_(dist), chosen) < 1e-5
    if n == 12_288:
        assert raw >= 0.999


def test_vq_staged_calls_equal_assign(xgs):
    """xgs_vq_stage -> xgs_vq_candidates -> xgs_vq_rescore is xgs_vq_assign
    (bitwise), with K spanning two codebook parts and a ragged row tail."""
    X, E = vq_case(2_000 + 37, 40, 4_400, 32, seed=12)
    Xg, Eg = t(X), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    idx_a, dist_a = xgs.xgs_vq_assign(Xg, Eg, Eb, en, xgs.VQ_BF16_RESCORE4)
    ws = xgs.vq_assign_workspace(len(X), 40, 4_400)
    xgs.xgs_vq_stage(Xg, Eb, en, ws)
    xgs.xgs_vq_candidates(len(X), 40, 4_400, ws)
    idx_s, dist_s = xgs.xgs_vq_rescore(Xg, Eg, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(idx_a), np_(idx_s))
    np.testing.assert_array_equal(np_(dist_a), np_(dist_s))
    ri, d1, d2 = oracle.vq_assign(X, E)
    raw, adj = agreement(np_(idx_s), ri, d1, d2)
    assert adj >= 0.999, (raw, adj)


@pytest.mark.parametrize("n,d,k", [(816_000, 768, 4096), (2_037, 40, 4_400), (1000, 48, 77), (3001, 256, 520)])
def test_vq_two_sweeps_agree_bitwise(xgs, n, d, k):
    """The plain assignment's sweep (codeword operand in registers) and the
    confidence form's sweep (both operands through LDS) form the same
    products in the same order, so their candidates, and hence the rescored
    index and distance, are bitwise equal: at the workload shape, with K over
    two parts and a ragged row tail, with a part past the last codeword, and
    with D not a multiple of 32 in the staged layout."""
    X, E = vq_case(n, d, k, 256 if n > 100_000 else 16, seed=17)
    Xg, Eg = t(X), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    idx_a, dist_a = xgs.xgs_vq_assign(Xg, Eg, Eb, en, xgs.VQ_BF16_RESCORE4)
    idx_c, dist_c, conf = xgs.xgs_vq_assign_conf(Xg, Eg, Eb, en, 0.7)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(idx_a), np_(idx_c))
    np.testing.assert_array_equal(np_(dist_a), np_(dist_c))
    assert np.all(np_(conf) > 0)


def test_vq_prepare_is_bf16_rounding(xgs):
    E = synth.vq_codebook(64, 32, 8, seed=9, centre_seed=8)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    torch.cuda.synchronize()
    eb = np_(Eb).view(np.uint16)
    ref = torch.from_numpy(E).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(eb, ref)
    f = torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy().astype(np.float64)
    assert rel_max(np_(en), (f * f).sum(1)) < 1e-6


def test_vq_assign_precision_form_sampled(xgs):
    """816,000 x 768 against K = 4,096 (the precision form): the full batch runs
    on the GPU in both precisions; agreement with the FP64 oracle is measured on
    a seeded 4,096-row sample (the oracle's brute force)."""
    X, E = vq_case(816_000, 768, 4096, 256, seed=30)
    Xg, Eg = t(X), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    idx_b, _ = xgs.xgs_vq_assign(Xg, Eg, Eb, en, xgs.VQ_BF16_RESCORE4)
    idx_f, _ = xgs.xgs_vq_assign(Xg, Eg, Eb, en, xgs.VQ_FP32)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(31).choice(len(X), 4096, replace=False))
    ri, d1, d2 = oracle.vq_assign(X[rows], E)
    raw_b, adj_b = agreement(np_(idx_b)[rows], ri, d1, d2)
    raw_f, adj_f = agreement(np_(idx_f)[rows], ri, d1, d2)
    print(f"agreement bf16+rescore raw {raw_b:.5f} tie-adjusted {adj_b:.5f}; fp32 raw {raw_f:.5f} adj {adj_f:.5f}")
    assert adj_b >= 0.999 and adj_f >= 0.999


def test_vq_edge_cases(xgs):
    # duplicated codewords: ties go to the lowest index on both paths
    E = np.array([[1, 0, 0, 0] * 4, [0, 1, 0, 0] * 4, [1, 0, 0, 0] * 4, [0, 1, 0, 0] * 4], np.float32)
    X = np.array([[1, 0, 0, 0] * 4, [0, 1, 0, 0] * 4, [0.5, 0.5, 0, 0] * 4], np.float32)
    Eb, en = xgs.xgs_vq_prepare(t(E))
    for prec in (xgs.VQ_FP32, xgs.VQ_BF16_RESCORE4):
        idx, _ = xgs.xgs_vq_assign(t(X), t(E), Eb, en, prec)
        torch.cuda.synchronize()
        assert list(np_(idx)) == [0, 1, 0], prec
    with pytest.raises(xgs.XgsError):
        xgs.xgs_vq_assign(t(X[:, :15].copy()), t(E[:, :15].copy()), Eb, en, xgs.VQ_BF16_RESCORE4)
    idx, dist = xgs.xgs_vq_assign(t(X[:0].copy()), t(E), Eb, en, xgs.VQ_BF16_RESCORE4)
    assert idx.numel() == 0


# ------------------------------------------------------------------ a7
@pytest.mark.parametrize("mode", ["paper", "laplace"])
def test_ema_update_matches_oracle(xgs, mode):
    X, E = vq_case(12_288, 64, 128, 16)
    m = xgs.EMA_PAPER if mode == "paper" else xgs.EMA_LAPLACE
    ri, _, _ = oracle.vq_assign(X, E)
    N0, M0 = oracle.ema_init(E)
    Nr, Mr, Er, cr, _ = oracle.ema_update(X, ri, N0, M0, 0.99, 1e-5, m)
    Ng, Mg, Eg = t(N0.astype(np.float32)), t(M0.astype(np.float32)), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    counts = xgs.xgs_vq_ema_update(t(X), t(ri.astype(np.int32)), Ng, Mg, Eg, Eb, en, 0.99, 1e-5, m)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(counts), cr)
    assert rel_max(np_(Ng), Nr) < 1e-6
    assert rel_max(np_(Mg), Mr) < 1e-5
    assert rel_max(np_(Eg), Er) < 1e-5
    # the shadow follows the new codebook
    ref = torch.from_numpy(np_(Eg)).to(torch.bfloat16).view(torch.int16).numpy()
    np.testing.assert_array_equal(np_(Eb), ref)


def test_ema_update_skewed_codes_match_oracle(xgs):
    """One code takes 10,000 rows (79 pieces of 128), one code one row, three
    codes none, D not a multiple of the column block: the per-piece sums added
    in piece order against the FP64 oracle."""
    X, E = vq_case(20_000, 40, 8, 4, seed=5)
    rng = np.random.default_rng(11)
    idx = np.where(rng.random(len(X)) < 0.5, 0, rng.integers(1, 5, len(X))).astype(np.int32)
    idx[idx == 3] = 4
    idx[17] = 3
    for mode in (xgs.EMA_PAPER, xgs.EMA_LAPLACE):
        N0, M0 = oracle.ema_init(E)
        Nr, Mr, Er, cr, _ = oracle.ema_update(X, idx, N0, M0, 0.9, 1e-5, mode)
        Ng, Mg, Eg = t(N0.astype(np.float32)), t(M0.astype(np.float32)), t(E)
        counts = xgs.xgs_vq_ema_update(t(X), t(idx), Ng, Mg, Eg, None, None, 0.9, 1e-5, mode)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(np_(counts), cr)
        assert cr[0] > 9000 and cr[3] == 1 and cr[5:].sum() == 0
        assert rel_max(np_(Ng), Nr) < 1e-6
        assert rel_max(np_(Mg), Mr) < 1e-5
        assert rel_max(np_(Eg), Er) < 1e-5


def zipf_codes(n, k, seed):
    """Code indices with a Zipf(1) popularity over a random permutation of the
    K codes: the most popular code takes about n / ln(K) rows (dozens of
    128-row pieces) and a few hundred codes take none."""
    rng = np.random.default_rng(seed)
    p = 1.0 / np.arange(1, k + 1)
    return rng.permutation(k)[rng.choice(k, n, p=p / p.sum())].astype(np.int32)


@pytest.mark.parametrize("mode", ["paper", "laplace"])
def test_ema_update_workload_shape(xgs, mode):
    """K = 4096 codes of D = 768 (the precision-form codebook) on 65,536 rows:
    every thread of the per-code kernels handles ceil(K / 1024) = 4 codes, the
    most popular code is summed from ~60 pieces, and the bf16 shadow and its
    squared norms are refreshed from the new codebook."""
    K, D, n = 4096, 768, 65_536
    X = synth.vq_mixture(n, D, 256, seed=33)
    E = synth.vq_codebook(K, D, 256, seed=31, centre_seed=30)
    idx = zipf_codes(n, K, seed=34)
    m = xgs.EMA_PAPER if mode == "paper" else xgs.EMA_LAPLACE
    N0, M0 = oracle.ema_init(E)
    Nr, Mr, Er, cr, _ = oracle.ema_update(X, idx, N0, M0, 0.99, 1e-5, m)
    assert cr.max() > 50 * 128 and (cr == 0).sum() > 100
    Ng, Mg, Eg = t(N0.astype(np.float32)), t(M0.astype(np.float32)), t(E)
    Eb, en = xgs.xgs_vq_prepare(Eg)
    counts = xgs.xgs_vq_ema_update(t(X), t(idx), Ng, Mg, Eg, Eb, en, 0.99, 1e-5, m)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(counts), cr)
    assert rel_max(np_(Ng), Nr) < 1e-6
    assert rel_max(np_(Mg), Mr) < 1e-5
    assert rel_max(np_(Eg), Er) < 1e-5
    # shadow and norms of the updated codebook (bf16 rounding of the kernel's E)
    eb_ref = torch.from_numpy(np_(Eg)).to(torch.bfloat16)
    np.testing.assert_array_equal(np_(Eb), eb_ref.view(torch.int16).numpy())
    f = eb_ref.float().numpy().astype(np.float64)
    assert rel_max(np_(en), (f * f).sum(1)) < 1e-6


def test_ema_update_is_bitwise_reproducible(xgs):
    X, E = vq_case(50_000, 64, 128, 16, seed=7)
    idx = t(np.random.default_rng(1).integers(0, 128, len(X)).astype(np.int32))
    outs = []
    for _ in range(2):
        N0, M0 = oracle.ema_init(E)
        Ng, Mg, Eg = t(N0.astype(np.float32)), t(M0.astype(np.float32)), t(E)
        xgs.xgs_vq_ema_update(t(X), idx, Ng, Mg, Eg, None, None, 0.99, 1e-5, xgs.EMA_LAPLACE)
        torch.cuda.synchronize()
        outs.append((np_(Ng), np_(Mg), np_(Eg)))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_ema_update_no_samples(xgs):
    E = synth.vq_codebook(16, 8, 4, seed=2, centre_seed=1)
    N0, M0 = oracle.ema_init(E)
    Ng, Mg, Eg = t(N0.astype(np.float32)), t(M0.astype(np.float32)), t(E)
    X0 = torch.empty((0, 8), device="cuda")
    i0 = torch.empty(0, dtype=torch.int32, device="cuda")
    xgs.xgs_vq_ema_update(X0, i0, Ng, Mg, Eg, None, None, 0.99, 1e-5, xgs.EMA_PAPER)
    torch.cuda.synchronize()
    assert rel_max(np_(Ng), 0.99 * N0) < 1e-6
