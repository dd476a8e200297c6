"""FP64 CPU oracle for the X-GS Perceiver hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
bench's CPU-baseline leg are the only callers.  Nothing here is imported by the
HIP path, and nothing here imports it.  The compiled part (``oracle.c``) covers
projection, binning, compositing and their gradients and the VQ distances; this
module wraps it and adds the two steps that are plain array arithmetic in numpy
(grid-sampled targets and the EMA codebook update).

Every function works in float64.  Inputs that the product stores in binary32
are widened exactly before use.

Parity pins: see ``tests/test_oracle_*.py`` (closed forms, invariants, brute
force, finite differences, library cross-checks).  Every function here is
pinned; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TILE = 16
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (IEEE double, no
    fast-math).  OpenMP parallelises the independent loops: grid rows of the
    compositing walks (the backward adds into the per-Gaussian sums with atomic
    adds) and rows of X in the VQ distances."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        for name in ("orc_project", "orc_composite_fwd", "orc_composite_list", "orc_composite_bwd", "orc_composite_tiles",
                     "orc_project_bwd", "orc_pose_grad", "orc_vq_assign", "orc_vq_confidence", "orc_grid_info", "orc_set_threads"):
            getattr(_lib, name).restype = ctypes.c_int
        _lib.orc_bin.restype = ctypes.c_int64
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's parallel loops (n <= 0 leaves the count as it
    is); returns the count in effect."""
    return int(lib().orc_set_threads(ctypes.c_int32(n)))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam_array(cam) -> np.ndarray:
    """Camera -> the double[26] layout documented in oracle.c."""
    v = np.asarray(cam.viewmat, dtype=np.float64).reshape(16)
    return np.concatenate([[cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.near,
                            cam.stride, cam.off_y, cam.off_x], v]).astype(np.float64)


def grid_info(cam):
    out = np.zeros(4, dtype=np.int32)
    lib().orc_grid_info(_p(cam_array(cam)), _p(out))
    hs, ws, ty, tx = (int(v) for v in out)
    return hs, ws, ty, tx


@dataclass
class Projection:
    mean2d: np.ndarray   # [n,2]
    conic: np.ndarray    # [n,3]  A, B, C of A dx^2 + 2B dx dy + C dy^2
    depth: np.ndarray    # [n]    camera z
    cov2d: np.ndarray    # [n,3]  a, b, c of Sigma' (with dilation)
    ext: np.ndarray      # [n,2]  half-widths of the opacity-aware box
    rect: np.ndarray     # [n,4]  int32 tiles [x0, y0, x1, y1) exclusive upper
    touched: np.ndarray  # [n]    int64
    visible: np.ndarray  # [n]    int32


def project(scene, cam) -> Projection:
    """EWA projection of every Gaussian (App. A: Sigma = R S S^T R^T,
    Sigma' = J W Sigma W^T J^T), plus the opacity-aware tile rectangle."""
    n = scene.n
    out = Projection(np.zeros((n, 2)), np.zeros((n, 3)), np.zeros(n), np.zeros((n, 3)),
                     np.zeros((n, 2)), np.zeros((n, 4), np.int32), np.zeros(n, np.int64),
                     np.zeros(n, np.int32))
    lib().orc_project(ctypes.c_int64(n), _p(_f64(scene.means)), _p(_f64(scene.log_scales)),
                      _p(_f64(scene.quats)), _p(_f64(scene.opacity)), _p(cam_array(cam)),
                      _p(out.mean2d), _p(out.conic), _p(out.depth), _p(out.cov2d), _p(out.ext),
                      _p(out.rect), _p(out.touched), _p(out.visible))
    return out


def depth_bits(depth) -> np.ndarray:
    """The sort key's depth part: the binary32 value of camera z, as bits."""
    return np.ascontiguousarray(np.asarray(depth, dtype=np.float32).view(np.uint32))


def bin_instances(rect, dbits, tiles_x: int, tiles_y: int):
    """(tile, depth-bits, index)-sorted instance list and per-tile ranges."""
    rect = np.ascontiguousarray(rect, dtype=np.int32)
    dbits = np.ascontiguousarray(dbits, dtype=np.uint32)
    n = rect.shape[0]
    m = int(((rect[:, 2] - rect[:, 0]).astype(np.int64) * (rect[:, 3] - rect[:, 1])).sum())
    keys = np.zeros(max(m, 1), np.uint64)
    vals = np.zeros(max(m, 1), np.uint32)
    ranges = np.zeros(2 * tiles_x * tiles_y, np.uint32)
    got = lib().orc_bin(ctypes.c_int64(n), _p(rect), _p(dbits), ctypes.c_int32(tiles_x),
                        ctypes.c_int32(tiles_y), ctypes.c_int64(m), _p(keys), _p(vals), _p(ranges))
    assert got == m
    return keys[:m], vals[:m], ranges.reshape(-1, 2)


def channels(scene, depth) -> np.ndarray:
    """Per-Gaussian channel rows [RGB, depth, semantic...] (Sec. 3.1 and
    App. B: the depth and feature maps substitute d_i and f_i for c_i)."""
    return np.ascontiguousarray(np.concatenate(
        [_f64(scene.colors), _f64(depth)[:, None], _f64(scene.features)], axis=1))


@dataclass
class Render:
    proj: Projection
    keys: np.ndarray
    order: np.ndarray
    ranges: np.ndarray
    out: np.ndarray       # [C, Hs, Ws]
    final_T: np.ndarray   # [Hs, Ws]
    n_last: np.ndarray    # [Hs, Ws]
    amb: np.ndarray       # [4, Hs, Ws] skip, stop, depth-gap measures; blend signature
    chan: np.ndarray


def composite_fwd(proj: Projection, opacity, chan, order, ranges, cam, tile_mask=None,
                  depth=None):
    hs, ws, ty, tx = grid_info(cam)
    C = chan.shape[1]
    out = np.zeros((C, hs, ws))
    fT = np.ones((hs, ws))
    nl = np.zeros((hs, ws), np.int64)
    amb = np.full((4, hs, ws), np.inf)
    amb[3] = 0.0
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    lib().orc_composite_fwd(ctypes.c_int64(len(opacity)), _p(_f64(proj.mean2d)),
                            _p(_f64(proj.conic)), _p(_f64(opacity)), _p(_f64(chan)),
                            _p(_f64(proj.depth if depth is None else depth)), ctypes.c_int32(C),
                            _p(np.ascontiguousarray(order, np.uint32)),
                            _p(np.ascontiguousarray(ranges, np.uint32)), _p(cam_array(cam)),
                            _p(tm), _p(out), _p(fT), _p(nl), _p(amb))
    return out, fT, nl, amb


def render(scene, cam, tile_mask=None) -> Render:
    """Project -> bin -> composite, all in the oracle (FP64 arithmetic; only the
    depth sort key is binary32, as the reading of the sort key requires)."""
    hs, ws, ty, tx = grid_info(cam)
    pr = project(scene, cam)
    keys, order, ranges = bin_instances(pr.rect, depth_bits(pr.depth), tx, ty)
    chan = channels(scene, pr.depth)
    out, fT, nl, amb = composite_fwd(pr, scene.opacity, chan, order, ranges, cam, tile_mask)
    return Render(pr, keys, order, ranges, out, fT, nl, amb, chan)


def render_tiles(scene, cam, tiles):
    """Project -> bin -> composite of the listed tiles only, returned compactly:
    out [k][C][16][16], final_T [k][16][16], amb [k][4][16][16] (skip, stop and
    depth-gap measures and the blend signature, as in Render.amb)."""
    hs, ws, ty, tx = grid_info(cam)
    pr = project(scene, cam)
    keys, order, ranges = bin_instances(pr.rect, depth_bits(pr.depth), tx, ty)
    chan = channels(scene, pr.depth)
    tiles = np.ascontiguousarray(tiles, dtype=np.int32)
    C = chan.shape[1]
    out = np.zeros((len(tiles), C, 16, 16))
    fT = np.ones((len(tiles), 16, 16))
    amb = np.full((len(tiles), 4, 16, 16), np.inf)
    amb[:, 3] = 0.0
    lib().orc_composite_tiles(_p(_f64(pr.mean2d)), _p(_f64(pr.conic)), _p(_f64(scene.opacity)), _p(chan),
                              _p(_f64(pr.depth)), ctypes.c_int32(C), _p(np.ascontiguousarray(order, np.uint32)),
                              _p(np.ascontiguousarray(ranges, np.uint32)), _p(cam_array(cam)), _p(tiles),
                              ctypes.c_int32(len(tiles)), _p(out), _p(fT), _p(amb))
    return pr, out, fT, amb


def tile_view(img, cam, tiles):
    """[..., Hs, Ws] image -> [k, ..., 16, 16] stack of the listed tiles (zero past the edge)."""
    hs, ws, ty, tx = grid_info(cam)
    img = np.asarray(img)
    lead = img.shape[:-2]
    res = np.zeros((len(tiles),) + lead + (16, 16), dtype=img.dtype)
    for q, t in enumerate(tiles):
        y, x = divmod(int(t), tx)
        blk = img[..., 16 * y:16 * y + 16, 16 * x:16 * x + 16]
        res[(q,) + (slice(None),) * len(lead) + (slice(0, blk.shape[-2]), slice(0, blk.shape[-1]))] = blk
    return res


def untile(stack, cam, tiles):
    """Inverse of tile_view: [k, ..., 16, 16] -> [..., Hs, Ws], zero elsewhere."""
    hs, ws, ty, tx = grid_info(cam)
    stack = np.asarray(stack)
    lead = stack.shape[1:-2]
    img = np.zeros(lead + (hs, ws), dtype=stack.dtype)
    for q, t in enumerate(tiles):
        y, x = divmod(int(t), tx)
        h = min(16, hs - 16 * y); w = min(16, ws - 16 * x)
        img[..., 16 * y:16 * y + h, 16 * x:16 * x + w] = stack[q, ..., :h, :w]
    return img


def composite_list(proj: Projection, opacity, chan, order, cam):
    """No tiles: every pixel walks the same global list."""
    hs, ws, _, _ = grid_info(cam)
    C = chan.shape[1]
    out = np.zeros((C, hs, ws))
    fT = np.ones((hs, ws))
    order = np.ascontiguousarray(order, np.uint32)
    lib().orc_composite_list(_p(_f64(proj.mean2d)), _p(_f64(proj.conic)), _p(_f64(opacity)),
                             _p(_f64(chan)), ctypes.c_int32(C), _p(order),
                             ctypes.c_int64(len(order)), _p(cam_array(cam)), _p(out), _p(fT))
    return out, fT


@dataclass
class Grads:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    colors: np.ndarray
    features: np.ndarray
    mean2d: np.ndarray
    conic: np.ndarray


def composite_bwd(scene, cam, g, r: Render, tile_mask=None):
    """Gradient of L = sum g * out with respect to the 2D splat parameters and
    the channels: (d_mean2d [n][2], d_conic [n][3], d_opacity [n], d_chan [n][C])."""
    n = scene.n
    C = r.chan.shape[1]
    d_m2 = np.zeros((n, 2)); d_co = np.zeros((n, 3)); d_op = np.zeros(n); d_ch = np.zeros((n, C))
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    lib().orc_composite_bwd(ctypes.c_int64(n), _p(_f64(r.proj.mean2d)), _p(_f64(r.proj.conic)),
                            _p(_f64(scene.opacity)), _p(r.chan), ctypes.c_int32(C),
                            _p(np.ascontiguousarray(r.order, np.uint32)),
                            _p(np.ascontiguousarray(r.ranges, np.uint32)), _p(cam_array(cam)),
                            _p(_f64(g)), _p(tm), _p(d_m2), _p(d_co), _p(d_op), _p(d_ch))
    return d_m2, d_co, d_op, d_ch


def render_grad(scene, cam, g, r: Render | None = None, tile_mask=None) -> Grads:
    """Analytic FP64 gradient of L = sum g * out for every parameter group:
    the compositing backward, then the projection backward of every Gaussian."""
    if r is None:
        r = render(scene, cam, tile_mask)
    d_m2, d_co, d_op, d_ch = composite_bwd(scene, cam, g, r, tile_mask)
    d_means, d_ls, d_q = project_bwd(scene, cam, d_m2, d_co, np.ascontiguousarray(d_ch[:, 3]))
    return Grads(d_means, d_ls, d_q, d_op, d_ch[:, :3].copy(), d_ch[:, 4:].copy(), d_m2, d_co)


def project_bwd(scene, cam, d_mean2d, d_conic, d_depth):
    n = scene.n
    d_means = np.zeros((n, 3)); d_ls = np.zeros((n, 3)); d_q = np.zeros((n, 4))
    lib().orc_project_bwd(ctypes.c_int64(n), _p(_f64(scene.means)), _p(_f64(scene.log_scales)),
                          _p(_f64(scene.quats)), _p(_f64(scene.opacity)), _p(cam_array(cam)),
                          _p(_f64(d_mean2d)), _p(_f64(d_conic)), _p(_f64(d_depth)), _p(d_means),
                          _p(d_ls), _p(d_q))
    return d_means, d_ls, d_q


def loss(out, g) -> float:
    return float((np.asarray(out, np.float64) * np.asarray(g, np.float64)).sum())


# --------------------------------------------------------------- grid sample
BILINEAR = 0
NEAREST = 1


def grid_sample(P, H: int, W: int, stride: int = 1, off_y: int = 0, off_x: int = 0,
                mode: int = BILINEAR):
    """Targets on the sampled grid (App. D, Eq. (sampled_loc), Eq. (target_continuous)).

    (u, v) = (off_y + m s, off_x + n s); u~ = u (Hf-1)/max(H-1,1), v~ likewise.
    NEAREST takes P at the rounded (u~, v~) (round half to even, done exactly in
    integers); BILINEAR interpolates P at (u~, v~).  V = 1 inside the image and
    0 (with G = 0) where u >= H or v >= W.
    """
    P = _f64(P)
    D, Hf, Wf = P.shape
    Hs, Ws = -(-H // stride), -(-W // stride)
    u = off_y + np.arange(Hs, dtype=np.int64) * stride
    v = off_x + np.arange(Ws, dtype=np.int64) * stride
    by, bx = max(H - 1, 1), max(W - 1, 1)
    ay, ax = u * (Hf - 1), v * (Wf - 1)
    qy, ry = np.divmod(ay, by)
    qx, rx = np.divmod(ax, bx)
    valid = (u[:, None] < H) & (v[None, :] < W)
    if mode == NEAREST:
        iy = qy + ((2 * ry > by) | ((2 * ry == by) & (qy % 2 == 1)))
        ix = qx + ((2 * rx > bx) | ((2 * rx == bx) & (qx % 2 == 1)))
        iy = np.minimum(iy, Hf - 1); ix = np.minimum(ix, Wf - 1)
        G = P[:, iy[:, None], ix[None, :]]
    else:
        y0 = np.minimum(qy, Hf - 1); x0 = np.minimum(qx, Wf - 1)
        y1 = np.minimum(y0 + 1, Hf - 1); x1 = np.minimum(x0 + 1, Wf - 1)
        wy = (ry / by)[:, None]; wx = (rx / bx)[None, :]
        G = ((1 - wy) * (1 - wx) * P[:, y0[:, None], x0[None, :]]
             + (1 - wy) * wx * P[:, y0[:, None], x1[None, :]]
             + wy * (1 - wx) * P[:, y1[:, None], x0[None, :]]
             + wy * wx * P[:, y1[:, None], x1[None, :]])
    G = np.where(valid[None], G, 0.0)
    return G, valid.astype(np.uint8)


# ------------------------------------------------------------------------ VQ
def vq_assign(X, E):
    """a_n = argmin_l ||x_n - E_l||^2 in FP64 (Sec. 3.2.2), lowest index on ties.
    Returns (idx int32, best squared distance, second-best squared distance)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    E = np.ascontiguousarray(E, dtype=np.float32)
    N, D = X.shape
    K = E.shape[0]
    idx = np.zeros(N, np.int32); d1 = np.zeros(N); d2 = np.zeros(N)
    lib().orc_vq_assign(ctypes.c_int64(N), ctypes.c_int32(D), _p(X), ctypes.c_int32(K), _p(E),
                        _p(idx), _p(d1), _p(d2))
    return idx, d1, d2


PAPER = 0
LAPLACE = 1


def ema_init(E):
    """Reading: the EMA state starts at N = 1, M = E for every codeword."""
    E = _f64(E)
    return np.ones(E.shape[0]), E.copy()


def ema_update(X, idx, N_ema, M_ema, decay: float, eps: float, mode: int = LAPLACE):
    """One step of Eq. (ema_update).

    c_l = #{n : a_n = l},  s_l = sum_{a_n = l} x_n,
    N <- lambda N + (1-lambda) c,  M <- lambda M + (1-lambda) s,
    PAPER:   E_l = M_l / (N_l + eps)
    LAPLACE: E_l = M_l / Ntilde_l, Ntilde_l = (N_l + eps) / (n + K eps) * n, n = sum_l N_l.
    Returns (N, M, E, counts, sums) in FP64."""
    X = _f64(X)
    idx = np.asarray(idx, dtype=np.int64)
    K, D = M_ema.shape
    counts = np.zeros(K)
    sums = np.zeros((K, D))
    for n in range(X.shape[0]):
        counts[idx[n]] += 1.0
        sums[idx[n]] += X[n]
    N_new = decay * _f64(N_ema) + (1.0 - decay) * counts
    M_new = decay * _f64(M_ema) + (1.0 - decay) * sums
    if mode == PAPER:
        E_new = M_new / (N_new + eps)[:, None]
    else:
        tot = N_new.sum()
        nt = (N_new + eps) / (tot + K * eps) * tot
        E_new = M_new / nt[:, None]
    return N_new, M_new, E_new, counts, sums


# ------------------------------------------------------------ semantic phase
# Sec. 3.2.2 (online VQ module): each Gaussian carries logits z_i over the L
# codewords, w_i = softmax(z_i), decoded feature E^T w_i; App. E renders the
# mixture weights and decodes per pixel, F(x) = E^T w(x).  App. D (masked loss
# evaluation): L_grid = lambda_sem [L_cos + L_1] over the valid grid pixels,
# geometry frozen (Sec. 3.2.2, parallelized pipeline).
#
# Readings (the paper does not spell these out):
#   L_cos = (1/n) sum_{x valid} (1 - cos(G^(x), G*(x))),
#           cos(a, b) = <a, b> / max(|a| |b|, 1e-8);
#   L_1   = (1/(n D)) sum_{x valid} sum_d |G^_d(x) - G*_d(x)|;
#   n = number of valid pixels; n = 0 gives L = 0 and zero gradients;
#   d|t|/dt = sign(t) with sign(0) = 0.
COS_EPS = 1e-8


def semantic_softmax(z):
    """w_i = softmax(z_i) over the codewords (rows of z)."""
    z = _f64(z)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def semantic_softmax_bwd(w, dw):
    """dL/dz_i = w_i * (dL/dw_i - <dL/dw_i, w_i>)."""
    w = _f64(w)
    dw = _f64(dw)
    return w * (dw - (dw * w).sum(axis=1, keepdims=True))


def semantic_loss(wmap, E, Gstar, V, lam: float = 1.0):
    """Masked cosine + L1 loss of the decoded map against the targets.

    wmap [L][Hs][Ws] rendered mixture weights, E [L][D] codebook,
    Gstar [D][Hs][Ws] targets, V [Hs][Ws] validity.  Returns (loss,
    dL/dwmap [L][Hs][Ws]) in FP64."""
    wmap = _f64(wmap)
    E = _f64(E)
    Gs = _f64(Gstar)
    L, Hs, Ws = wmap.shape
    D = E.shape[1]
    valid = np.asarray(V).astype(bool)
    n = int(valid.sum())
    dw = np.zeros_like(wmap)
    if n == 0:
        return 0.0, dw
    W = wmap.reshape(L, -1)[:, valid.ravel()]          # [L][n]
    B = Gs.reshape(D, -1)[:, valid.ravel()]            # [D][n]
    A = E.T @ W                                         # decoded G^ [D][n]
    na = np.sqrt((A * A).sum(0))
    nb = np.sqrt((B * B).sum(0))
    dot = (A * B).sum(0)
    den = np.maximum(na * nb, COS_EPS)
    cos = dot / den
    diff = A - B
    loss_cos = (1.0 - cos).sum() / n
    loss_l1 = np.abs(diff).sum() / (n * D)
    # d cos / dA = B / den - [den > eps] cos A / |A|^2
    scale = np.where(na * nb > COS_EPS, 1.0, 0.0)
    na2 = np.where(na > 0, na * na, 1.0)
    dcos = B / den - scale * cos * A / na2
    g = lam * (-dcos / n + np.sign(diff) / (n * D))    # dL/dA [D][n]
    dwv = E @ g                                         # dL/dW [L][n]
    dw.reshape(L, -1)[:, valid.ravel()] = dwv
    return lam * (loss_cos + loss_l1), dw


def semantic_phase(scene, cam, z, E, Gstar, V, lam: float = 1.0, tile_mask=None):
    """One semantic-phase evaluation: w = softmax(z) rendered as the feature
    channels, decoded, masked loss, and dL/dz through the feature-only
    backward.  Returns (loss, dL/dz [N][L], rendered wmap [L][Hs][Ws])."""
    w = semantic_softmax(z)
    sc = scene.__class__(**{**scene.__dict__, "features": w})
    r = render(sc, cam, tile_mask)
    wmap = r.out[4:]
    val, dwmap = semantic_loss(wmap, E, Gstar, V, lam)
    g = np.concatenate([np.zeros((4,) + wmap.shape[1:]), dwmap], axis=0)
    gr = render_grad(sc, cam, g, r, tile_mask=tile_mask)
    return val, semantic_softmax_bwd(w, gr.features), wmap


# ----------------------------------------------------------------- tracking
# Eq. (tracking) / Eq. (loss_track): the pose is refined against the colour
# image and the depth map with the map frozen.
# Readings: L_photo = (1/(3 P)) sum_x sum_{c<3} |I^_c(x) - I_c(x)| over the P
# grid pixels; the depth term is lambda_d (1/P_D) sum_{x: D(x) > 0}
# |D^(x) - D(x)| over the P_D pixels with a depth value (0 when there are
# none); d|t|/dt = sign(t), sign(0) = 0.


def track_loss(out, image, depth, lam_d: float):
    """Returns (L_track, dL/dout) with dL/dout shaped like out [C][Hs][Ws]
    (zero on the semantic channels)."""
    out = _f64(out)
    I = _f64(image)
    P = out.shape[1] * out.shape[2]
    d = np.zeros_like(out)
    diff = out[:3] - I
    val = np.abs(diff).sum() / (3 * P)
    d[:3] = np.sign(diff) / (3 * P)
    if depth is not None and lam_d != 0.0:
        Dm = _f64(depth)
        has = Dm > 0
        nd = int(has.sum())
        if nd:
            dd = out[3] - Dm
            val += lam_d * np.abs(dd[has]).sum() / nd
            d[3][has] = lam_d * np.sign(dd[has]) / nd
    return float(val), d


def pose_grad(scene, cam, g, r: Render | None = None, tile_mask=None):
    """dL/dxi (6 values: translation, rotation) of L = sum g * out for the
    left perturbation T(xi) = exp(xi^) T of the world-to-camera pose."""
    if r is None:
        r = render(scene, cam, tile_mask)
    n = scene.n
    C = r.chan.shape[1]
    d_m2 = np.zeros((n, 2)); d_co = np.zeros((n, 3)); d_op = np.zeros(n); d_ch = np.zeros((n, C))
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    lib().orc_composite_bwd(ctypes.c_int64(n), _p(_f64(r.proj.mean2d)), _p(_f64(r.proj.conic)),
                            _p(_f64(scene.opacity)), _p(r.chan), ctypes.c_int32(C),
                            _p(np.ascontiguousarray(r.order, np.uint32)),
                            _p(np.ascontiguousarray(r.ranges, np.uint32)), _p(cam_array(cam)),
                            _p(_f64(g)), _p(tm), _p(d_m2), _p(d_co), _p(d_op), _p(d_ch))
    d_pose = np.zeros(6)
    lib().orc_pose_grad(ctypes.c_int64(n), _p(_f64(scene.means)), _p(_f64(scene.log_scales)),
                        _p(_f64(scene.quats)), _p(_f64(scene.opacity)), _p(cam_array(cam)), _p(d_m2), _p(d_co),
                        _p(np.ascontiguousarray(d_ch[:, 3])), _p(d_pose))
    return d_pose


def se3_exp(xi):
    """exp(xi^) for xi = (rho, phi) as a 4x4 matrix (Rodrigues; the
    translation part uses the left Jacobian V)."""
    rho = np.asarray(xi[:3], np.float64)
    phi = np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        a = np.sin(th) / th
        b = (1 - np.cos(th)) / th ** 2
        c = (th - np.sin(th)) / th ** 3
        R = np.eye(3) + a * K + b * K @ K
        V = np.eye(3) + b * K + c * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


# ------------------------------------------------ region targets, occluders
def region_targets(S, Phi, stride: int = 1, off_y: int = 0, off_x: int = 0):
    """App. D Eq. (target_discrete): G*[:, m, n] = Phi[S(u, v)] and
    V = [S(u, v) != -1] at (u, v) = (off_y + m s, off_x + n s) on the
    ceil(H/s) x ceil(W/s) grid; zero target and V = 0 where S = -1 or (u, v)
    lies outside the image.  Reading: labels outside [0, R) are treated as
    unannotated.  Straight loops (the definition)."""
    S = np.asarray(S)
    Phi = _f64(Phi)
    H, W = S.shape
    R, D = Phi.shape
    hs, ws = -(-H // stride), -(-W // stride)
    G = np.zeros((D, hs, ws))
    V = np.zeros((hs, ws), np.uint8)
    for m in range(hs):
        u = off_y + m * stride
        for n in range(ws):
            v = off_x + n * stride
            if u >= H or v >= W:
                continue
            lab = int(S[u, v])
            if 0 <= lab < R:
                G[:, m, n] = Phi[lab]
                V[m, n] = 1
    return G, V


def occluder_mask(mean2d, depth, visible, depth_map, margin: float = 0.1):
    """Occluder pruning (Sec. 3.2.1 mapping; relative margin 10%, Sec. 4.1).
    Reading: Gaussian i is an occluder when it is visible, the depth map is
    positive at the pixel holding its projected mean (floor of mean2d, inside
    the image), and its camera depth is below (1 - margin) times that depth.
    Inputs in the caller's precision; the comparison runs in that precision
    (binary32 inputs: binary32, the kernel's)."""
    mean2d = np.asarray(mean2d)
    depth = np.asarray(depth)
    Dm = np.asarray(depth_map)
    H, W = Dm.shape
    n = depth.shape[0]
    out = np.zeros(n, np.uint8)
    one = depth.dtype.type(1)
    keep = one - depth.dtype.type(margin)
    for i in range(n):
        if not visible[i]:
            continue
        x, y = mean2d[i, 0], mean2d[i, 1]
        if not (x >= 0 and y >= 0):
            continue
        c, r = int(np.floor(x)), int(np.floor(y))
        if r >= H or c >= W:
            continue
        d = Dm[r, c]
        if d > 0 and depth[i] < keep * d:
            out[i] = 1
    return out


# ------------------------------------------------------------- robust VQ
# App. C (online VQ codebook details): confidence p_nk = softmax_k(-|x_n - e_k|/tau)
# (Eq. (confidence_score)), mask m_n = [max_k p_nk >= gamma] (Eq. (mask_confidence))
# on the samples that update the EMA statistics, hard nearest-neighbour
# assignments unchanged, dead-code reinitialisation M_k <- x~, N_k <- 1 + eps
# when N_k < delta (Eq. (dead_code)) with x~ from a reservoir of recent features.
# Readings: the dead-code test runs on N after the EMA step; the j-th dead
# code in index order takes reservoir row (offset + j) mod R; the warm start
# is the masked pass with decay 0 (N = c, M = s).


def vq_confidence(X, E, tau: float):
    """conf[n] = max_k p_nk in FP64 over every codeword."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    E = np.ascontiguousarray(E, dtype=np.float32)
    N, D = X.shape
    K = E.shape[0]
    conf = np.zeros(N)
    lib().orc_vq_confidence(ctypes.c_int64(N), ctypes.c_int32(D), _p(X), ctypes.c_int32(K), _p(E),
                            ctypes.c_double(tau), _p(conf))
    return conf


def ema_update_robust(X, idx, conf, gamma: float, N_ema, M_ema, decay: float, eps: float, mode: int,
                      delta: float, reservoir, offset: int = 0):
    """Masked EMA step plus dead-code reinitialisation.  conf may be None (all
    samples count).  Returns (N, M, E, counts, dead_mask)."""
    X = _f64(X)
    idx = np.asarray(idx, dtype=np.int64)
    K, D = M_ema.shape
    use = np.ones(X.shape[0], bool) if conf is None else (np.asarray(conf) >= gamma)
    counts = np.zeros(K)
    sums = np.zeros((K, D))
    for n in range(X.shape[0]):
        if use[n]:
            counts[idx[n]] += 1.0
            sums[idx[n]] += X[n]
    N_new = decay * _f64(N_ema) + (1.0 - decay) * counts
    M_new = decay * _f64(M_ema) + (1.0 - decay) * sums
    dead = N_new < delta
    res = _f64(reservoir)
    j = 0
    for k in range(K):
        if dead[k]:
            M_new[k] = res[(offset + j) % res.shape[0]]
            N_new[k] = 1.0 + eps
            j += 1
    if mode == PAPER:
        E_new = M_new / (N_new + eps)[:, None]
    else:
        tot = N_new.sum()
        nt = (N_new + eps) / (tot + K * eps) * tot
        E_new = M_new / nt[:, None]
    return N_new, M_new, E_new, counts, dead
