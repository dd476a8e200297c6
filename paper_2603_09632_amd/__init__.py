"""Python binding of libxgs (include/xgs.h): the MI355X hot path of the X-GS
Perceiver (arXiv 2603.09632).

Every function here only marshals torch tensors (device memory, streams) into
the C ABI of the same name; all arithmetic runs in the HIP kernels.  There is
no CPU fallback: without the built library the import fails.

Conventions: tensors live on the current CUDA (HIP) device, are contiguous
float32 unless stated, and calls are enqueued on torch's current stream.
Unsigned device arrays of the ABI are held in signed torch tensors of the same
width (uint16 -> int16, uint32 -> int32, uint64 -> int64).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import XgsBatchSlot, XgsBinning, XgsCamera, XgsError, XgsGaussians, XgsProjected, check

lib = _lib.load()

TILE = 16
SPLAT_STRIDE = 8
GRID_BILINEAR, GRID_NEAREST = 0, 1
VQ_FP32, VQ_BF16_RESCORE4 = 0, 1
EMA_PAPER, EMA_LAPLACE = 0, 1
BWD_ALL, BWD_FEATURES_ONLY, BWD_PREZEROED = 0, 1, 2

__all__ = [
    "XgsError", "Gaussians", "Projected", "Binning", "camera", "camera_from", "grid_dims",
    "xgs_project", "xgs_project_posed", "alloc_binning", "xgs_tile_sort", "xgs_tile_sort_noalloc", "xgs_render_fwd",
    "xgs_render_bwd", "xgs_render_bwd_zero",
    "xgs_grid_sample", "xgs_grid_sample_offsets", "xgs_vq_prepare", "xgs_vq_assign", "xgs_vq_stage", "xgs_vq_candidates", "xgs_vq_rescore",
    "vq_assign_workspace", "xgs_vq_ema_update", "xgs_semantic_softmax", "xgs_semantic_softmax_bwd",
    "xgs_semantic_loss", "semantic_step", "xgs_pose_grad", "xgs_tracking_loss", "tracking_step", "xgs_region_targets",
    "xgs_occluder_mask", "xgs_vq_assign_conf", "xgs_vq_ema_update_robust", "render", "BatchLayout",
    "batch_layout", "batch_table", "xgs_batch_check", "xgs_batch_project", "xgs_batch_render_fwd", "render_batch",
]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise XgsError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise XgsError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- camera
def camera(width, height, fx, fy, cx, cy, viewmat=None, near=0.2, stride=1, off_y=0, off_x=0) -> XgsCamera:
    c = XgsCamera()
    c.width, c.height = int(width), int(height)
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    vm = [1.0, 0, 0, 0, 0, 1.0, 0, 0, 0, 0, 1.0, 0, 0, 0, 0, 1.0] if viewmat is None else \
        [float(v) for v in torch.as_tensor(viewmat, dtype=torch.float64).reshape(16).tolist()]
    for i, v in enumerate(vm):
        c.viewmat[i] = v
    c.near_plane = float(near)
    c.stride, c.off_y, c.off_x = int(stride), int(off_y), int(off_x)
    return c


def camera_from(obj) -> XgsCamera:
    """From any object with width/height/fx/fy/cx/cy/viewmat/near/stride/off_y/off_x."""
    if isinstance(obj, XgsCamera):
        return obj
    return camera(obj.width, obj.height, obj.fx, obj.fy, obj.cx, obj.cy, obj.viewmat,
                  getattr(obj, "near", 0.2), getattr(obj, "stride", 1), getattr(obj, "off_y", 0),
                  getattr(obj, "off_x", 0))


def grid_dims(cam) -> tuple[int, int, int, int]:
    """(H_s, W_s, tiles_y, tiles_x) of the sampled grid."""
    c = camera_from(cam)
    hs, ws, ty, tx = (ctypes.c_int32() for _ in range(4))
    check(lib.xgs_grid_dims(ctypes.byref(c), ctypes.byref(hs), ctypes.byref(ws), ctypes.byref(ty),
                            ctypes.byref(tx)), "xgs_grid_dims")
    return hs.value, ws.value, ty.value, tx.value


# ------------------------------------------------------------- Gaussians
@dataclass
class Gaussians:
    means: torch.Tensor       # [n,3]
    log_scales: torch.Tensor  # [n,3]
    quats: torch.Tensor       # [n,4] (w,x,y,z)
    opacity: torch.Tensor     # [n]   activated
    colors: torch.Tensor      # [n,3]
    features: torch.Tensor    # [n,c_sem]

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def c_sem(self) -> int:
        return int(self.features.shape[1]) if self.features is not None and self.features.dim() == 2 else 0

    def struct(self) -> XgsGaussians:
        s = XgsGaussians()
        s.n, s.c_sem = self.n, self.c_sem
        s.means, s.log_scales, s.quats, s.opacity, s.colors = (
            _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats), _ptr(self.opacity),
            _ptr(self.colors))
        s.features = _ptr(self.features) if self.c_sem > 0 else None
        return s

    @staticmethod
    def empty_like(g: "Gaussians") -> "Gaussians":
        return Gaussians(*(torch.empty_like(t) for t in (g.means, g.log_scales, g.quats, g.opacity,
                                                          g.colors, g.features)))


@dataclass
class Projected:
    splat: torch.Tensor          # [n,8] f32
    radius: torch.Tensor         # [n]   i32
    tile_rect: torch.Tensor      # [n,4] u16 (as int16)
    tiles_touched: torch.Tensor  # [n]   u32 (as int32)

    @staticmethod
    def alloc(n: int, device=None) -> "Projected":
        d = device or torch.device("cuda")
        return Projected(torch.empty((n, SPLAT_STRIDE), dtype=torch.float32, device=d),
                         torch.empty(n, dtype=torch.int32, device=d),
                         torch.empty((n, 4), dtype=torch.int16, device=d),
                         torch.empty(n, dtype=torch.int32, device=d))

    def struct(self) -> XgsProjected:
        s = XgsProjected()
        s.splat, s.radius, s.tile_rect, s.tiles_touched = (_ptr(self.splat), _ptr(self.radius),
                                                           _ptr(self.tile_rect), _ptr(self.tiles_touched))
        return s


@dataclass
class Binning:
    keys: torch.Tensor           # [cap] u64 (as int64)
    vals: torch.Tensor           # [cap] u32 (as int32)
    ranges: torch.Tensor         # [tiles,2] u32 (as int32)
    num_instances: torch.Tensor  # [1] int64
    status: torch.Tensor         # [1] int32
    workspace: torch.Tensor      # u8
    max_instances: int
    tile_order: Optional[torch.Tensor] = None  # [tiles] u32 (as int32); None: id order

    def struct(self) -> XgsBinning:
        s = XgsBinning()
        s.keys, s.vals, s.ranges, s.num_instances, s.status = (
            _ptr(self.keys), _ptr(self.vals), _ptr(self.ranges), _ptr(self.num_instances), _ptr(self.status))
        s.max_instances = int(self.max_instances)
        s.tile_order = _ptr(self.tile_order)
        return s


def xgs_project(g: Gaussians, cam, out: Optional[Projected] = None, stream=None) -> Projected:
    c = camera_from(cam)
    out = out or Projected.alloc(g.n, g.means.device)
    gs, ps = g.struct(), out.struct()
    check(lib.xgs_project(ctypes.byref(gs), ctypes.byref(c), ctypes.byref(ps), _stream(stream)), "xgs_project")
    return out


def xgs_project_posed(g: Gaussians, cam, viewmat_dev: torch.Tensor, out: Optional[Projected] = None,
                      stream=None) -> Projected:
    """Projection with the world->camera matrix taken from a device tensor [4,4]."""
    c = camera_from(cam)
    out = out or Projected.alloc(g.n, g.means.device)
    gs, ps = g.struct(), out.struct()
    check(lib.xgs_project_posed(ctypes.byref(gs), ctypes.byref(c), _ptr(viewmat_dev), ctypes.byref(ps),
                                _stream(stream)), "xgs_project_posed")
    return out


def alloc_binning(n: int, max_instances: int, cam, device=None) -> Binning:
    d = device or torch.device("cuda")
    _, _, ty, tx = grid_dims(cam)
    cap = max(int(max_instances), 1)
    ws = int(lib.xgs_tile_sort_workspace(n, cap, ty * tx))
    return Binning(torch.empty(cap, dtype=torch.int64, device=d), torch.empty(cap, dtype=torch.int32, device=d),
                   torch.empty((ty * tx, 2), dtype=torch.int32, device=d),
                   torch.zeros(1, dtype=torch.int64, device=d), torch.zeros(1, dtype=torch.int32, device=d),
                   torch.empty(max(ws, 1), dtype=torch.uint8, device=d), cap,
                   torch.empty(ty * tx, dtype=torch.int32, device=d))


def xgs_tile_sort(p: Projected, cam, n: int, b: Binning, stream=None) -> Binning:
    c = camera_from(cam)
    ps, bs = p.struct(), b.struct()
    check(lib.xgs_tile_sort(ctypes.byref(ps), ctypes.byref(c), int(n), _ptr(b.workspace), b.workspace.numel(),
                            ctypes.byref(bs), _stream(stream)), "xgs_tile_sort")
    return b


def xgs_tile_sort_noalloc(p: Projected, cam, n: int, b: Binning, stream=None) -> Binning:
    """xgs_tile_sort in the library's own scratch (b.workspace is not used)."""
    c = camera_from(cam)
    ps, bs = p.struct(), b.struct()
    check(lib.xgs_tile_sort_noalloc(ctypes.byref(ps), ctypes.byref(c), int(n), ctypes.byref(bs), _stream(stream)),
          "xgs_tile_sort_noalloc")
    return b


# ---------------------------------------------------------------- batches
@dataclass
class BatchLayout:
    """Where each request of a batch sits: Gaussian rows and tile-grid band."""
    tiles_x: int           # width of the virtual tile grid
    tile_rows: int         # rows of the virtual grid (capacity)
    cap_gaussians: int     # Gaussian rows of the batch buffers (capacity)
    gauss_base: list       # first global Gaussian row per slot
    row_base: list         # first tile row per slot

    def sort_camera(self) -> XgsCamera:
        """Camera whose grid is the virtual tile grid (for xgs_tile_sort)."""
        return camera(16 * self.tiles_x, 16 * self.tile_rows, 1.0, 1.0, 0.0, 0.0)

    @property
    def tiles(self) -> int:
        return self.tiles_x * self.tile_rows


def batch_layout(ns, cams, tiles_x: int, tile_rows: int, cap_gaussians: int) -> BatchLayout:
    """Packs requests with ns[i] Gaussians and cameras cams[i] into ascending
    Gaussian rows and tile-row bands; raises XgsError when they do not fit."""
    gb, rb, g0, r0 = [], [], 0, 0
    for n, c in zip(ns, cams):
        _, _, ty, tx = grid_dims(c)
        if tx > tiles_x:
            raise XgsError(f"a request is {tx} tiles wide, the batch grid {tiles_x}")
        gb.append(g0)
        rb.append(r0)
        g0 += int(n)
        r0 += ty
    if g0 > cap_gaussians or r0 > tile_rows:
        raise XgsError(f"batch needs {g0} Gaussian rows and {r0} tile rows, capacity {cap_gaussians} / {tile_rows}")
    return BatchLayout(tiles_x, tile_rows, cap_gaussians, gb, rb)


def batch_table(items, layout: BatchLayout):
    """Host slot table (ctypes array) for items = [(Gaussians, camera, out,
    final_T, n_last)] in layout's places."""
    arr = (XgsBatchSlot * max(len(items), 1))()
    for k, (g, cam, out, fT, nl) in enumerate(items):
        e = arr[k]
        e.g = g.struct()
        e.cam = camera_from(cam)
        e.out, e.final_T, e.n_last = _ptr(out), _ptr(fT), _ptr(nl)
        e.gauss_base = layout.gauss_base[k]
        e.row_base = layout.row_base[k]
    return arr


def xgs_batch_check(table, n_slots: int, layout: BatchLayout, c_sem: int):
    check(lib.xgs_batch_check(table, int(n_slots), layout.cap_gaussians, layout.tiles_x, layout.tile_rows,
                              int(c_sem)), "xgs_batch_check")


def xgs_batch_project(d_table: torch.Tensor, n_slots: int, layout: BatchLayout, out: Projected, stream=None):
    ps = out.struct()
    check(lib.xgs_batch_project(_ptr(d_table), int(n_slots), layout.cap_gaussians, layout.tiles_x, layout.tile_rows,
                                ctypes.byref(ps), _stream(stream)), "xgs_batch_project")
    return out


def xgs_batch_render_fwd(d_table: torch.Tensor, n_slots: int, c_sem: int, layout: BatchLayout, p: Projected,
                         b: Binning, stream=None):
    ps, bs = p.struct(), b.struct()
    check(lib.xgs_batch_render_fwd(_ptr(d_table), int(n_slots), int(c_sem), layout.tiles_x, layout.tile_rows,
                                   ctypes.byref(ps), ctypes.byref(bs), _stream(stream)), "xgs_batch_render_fwd")


def render_batch(requests, tiles_x: int = 75, tile_rows: Optional[int] = None, cap_gaussians: Optional[int] = None,
                 max_instances: Optional[int] = None, stream=None):
    """Renders requests = [(Gaussians, camera)] in one batch (project, tile
    sort and forward each one launch sequence for all of them).  Returns
    ([(out, final_T, n_last)], Binning)."""
    cams = [camera_from(c) for _, c in requests]
    ns = [g.n for g, _ in requests]
    rows = sum(grid_dims(c)[2] for c in cams)
    layout = batch_layout(ns, cams, tiles_x, tile_rows or max(rows, 1), cap_gaussians or max(sum(ns), 1))
    dev = requests[0][0].means.device
    c_sem = requests[0][0].c_sem
    outs = []
    for g, c in zip((g for g, _ in requests), cams):
        hs, ws, _, _ = grid_dims(c)
        outs.append((torch.empty((4 + c_sem, hs, ws), device=dev), torch.empty((hs, ws), device=dev),
                     torch.empty((hs, ws), dtype=torch.int32, device=dev)))
    table = batch_table([(g, c, *o) for (g, _), c, o in zip(requests, cams, outs)], layout)
    xgs_batch_check(table, len(requests), layout, c_sem)
    d_table = torch.frombuffer(bytearray(bytes(table)), dtype=torch.uint8).to(dev)
    p = Projected.alloc(layout.cap_gaussians, dev)
    xgs_batch_project(d_table, len(requests), layout, p, stream=stream)
    if max_instances is None:
        max_instances = int(p.tiles_touched.to(torch.int64).sum().item())
    scam = layout.sort_camera()
    b = alloc_binning(layout.cap_gaussians, max(max_instances, 1), scam, dev)
    xgs_tile_sort(p, scam, layout.cap_gaussians, b, stream=stream)
    xgs_batch_render_fwd(d_table, len(requests), c_sem, layout, p, b, stream=stream)
    return outs, b


def xgs_render_fwd(g: Gaussians, p: Projected, b: Binning, cam, out=None, final_T=None, n_last=None,
                   stream=None):
    c = camera_from(cam)
    hs, ws, _, _ = grid_dims(c)
    dev = g.means.device
    out = out if out is not None else torch.empty((4 + g.c_sem, hs, ws), dtype=torch.float32, device=dev)
    final_T = final_T if final_T is not None else torch.empty((hs, ws), dtype=torch.float32, device=dev)
    n_last = n_last if n_last is not None else torch.empty((hs, ws), dtype=torch.int32, device=dev)
    gs, ps, bs = g.struct(), p.struct(), b.struct()
    check(lib.xgs_render_fwd(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(bs), ctypes.byref(c), _ptr(out),
                             _ptr(final_T), _ptr(n_last), _stream(stream)), "xgs_render_fwd")
    return out, final_T, n_last


def xgs_render_bwd(g: Gaussians, p: Projected, b: Binning, cam, d_out, final_T, n_last,
                   flags: int = BWD_ALL, grads: Optional[Gaussians] = None, workspace=None,
                   stream=None) -> Gaussians:
    c = camera_from(cam)
    grads = grads or Gaussians.empty_like(g)
    need = int(lib.xgs_render_bwd_workspace(g.n))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=g.means.device)
    gs, ps, bs, gr = g.struct(), p.struct(), b.struct(), grads.struct()
    check(lib.xgs_render_bwd(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(bs), ctypes.byref(c), _ptr(d_out),
                             _ptr(final_T), _ptr(n_last), int(flags), ctypes.byref(gr), _ptr(workspace),
                             workspace.numel(), _stream(stream)), "xgs_render_bwd")
    return grads


def xgs_render_bwd_zero(g: Gaussians, grads: Gaussians, workspace: torch.Tensor, flags: int = BWD_ALL, stream=None):
    """The zeroing of xgs_render_bwd on its own (then call it with
    flags | BWD_PREZEROED)."""
    gs, gr = g.struct(), grads.struct()
    check(lib.xgs_render_bwd_zero(ctypes.byref(gs), int(flags), ctypes.byref(gr), _ptr(workspace), workspace.numel(),
                                  _stream(stream)), "xgs_render_bwd_zero")


def xgs_grid_sample(P: torch.Tensor, H: int, W: int, stride: int = 1, off_y: int = 0, off_x: int = 0,
                    mode: int = GRID_BILINEAR, G=None, V=None, stream=None):
    D, Hf, Wf = P.shape
    hs, ws = -(-H // stride), -(-W // stride)
    G = G if G is not None else torch.empty((D, hs, ws), dtype=torch.float32, device=P.device)
    V = V if V is not None else torch.empty((hs, ws), dtype=torch.uint8, device=P.device)
    check(lib.xgs_grid_sample(_ptr(P), D, Hf, Wf, int(H), int(W), int(stride), int(off_y), int(off_x), int(mode),
                              _ptr(G), _ptr(V), _stream(stream)), "xgs_grid_sample")
    return G, V


def xgs_grid_sample_offsets(P: torch.Tensor, H: int, W: int, stride: int, mode: int = GRID_BILINEAR, G=None, V=None,
                            stream=None):
    """Every offset's grid of one stride in one launch: G [s*s, D, hs, ws],
    V [s*s, hs, ws]; grid oy * s + ox equals xgs_grid_sample(..., oy, ox)."""
    D, Hf, Wf = P.shape
    hs, ws = -(-H // stride), -(-W // stride)
    n = stride * stride
    G = G if G is not None else torch.empty((n, D, hs, ws), dtype=torch.float32, device=P.device)
    V = V if V is not None else torch.empty((n, hs, ws), dtype=torch.uint8, device=P.device)
    check(lib.xgs_grid_sample_offsets(_ptr(P), D, Hf, Wf, int(H), int(W), int(stride), int(mode), _ptr(G), _ptr(V),
                                      _stream(stream)), "xgs_grid_sample_offsets")
    return G, V


def xgs_vq_prepare(E: torch.Tensor, E_bf16=None, e_norm2=None, stream=None):
    K, D = E.shape
    E_bf16 = E_bf16 if E_bf16 is not None else torch.empty((K, D), dtype=torch.int16, device=E.device)
    e_norm2 = e_norm2 if e_norm2 is not None else torch.empty(K, dtype=torch.float32, device=E.device)
    check(lib.xgs_vq_prepare(_ptr(E), K, D, _ptr(E_bf16), _ptr(e_norm2), _stream(stream)), "xgs_vq_prepare")
    return E_bf16, e_norm2


def vq_assign_workspace(N: int, D: int, K: int, precision: int = VQ_BF16_RESCORE4, device=None) -> torch.Tensor:
    nbytes = int(lib.xgs_vq_assign_workspace(N, D, K, int(precision)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or "cuda")


def xgs_vq_assign(X: torch.Tensor, E: torch.Tensor, E_bf16=None, e_norm2=None, precision: int = VQ_BF16_RESCORE4,
                  idx=None, dist=None, workspace=None, stream=None):
    N, D = X.shape
    K = E.shape[0]
    idx = idx if idx is not None else torch.empty(N, dtype=torch.int32, device=X.device)
    dist = dist if dist is not None else torch.empty(N, dtype=torch.float32, device=X.device)
    if workspace is None:
        workspace = vq_assign_workspace(N, D, K, precision, X.device)
    check(lib.xgs_vq_assign(_ptr(X), N, D, _ptr(E), _ptr(E_bf16), _ptr(e_norm2), K, int(precision), _ptr(idx),
                            _ptr(dist), _ptr(workspace), workspace.numel(), _stream(stream)), "xgs_vq_assign")
    return idx, dist


def xgs_vq_stage(X: torch.Tensor, E_bf16: torch.Tensor, e_norm2: torch.Tensor, workspace: torch.Tensor,
                 stream=None):
    N, D = X.shape
    K = E_bf16.shape[0]
    check(lib.xgs_vq_stage(_ptr(X), N, D, _ptr(E_bf16), _ptr(e_norm2), K, _ptr(workspace), workspace.numel(),
                           _stream(stream)), "xgs_vq_stage")


def xgs_vq_candidates(N: int, D: int, K: int, workspace: torch.Tensor, stream=None):
    check(lib.xgs_vq_candidates(N, D, K, _ptr(workspace), workspace.numel(), _stream(stream)), "xgs_vq_candidates")


def xgs_vq_rescore(X: torch.Tensor, E: torch.Tensor, workspace: torch.Tensor, idx=None, dist=None, stream=None):
    N, D = X.shape
    K = E.shape[0]
    idx = idx if idx is not None else torch.empty(N, dtype=torch.int32, device=X.device)
    dist = dist if dist is not None else torch.empty(N, dtype=torch.float32, device=X.device)
    check(lib.xgs_vq_rescore(_ptr(X), N, D, _ptr(E), K, _ptr(idx), _ptr(dist), _ptr(workspace), workspace.numel(),
                             _stream(stream)), "xgs_vq_rescore")
    return idx, dist


def xgs_region_targets(S: torch.Tensor, Phi: torch.Tensor, stride: int = 1, off_y: int = 0, off_x: int = 0,
                       G=None, V=None, stream=None):
    H, W = S.shape
    R, D = Phi.shape
    hs, ws = -(-H // stride), -(-W // stride)
    G = G if G is not None else torch.empty((D, hs, ws), dtype=torch.float32, device=S.device)
    V = V if V is not None else torch.empty((hs, ws), dtype=torch.uint8, device=S.device)
    check(lib.xgs_region_targets(_ptr(S), H, W, _ptr(Phi), R, D, int(stride), int(off_y), int(off_x), _ptr(G),
                                 _ptr(V), _stream(stream)), "xgs_region_targets")
    return G, V


def xgs_occluder_mask(p: "Projected", n: int, depth_map: torch.Tensor, margin: float = 0.1, prune=None, count=None,
                      stream=None):
    H, W = depth_map.shape
    prune = prune if prune is not None else torch.empty(n, dtype=torch.uint8, device=depth_map.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=depth_map.device)
    ps = p.struct()
    check(lib.xgs_occluder_mask(ctypes.byref(ps), n, _ptr(depth_map), H, W, float(margin), _ptr(prune), _ptr(count),
                                _stream(stream)), "xgs_occluder_mask")
    return prune, count


def xgs_pose_grad(g: Gaussians, p: Projected, cam, workspace: torch.Tensor, d_pose=None, stream=None):
    """dL/dxi (translation, rotation) of the left pose perturbation; call after
    xgs_render_bwd(..., workspace=workspace) on the same stream."""
    c = camera_from(cam)
    d_pose = d_pose if d_pose is not None else torch.empty(6, dtype=torch.float32, device=g.means.device)
    gs, ps = g.struct(), p.struct()
    check(lib.xgs_pose_grad(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(c), _ptr(workspace), workspace.numel(),
                            _ptr(d_pose), _stream(stream)), "xgs_pose_grad")
    return d_pose


def xgs_tracking_loss(out: torch.Tensor, image: torch.Tensor, depth=None, lam_d: float = 1.0, d_out=None, loss=None,
                      workspace=None, stream=None):
    C, Hs, Ws = out.shape
    d_out = d_out if d_out is not None else torch.empty_like(out)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=out.device)
    if workspace is None:
        workspace = torch.empty(int(lib.xgs_tracking_loss_workspace(Hs, Ws)), dtype=torch.uint8, device=out.device)
    check(lib.xgs_tracking_loss(_ptr(out), C, Hs, Ws, _ptr(image), _ptr(depth), float(lam_d), _ptr(d_out), _ptr(loss),
                                _ptr(workspace), workspace.numel(), _stream(stream)), "xgs_tracking_loss")
    return loss, d_out


def tracking_step(g: Gaussians, p: Projected, b: Binning, cam, image: torch.Tensor, depth=None, lam_d: float = 1.0,
                  workspace=None, stream=None):
    """One tracking evaluation with the map frozen (Eq. (tracking)): render,
    L1 photometric + depth loss, backward, and the pose gradient.  ``p`` and
    ``b`` must come from xgs_project / xgs_tile_sort at ``cam``.  Returns
    (loss [1], dL/dxi [6], rendered map)."""
    out, fT, nl = xgs_render_fwd(g, p, b, cam, stream=stream)
    loss, d_out = xgs_tracking_loss(out, image, depth, lam_d, stream=stream)
    need = int(lib.xgs_render_bwd_workspace(g.n))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=g.means.device)
    xgs_render_bwd(g, p, b, cam, d_out, fT, nl, workspace=workspace, stream=stream)
    d_pose = xgs_pose_grad(g, p, cam, workspace, stream=stream)
    return loss, d_pose, out


def xgs_semantic_softmax(z: torch.Tensor, w=None, stream=None) -> torch.Tensor:
    N, L = z.shape
    w = w if w is not None else torch.empty_like(z)
    check(lib.xgs_semantic_softmax(_ptr(z), N, L, _ptr(w), _stream(stream)), "xgs_semantic_softmax")
    return w


def xgs_semantic_softmax_bwd(w: torch.Tensor, dw: torch.Tensor, dz=None, stream=None) -> torch.Tensor:
    N, L = w.shape
    dz = dz if dz is not None else torch.empty_like(w)
    check(lib.xgs_semantic_softmax_bwd(_ptr(w), _ptr(dw), N, L, _ptr(dz), _stream(stream)),
          "xgs_semantic_softmax_bwd")
    return dz


def xgs_semantic_loss(wmap: torch.Tensor, E: torch.Tensor, Gstar: torch.Tensor, V=None, lam: float = 1.0,
                      d_out=None, loss=None, workspace=None, stream=None):
    """Masked cosine + L1 grid loss of the decoded map E^T w(x) (wmap is the
    [4+L][Hs][Ws] render); returns (loss [1] device tensor, d_out)."""
    C, Hs, Ws = wmap.shape
    L, D = E.shape
    assert C == 4 + L and Gstar.shape == (D, Hs, Ws)
    d_out = d_out if d_out is not None else torch.empty_like(wmap)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=wmap.device)
    if workspace is None:
        workspace = torch.empty(int(lib.xgs_semantic_loss_workspace(Hs, Ws)), dtype=torch.uint8,
                                device=wmap.device)
    check(lib.xgs_semantic_loss(_ptr(wmap), L, Hs, Ws, _ptr(E), D, _ptr(Gstar), _ptr(V), float(lam), _ptr(d_out),
                                _ptr(loss), _ptr(workspace), workspace.numel(), _stream(stream)),
          "xgs_semantic_loss")
    return loss, d_out


def semantic_step(g: "Gaussians", p: "Projected", b: "Binning", cam, z: torch.Tensor, E: torch.Tensor,
                  Gstar: torch.Tensor, V=None, lam: float = 1.0, stream=None):
    """One semantic-phase evaluation with the geometry frozen (Sec. 3.2.2):
    w = softmax(z) rendered as the semantic channels over the given binning,
    decoded, masked loss against Gstar, and dL/dz through the feature-only
    backward.  ``g`` supplies the frozen geometry and colours; its features are
    replaced by w.  Returns (loss [1], dL/dz [N][L], rendered map)."""
    w = xgs_semantic_softmax(z, stream=stream)
    gw = Gaussians(g.means, g.log_scales, g.quats, g.opacity, g.colors, w)
    out, fT, nl = xgs_render_fwd(gw, p, b, cam, stream=stream)
    loss, d_out = xgs_semantic_loss(out, E, Gstar, V, lam, stream=stream)
    grads = xgs_render_bwd(gw, p, b, cam, d_out, fT, nl, flags=BWD_FEATURES_ONLY, stream=stream)
    dz = xgs_semantic_softmax_bwd(w, grads.features, stream=stream)
    return loss, dz, out


def xgs_vq_assign_conf(X: torch.Tensor, E: torch.Tensor, E_bf16, e_norm2, tau: float = 0.7, idx=None, dist=None,
                       conf=None, workspace=None, stream=None):
    N, D = X.shape
    K = E.shape[0]
    idx = idx if idx is not None else torch.empty(N, dtype=torch.int32, device=X.device)
    dist = dist if dist is not None else torch.empty(N, dtype=torch.float32, device=X.device)
    conf = conf if conf is not None else torch.empty(N, dtype=torch.float32, device=X.device)
    if workspace is None:
        workspace = vq_assign_workspace(N, D, K, VQ_BF16_RESCORE4, X.device)
    check(lib.xgs_vq_assign_conf(_ptr(X), N, D, _ptr(E), _ptr(E_bf16), _ptr(e_norm2), K, float(tau), _ptr(idx),
                                 _ptr(dist), _ptr(conf), _ptr(workspace), workspace.numel(), _stream(stream)),
          "xgs_vq_assign_conf")
    return idx, dist, conf


def xgs_vq_ema_update_robust(X, idx, conf, gamma: float, N_ema, M_ema, E, E_bf16=None, e_norm2=None,
                             decay: float = 0.96, eps: float = 1e-5, mode: int = EMA_PAPER, delta: float = 0.0,
                             reservoir=None, offset: int = 0, counts=None, n_dead=None, workspace=None, stream=None):
    N, D = X.shape
    K = M_ema.shape[0]
    counts = counts if counts is not None else torch.empty(K, dtype=torch.float32, device=X.device)
    n_dead = n_dead if n_dead is not None else torch.empty(1, dtype=torch.int32, device=X.device)
    need = int(lib.xgs_vq_ema_workspace(N, D, K))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    R = 0 if reservoir is None else reservoir.shape[0]
    check(lib.xgs_vq_ema_update_robust(_ptr(X), _ptr(idx), _ptr(conf), float(gamma), N, D, K, _ptr(N_ema),
                                       _ptr(M_ema), _ptr(E), _ptr(E_bf16), _ptr(e_norm2), _ptr(counts), float(decay),
                                       float(eps), int(mode), float(delta), _ptr(reservoir), R, int(offset),
                                       _ptr(n_dead), _ptr(workspace), workspace.numel(), _stream(stream)),
          "xgs_vq_ema_update_robust")
    return counts, n_dead


def xgs_vq_ema_update(X, idx, N_ema, M_ema, E, E_bf16=None, e_norm2=None, decay: float = 0.99,
                      eps: float = 1e-5, mode: int = EMA_LAPLACE, counts=None, workspace=None, stream=None):
    N, D = X.shape
    K = E.shape[0]
    need = int(lib.xgs_vq_ema_workspace(N, D, K))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    counts = counts if counts is not None else torch.empty(K, dtype=torch.float32, device=X.device)
    check(lib.xgs_vq_ema_update(_ptr(X), _ptr(idx), N, D, K, _ptr(N_ema), _ptr(M_ema), _ptr(E), _ptr(E_bf16),
                                _ptr(e_norm2), _ptr(counts), float(decay), float(eps), int(mode),
                                _ptr(workspace), workspace.numel(), _stream(stream)), "xgs_vq_ema_update")
    return counts


def render(g: Gaussians, cam, max_instances: Optional[int] = None, stream=None):
    """project -> tile_sort -> render_fwd.  Without max_instances the exact
    instance count is read back once (a host synchronisation)."""
    c = camera_from(cam)
    p = xgs_project(g, c, stream=stream)
    if max_instances is None:
        max_instances = int(p.tiles_touched.to(torch.int64).sum().item())
    b = alloc_binning(g.n, max_instances, c, g.means.device)
    xgs_tile_sort(p, c, g.n, b, stream=stream)
    out, final_T, n_last = xgs_render_fwd(g, p, b, c, stream=stream)
    return out, final_T, n_last, p, b
