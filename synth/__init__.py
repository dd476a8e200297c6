"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random inputs only.  It holds none of the method's arithmetic
(no projection, no compositing, no distances): every function returns plain
float32/int arrays and camera descriptions that both the FP64 oracle and the
HIP path consume unchanged.

Workload recipes (stand-ins for the indoor RGB-D sequences and VFM feature maps
that the paper evaluates on; no dataset item is reproduced):

* ``tiny_scene``      2,000 Gaussians, x,y ~ U[-1,1], z ~ U[2,4], log-scales
                      N(-3, 0.5), unit quaternions from normalised N(0, I4),
                      opacity sigmoid(N(0,1)), RGB U[0,1], semantic N(0,1);
                      pinhole camera fx=fy=100, 128x96, principal point at the
                      image centre, identity view.
* ``room_scene``      points on the 6 faces of a 6x4x3 m box plus the 5 exposed
                      faces of 20 floor boxes (sides U[0.2,1.0] m), allocated in
                      proportion to area, jittered by N(0, 0.01^2) per axis;
                      log-scale ln(sqrt(area/N)) + N(0, 0.3^2) per axis; the
                      other attributes as in ``tiny_scene``.
* ``room_trajectory`` a random walk of camera poses from the room centre at
                      1.5 m height, steps N(0, 0.05^2) per axis clipped 0.5 m
                      inside the walls, yaw steps N(0, 3 deg), pitch steps
                      N(0, 2 deg) clipped to +-30 deg; OpenCV camera axes.
* ``vq_mixture``      rows = centre + N(0, sigma^2 I), L2-normalised, centres
                      N(0, I); codebooks are fresh draws of the same mixture.
* ``feature_map``     VFM-like map P[D][Hf][Wf] ~ N(0,1), or an affine ramp.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Camera", "Scene", "tiny_scene", "tiny_camera", "room_scene", "room_trajectory",
    "room_camera", "upstream_grad", "vq_mixture", "vq_codebook", "feature_map",
    "affine_feature_map", "grid_shape",
]


@dataclass
class Camera:
    """Pinhole camera.  ``viewmat`` maps world to camera coordinates (row-major
    4x4, OpenCV axes: x right, y down, z forward).  The sampled grid has pixel
    (m, n) at image row ``off_y + m*stride`` and column ``off_x + n*stride``."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: np.ndarray = field(default_factory=lambda: np.eye(4, dtype=np.float32))
    near: float = 0.2
    stride: int = 1
    off_y: int = 0
    off_x: int = 0

    def with_grid(self, stride: int, off_y: int = 0, off_x: int = 0) -> "Camera":
        return replace(self, stride=int(stride), off_y=int(off_y), off_x=int(off_x))

    def with_view(self, viewmat: np.ndarray) -> "Camera":
        return replace(self, viewmat=np.asarray(viewmat, dtype=np.float32).reshape(4, 4))


def grid_shape(cam: Camera) -> tuple[int, int]:
    """(H_s, W_s) = (ceil(H/s), ceil(W/s)) -- the fixed-size sampled grid."""
    s = cam.stride
    return (cam.height + s - 1) // s, (cam.width + s - 1) // s


@dataclass
class Scene:
    means: np.ndarray       # [N,3] f32 world positions
    log_scales: np.ndarray  # [N,3] f32
    quats: np.ndarray       # [N,4] f32 (w,x,y,z), not necessarily unit
    opacity: np.ndarray     # [N]   f32 activated opacity in (0,1)
    colors: np.ndarray      # [N,3] f32
    features: np.ndarray    # [N,C_sem] f32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def c_sem(self) -> int:
        return int(self.features.shape[1])

    def subset(self, idx) -> "Scene":
        return Scene(*(np.ascontiguousarray(a[idx]) for a in
                       (self.means, self.log_scales, self.quats, self.opacity,
                        self.colors, self.features)))


def _attributes(rng: np.random.Generator, n: int, c_sem: int):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.standard_normal(n)))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    feat = rng.standard_normal((n, c_sem))
    return (q.astype(np.float32), opac.astype(np.float32), rgb.astype(np.float32),
            feat.astype(np.float32))


def tiny_scene(seed: int = 0, n: int = 2000, c_sem: int = 8) -> Scene:
    rng = np.random.default_rng(seed)
    means = np.empty((n, 3))
    means[:, 0:2] = rng.uniform(-1.0, 1.0, (n, 2))
    means[:, 2] = rng.uniform(2.0, 4.0, n)
    ls = rng.normal(-3.0, 0.5, (n, 3))
    q, o, rgb, f = _attributes(rng, n, c_sem)
    return Scene(means.astype(np.float32), ls.astype(np.float32), q, o, rgb, f)


def tiny_camera() -> Camera:
    return Camera(width=128, height=96, fx=100.0, fy=100.0, cx=64.0, cy=48.0)


ROOM = (6.0, 4.0, 3.0)


def _room_faces(rng: np.random.Generator, n_boxes: int = 20):
    """Axis-aligned rectangles (origin, edge_u, edge_v) covering the room shell
    and the exposed faces of ``n_boxes`` boxes standing on the floor."""
    X, Y, Z = ROOM
    faces = []

    def box_faces(lo, hi, skip_bottom):
        (x0, y0, z0), (x1, y1, z1) = lo, hi
        ex, ey, ez = np.array([x1 - x0, 0, 0]), np.array([0, y1 - y0, 0]), np.array([0, 0, z1 - z0])
        o = np.array([x0, y0, z0], dtype=np.float64)
        out = [(o + ez, ex, ey),             # top
               (o, ex, ez), (o + ey, ex, ez),  # y-faces
               (o, ey, ez), (o + ex, ey, ez)]  # x-faces
        if not skip_bottom:
            out.append((o, ex, ey))
        return out

    faces += box_faces((0, 0, 0), (X, Y, Z), skip_bottom=False)
    for _ in range(n_boxes):
        sx, sy, sz = rng.uniform(0.2, 1.0, 3)
        x0 = rng.uniform(0.0, X - sx)
        y0 = rng.uniform(0.0, Y - sy)
        faces += box_faces((x0, y0, 0.0), (x0 + sx, y0 + sy, sz), skip_bottom=True)
    return faces


def room_scene(n: int, seed: int = 1, c_sem: int = 16, noise: float = 0.01) -> Scene:
    rng = np.random.default_rng(seed)
    faces = _room_faces(rng)
    areas = np.array([np.linalg.norm(np.cross(u, v)) for _, u, v in faces])
    counts = rng.multinomial(n, areas / areas.sum())
    pts = []
    for (o, u, v), k in zip(faces, counts):
        a = rng.uniform(0.0, 1.0, (k, 1))
        b = rng.uniform(0.0, 1.0, (k, 1))
        pts.append(o[None, :] + a * u[None, :] + b * v[None, :])
    means = np.concatenate(pts, axis=0)
    means = means[rng.permutation(n)]
    means += rng.normal(0.0, noise, means.shape)
    ls = math.log(math.sqrt(areas.sum() / n)) + rng.normal(0.0, 0.3, (n, 3))
    q, o, rgb, f = _attributes(rng, n, c_sem)
    return Scene(means.astype(np.float32), ls.astype(np.float32), q, o, rgb, f)


def _look(pos, yaw, pitch) -> np.ndarray:
    """World->camera matrix for a camera at ``pos`` looking along (yaw, pitch),
    world z up, OpenCV camera axes."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    rc2w = np.stack([r, d, f], axis=1)
    v = np.eye(4)
    v[:3, :3] = rc2w.T
    v[:3, 3] = -rc2w.T @ np.asarray(pos, dtype=np.float64)
    return v.astype(np.float32)


def room_trajectory(n_frames: int = 100, seed: int = 10) -> list[np.ndarray]:
    rng = np.random.default_rng(seed)
    lo = np.array([0.5, 0.5, 0.5])
    hi = np.array(ROOM) - 0.5
    pos = np.array([ROOM[0] / 2, ROOM[1] / 2, 1.5])
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = 0.0
    out = []
    for _ in range(n_frames):
        out.append(_look(pos, yaw, pitch))
        pos = np.clip(pos + rng.normal(0.0, 0.05, 3), lo, hi)
        yaw += math.radians(rng.normal(0.0, 3.0))
        pitch = float(np.clip(pitch + math.radians(rng.normal(0.0, 2.0)),
                              -math.radians(30), math.radians(30)))
    return out


def room_camera(width: int, height: int, f: float, viewmat=None) -> Camera:
    cam = Camera(width=width, height=height, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0)
    if viewmat is not None:
        cam = cam.with_view(viewmat)
    return cam


def upstream_grad(c: int, hs: int, ws: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((c, hs, ws)).astype(np.float32)


def _mixture_centres(n_clusters: int, d: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n_clusters, d))


def vq_mixture(n: int, d: int, n_clusters: int, sigma: float = 0.1, seed: int = 2,
               centre_seed: int | None = None) -> np.ndarray:
    """Rows drawn from a Gaussian mixture and L2-normalised.  The cluster centres
    come from ``centre_seed`` (default: ``seed``) so that a codebook can be drawn
    from the same mixture with a different row seed."""
    centres = _mixture_centres(n_clusters, d, seed if centre_seed is None else centre_seed)
    rng = np.random.default_rng(seed + 1_000_003)
    lab = rng.integers(0, n_clusters, n)
    x = np.empty((n, d), dtype=np.float32)
    chunk = 65536
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        blk = centres[lab[s:e]] + sigma * rng.standard_normal((e - s, d))
        blk /= np.linalg.norm(blk, axis=1, keepdims=True)
        x[s:e] = blk
    return x


def vq_codebook(k: int, d: int, n_clusters: int, sigma: float = 0.1, seed: int = 3,
                centre_seed: int = 2) -> np.ndarray:
    return vq_mixture(k, d, n_clusters, sigma=sigma, seed=seed, centre_seed=centre_seed)


def feature_map(d: int, hf: int, wf: int, seed: int = 5) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((d, hf, wf)).astype(np.float32)


def affine_feature_map(d: int, hf: int, wf: int, seed: int = 6) -> np.ndarray:
    """P[c,y,x] = a_c + b_c*y + c_c*x with small-integer coefficients, so that
    bilinear interpolation reproduces it exactly in binary floating point at
    coordinates that are dyadic rationals."""
    rng = np.random.default_rng(seed)
    a, b, c = (rng.integers(-4, 5, (3, d))).astype(np.float64)
    y = np.arange(hf, dtype=np.float64)[None, :, None]
    x = np.arange(wf, dtype=np.float64)[None, None, :]
    return (a[:, None, None] + b[:, None, None] * y + c[:, None, None] * x).astype(np.float32)
