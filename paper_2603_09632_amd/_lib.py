"""ctypes declarations of the C ABI in include/xgs.h.

Loading order matters: torch is imported first so that libxgs.so binds to the
HIP runtime torch already loaded (both use the soname libamdhip64.so.7); the
streams and device pointers that torch hands out are then valid in the
library.  A missing library is an error, never a silent fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL below)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxgs.so")

c_int32, c_int64, c_float, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                                ctypes.c_void_p, ctypes.c_size_t)
P = ctypes.POINTER


class XgsCamera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("viewmat", c_float * 16), ("near_plane", c_float),
                ("stride", c_int32), ("off_y", c_int32), ("off_x", c_int32)]


class XgsGaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("c_sem", c_int32), ("reserved", c_int32), ("means", c_void_p),
                ("log_scales", c_void_p), ("quats", c_void_p), ("opacity", c_void_p),
                ("colors", c_void_p), ("features", c_void_p)]


XgsGaussiansGrad = XgsGaussians  # same layout, writable pointers


class XgsProjected(ctypes.Structure):
    _fields_ = [("splat", c_void_p), ("radius", c_void_p), ("tile_rect", c_void_p),
                ("tiles_touched", c_void_p)]


class XgsBinning(ctypes.Structure):
    _fields_ = [("keys", c_void_p), ("vals", c_void_p), ("ranges", c_void_p),
                ("num_instances", c_void_p), ("status", c_void_p), ("max_instances", c_int64),
                ("tile_order", c_void_p)]


class XgsBatchSlot(ctypes.Structure):
    _fields_ = [("g", XgsGaussians), ("cam", XgsCamera), ("out", c_void_p), ("final_T", c_void_p),
                ("n_last", c_void_p), ("gauss_base", c_int64), ("row_base", c_int32), ("reserved", c_int32)]


SIGNATURES = {
    "xgs_status_string": (ctypes.c_char_p, [c_int32]),
    "xgs_last_error": (ctypes.c_char_p, []),
    "xgs_version": (c_int32, []),
    "xgs_grid_dims": (c_int32, [P(XgsCamera), P(c_int32), P(c_int32), P(c_int32), P(c_int32)]),
    "xgs_project": (c_int32, [P(XgsGaussians), P(XgsCamera), P(XgsProjected), c_void_p]),
    "xgs_project_posed": (c_int32, [P(XgsGaussians), P(XgsCamera), c_void_p, P(XgsProjected), c_void_p]),
    "xgs_tile_sort_workspace": (c_size_t, [c_int64, c_int64, c_int32]),
    "xgs_tile_sort": (c_int32, [P(XgsProjected), P(XgsCamera), c_int64, c_void_p, c_size_t,
                                P(XgsBinning), c_void_p]),
    "xgs_tile_sort_noalloc_max_bytes": (c_size_t, []),
    "xgs_tile_sort_noalloc": (c_int32, [P(XgsProjected), P(XgsCamera), c_int64, P(XgsBinning), c_void_p]),
    "xgs_batch_check": (c_int32, [P(XgsBatchSlot), c_int32, c_int64, c_int32, c_int32, c_int32]),
    "xgs_batch_project": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_int32, P(XgsProjected), c_void_p]),
    "xgs_batch_render_fwd": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, P(XgsProjected),
                                       P(XgsBinning), c_void_p]),
    "xgs_render_fwd": (c_int32, [P(XgsGaussians), P(XgsProjected), P(XgsBinning), P(XgsCamera),
                                 c_void_p, c_void_p, c_void_p, c_void_p]),
    "xgs_render_bwd_zero": (c_int32, [P(XgsGaussians), c_int32, P(XgsGaussiansGrad), c_void_p, c_size_t, c_void_p]),
    "xgs_render_bwd_workspace": (c_size_t, [c_int64]),
    "xgs_render_bwd": (c_int32, [P(XgsGaussians), P(XgsProjected), P(XgsBinning), P(XgsCamera),
                                 c_void_p, c_void_p, c_void_p, c_int32, P(XgsGaussiansGrad),
                                 c_void_p, c_size_t, c_void_p]),
    "xgs_grid_sample": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                                  c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "xgs_grid_sample_offsets": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                                          c_int32, c_void_p, c_void_p, c_void_p]),
    "xgs_vq_assign_workspace": (c_size_t, [c_int64, c_int32, c_int32, c_int32]),
    "xgs_vq_prepare": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "xgs_vq_assign": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "xgs_vq_stage": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_size_t,
                               c_void_p]),
    "xgs_vq_candidates": (c_int32, [c_int64, c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
    "xgs_vq_rescore": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                 c_size_t, c_void_p]),
    "xgs_pose_grad": (c_int32, [P(XgsGaussians), P(XgsProjected), P(XgsCamera), c_void_p, c_size_t, c_void_p,
                                c_void_p]),
    "xgs_tracking_loss_workspace": (c_size_t, [c_int32, c_int32]),
    "xgs_tracking_loss": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_float, c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "xgs_region_targets": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                     c_int32, c_void_p, c_void_p, c_void_p]),
    "xgs_occluder_mask": (c_int32, [P(XgsProjected), c_int64, c_void_p, c_int32, c_int32, c_float, c_void_p,
                                    c_void_p, c_void_p]),
    "xgs_semantic_softmax": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "xgs_semantic_softmax_bwd": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "xgs_semantic_loss_workspace": (c_size_t, [c_int32, c_int32]),
    "xgs_semantic_loss": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                    c_float, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "xgs_vq_assign_conf": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_float,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "xgs_vq_ema_update_robust": (c_int32, [c_void_p, c_void_p, c_void_p, c_float, c_int64, c_int32, c_int32,
                                           c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float,
                                           c_float, c_int32, c_float, c_void_p, c_int32, c_int64, c_void_p,
                                           c_void_p, c_size_t, c_void_p]),
    "xgs_vq_ema_workspace": (c_size_t, [c_int64, c_int32, c_int32]),
    "xgs_vq_ema_update": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float,
                                    c_float, c_int32, c_void_p, c_size_t, c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libxgs.so and declares every exported function."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2603_09632_amd/build.py`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class XgsError(RuntimeError):
    pass


def check(status: int, what: str) -> None:
    if status != 0:
        lib = load()
        raise XgsError(f"{what}: {lib.xgs_status_string(status).decode()} -- "
                       f"{lib.xgs_last_error().decode()}")
