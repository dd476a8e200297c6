"""The allocation-free tile sort (xgs_tile_sort_noalloc: the library's own
scratch instead of a workspace) against xgs_tile_sort, bit for bit, on two
calls in a row (the second with a smaller input, so stale scratch from the
first is present), and its capacity error."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import gaussians, np_, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xgs():
    return require_gpu()


def sort_both(xgs, scene, cam):
    g = gaussians(scene, xgs)
    c = xgs.camera_from(cam)
    p = xgs.xgs_project(g, c)
    m = int(p.tiles_touched.to(torch.int64).sum().item())
    ref = xgs.alloc_binning(g.n, m, c)
    xgs.xgs_tile_sort(p, c, g.n, ref)
    got = xgs.alloc_binning(g.n, m, c)
    got.keys.fill_(-1)
    got.vals.fill_(-1)
    got.ranges.fill_(-1)
    got.workspace = got.workspace[:1]   # not used by the allocation-free call
    xgs.xgs_tile_sort_noalloc(p, c, g.n, got)
    torch.cuda.synchronize()
    return m, ref, got


def test_noalloc_tile_sort_equals_workspace_sort_twice(xgs):
    cases = [
        (synth.room_scene(300_000, seed=2, c_sem=1),
         synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[3])),
        (synth.tiny_scene(seed=0, n=2000), synth.tiny_camera()),
    ]
    sizes = []
    for scene, cam in cases:
        print(f"noalloc tile sort: n = {scene.n}, {cam.width}x{cam.height}", flush=True)
        m, ref, got = sort_both(xgs, scene, cam)
        sizes.append(m)
        assert int(np_(got.status)[0]) == 0 and int(np_(ref.status)[0]) == 0
        assert int(np_(got.num_instances)[0]) == int(np_(ref.num_instances)[0]) == m
        np.testing.assert_array_equal(np_(got.keys)[:m], np_(ref.keys)[:m])
        np.testing.assert_array_equal(np_(got.vals)[:m], np_(ref.vals)[:m])
        np.testing.assert_array_equal(np_(got.ranges), np_(ref.ranges))
        np.testing.assert_array_equal(np_(got.tile_order), np_(ref.tile_order))
    assert sizes[1] < sizes[0] // 10


def test_noalloc_tile_sort_rejects_sizes_beyond_its_scratch(xgs):
    """Checked on the host before any launch (null buffers would otherwise be
    rejected as invalid arguments, so the status shows which check fired)."""
    lib = xgs.lib
    cap = int(lib.xgs_tile_sort_noalloc_max_bytes())
    assert cap == 68 << 20
    assert lib.xgs_tile_sort_workspace(2_000_000, 4_000_000, 3225) <= cap  # the documented fit
    cam = xgs.camera_from(synth.room_camera(1200, 680, 600.0, synth.room_trajectory(100, seed=10)[0]))
    n, m = 2_000_000, 8_000_000
    assert lib.xgs_tile_sort_workspace(n, m, 3225) > cap
    from paper_2603_09632_amd._lib import XgsBinning, XgsProjected
    b = XgsBinning()
    b.max_instances = m
    st = lib.xgs_tile_sort_noalloc(ctypes.byref(XgsProjected()), ctypes.byref(cam), n, ctypes.byref(b), None)
    assert st == 2 and b"scratch" in lib.xgs_last_error()
    # within the limit the same null buffers are invalid arguments
    b.max_instances = 1000
    st = lib.xgs_tile_sort_noalloc(ctypes.byref(XgsProjected()), ctypes.byref(cam), 10, ctypes.byref(b), None)
    assert st == 1
