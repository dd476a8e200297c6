"""The C-ABI library loads and exports every symbol include/xgs.h declares
(no GPU needed; only host-side calls that launch nothing are made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xgs.h")
LIB = os.path.join(ROOT, "paper_2603_09632_amd", "libxgs.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xgs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def xgs():
    if not os.path.exists(LIB):
        pytest.fail("libxgs.so is not built (python paper_2603_09632_amd/build.py)")
    import paper_2603_09632_amd as x
    return x


def test_header_declares_the_hot_path(xgs):
    names = declared()
    for n in ("xgs_project", "xgs_tile_sort", "xgs_render_fwd", "xgs_render_bwd", "xgs_grid_sample",
              "xgs_vq_assign", "xgs_vq_ema_update"):
        assert n in names


def test_every_declared_symbol_is_exported(xgs):
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    from paper_2603_09632_amd import _lib
    assert set(declared()) == set(_lib.SIGNATURES)


def test_status_strings_and_version(xgs):
    lib = xgs.lib
    assert lib.xgs_version() == 1
    assert lib.xgs_status_string(0) == b"ok"
    assert lib.xgs_status_string(2) == b"buffer or workspace too small"


def test_grid_dims_host_only(xgs):
    assert xgs.grid_dims(xgs.camera(128, 96, 100, 100, 64, 48)) == (96, 128, 6, 8)
    assert xgs.grid_dims(xgs.camera(1200, 680, 600, 600, 600, 340)) == (680, 1200, 43, 75)
    assert xgs.grid_dims(xgs.camera(640, 480, 525, 525, 320, 240, stride=3, off_y=2)) == (160, 214, 10, 14)


def test_invalid_arguments_are_rejected_before_launch(xgs):
    lib = xgs.lib
    bad = xgs.camera(128, 96, 100, 100, 64, 48, stride=2, off_y=2)
    st = lib.xgs_grid_dims(ctypes.byref(bad), None, None, None, None)
    assert st == 1 and b"offsets" in lib.xgs_last_error()
    st = lib.xgs_grid_sample(None, 4, 3, 3, 10, 10, 1, 0, 0, 7, None, None, None)
    assert st == 1 and b"mode" in lib.xgs_last_error()
    st = lib.xgs_grid_sample_offsets(None, 4, 3, 3, 10, 10, 2, 7, None, None, None)
    assert st == 1 and b"mode" in lib.xgs_last_error()
    st = lib.xgs_grid_sample_offsets(None, 4, 3, 3, 1000, 1000, 65, 0, None, None, None)
    assert st == 4 and b"stride" in lib.xgs_last_error()
    st = lib.xgs_grid_sample_offsets(None, 4, 3, 3, 10, 10, 0, 0, None, None, None)
    assert st == 1
    st = lib.xgs_vq_assign(None, 10, 20, None, None, None, 4, 1, None, None, None, 0, None)
    assert st == 1
    st = lib.xgs_vq_ema_update(None, None, 5, 4, 4, None, None, None, None, None, None, 1.5, 1e-5, 1, None, 0, None)
    assert st == 1 and b"decay" in lib.xgs_last_error()
    with pytest.raises(xgs.XgsError):
        xgs.grid_dims(xgs.camera(0, 96, 100, 100, 64, 48))


def test_workspace_queries_grow_with_size(xgs):
    lib = xgs.lib
    a = lib.xgs_tile_sort_workspace(1000, 5000, 48)
    b = lib.xgs_tile_sort_workspace(1_000_000, 4_000_000, 3225)
    assert 0 < a < b
    assert lib.xgs_render_bwd_workspace(1_000_000) >= 32_000_000
    assert lib.xgs_vq_ema_workspace(816_000, 768, 4096) > 816_000 * 24
    assert lib.xgs_vq_assign_workspace(816_000, 768, 4096, 0) == 0
    assert lib.xgs_vq_assign_workspace(816_000, 768, 4096, 1) >= 816_000 * 800 * 2
