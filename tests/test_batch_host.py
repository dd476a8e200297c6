"""Host-side validation of batch slot tables (xgs_batch_check): no GPU, no
launch; the pointers are placeholders that are never dereferenced."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def xgs():
    import paper_2603_09632_amd as x
    return x


def table(xgs, entries):
    from paper_2603_09632_amd._lib import XgsBatchSlot
    arr = (XgsBatchSlot * len(entries))()
    for k, (n, w, h, gb, rb, c_sem) in enumerate(entries):
        e = arr[k]
        e.g.n, e.g.c_sem = n, c_sem
        for f in ("means", "log_scales", "quats", "opacity", "colors", "features"):
            setattr(e.g, f, 4096)
        e.cam = xgs.camera(w, h, 500.0, 500.0, w / 2, h / 2)
        e.out = e.final_T = e.n_last = 4096
        e.gauss_base, e.row_base = gb, rb
    return arr


def check(xgs, entries, cap=10_000, tx=75, rows=100, c_sem=16):
    t = table(xgs, entries)
    return xgs.lib.xgs_batch_check(t, len(entries), cap, tx, rows, c_sem), xgs.lib.xgs_last_error()


def test_valid_table(xgs):
    assert check(xgs, [(1000, 640, 480, 0, 0, 16), (2000, 1200, 680, 1000, 30, 16), (0, 320, 240, 3000, 73, 16)])[0] == 0


@pytest.mark.parametrize("entries,word", [
    ([(1000, 640, 480, 0, 0, 16), (10, 640, 480, 999, 30, 16)], b"overlap"),       # Gaussian rows overlap
    ([(1000, 640, 480, 0, 0, 16), (10, 640, 480, 1000, 29, 16)], b"band"),         # tile bands overlap
    ([(20_000, 640, 480, 0, 0, 16)], b"cap_gaussians"),                              # beyond capacity
    ([(10, 1300, 480, 0, 0, 16)], b"band"),                                          # wider than the grid
    ([(10, 640, 480, 0, 90, 16)], b"band"),                                          # rows beyond the grid
    ([(10, 640, 480, 0, 0, 8)], b"c_sem"),                                           # channel count differs
])
def test_invalid_tables_are_rejected(xgs, entries, word):
    st, msg = check(xgs, entries)
    assert st == 1 and word in msg, msg


def test_layout_packs_requests(xgs):
    cams = [xgs.camera(640, 480, 525, 525, 320, 240), xgs.camera(1200, 680, 600, 600, 600, 340)]
    lay = xgs.batch_layout([100, 200], cams, 75, 100, 1000)
    assert lay.gauss_base == [0, 100] and lay.row_base == [0, 30]
    with pytest.raises(xgs.XgsError):
        xgs.batch_layout([900, 200], cams, 75, 100, 1000)
