"""C-ABI checks that need no GPU: the library loads, exports every function
include/*.h declares, validates its arguments, and sets up box geometry
(host FP64) exactly as the canonical definitions say."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2202_06427_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]

_dp = ctypes.POINTER(ctypes.c_double)


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        names |= set(re.findall(r"^\s*(?:clm_status|const char\*)\s+(clm_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def _box(dim, H, rc, lcell=1):
    H = np.ascontiguousarray(H, dtype=np.float64)
    h = ctypes.c_void_p()
    st = L.lib().clm_box_create(dim, H.ctypes.data_as(_dp), rc, lcell, ctypes.byref(h))
    return st, h


def _info(h):
    bi = L.BoxInfo()
    assert L.lib().clm_box_info_get(h, ctypes.byref(bi)) == 0
    return bi


@pytest.mark.parametrize("dim,H,rc,lcell,status", [
    (4, np.eye(4), 1.0, 1, 2),
    (1, np.eye(1), 1.0, 1, 2),
    (3, np.diag([10.0, 10.0, -10.0]), 1.0, 1, 2),       # left-handed / det < 0
    (3, np.zeros((3, 3)), 1.0, 1, 2),                  # degenerate
    (3, np.diag([10.0, np.nan, 10.0]), 1.0, 1, 2),     # non-finite
    (3, np.eye(3) * 10, 0.0, 1, 3),                    # cutoff 0
    (3, np.eye(3) * 10, -1.0, 1, 3),
    (3, np.eye(3) * 10, float("inf"), 1, 3),
    (3, np.eye(3) * 10, 1.0, 0, 3),                    # lcell 0
    (2, np.eye(2) * 10, 1.0, 1, 0),
])
def test_box_validation(dim, H, rc, lcell, status):
    st, h = _box(dim, H, rc, lcell)
    assert st == status, L.lib().clm_last_error()
    if st == 0:
        L.lib().clm_box_destroy(h)
    else:
        assert len(L.lib().clm_last_error()) > 0


BOXES = [
    np.diag([46.42] * 3),
    W.triclinic_h((215.4, 215.4, 215.4), (80.0, 95.0, 100.0)),
    W.triclinic_h((20.0, 22.0, 21.0), (70.0, 110.0, 75.0)),
    np.array([[10.0, 0.0, 0.0], [0.0, 10.0, 0.0], [0.0, 20.0, 10.0]]),  # Code 3 triclinic
    np.array([[24.0, -7.0], [0.0, 22.0]]),
    np.eye(2),
]


@pytest.mark.parametrize("k", range(len(BOXES)))
def test_inverse_matches_canonical_definition_bitwise(k):
    H = BOXES[k]
    dim = H.shape[0]
    st, h = _box(dim, H, 0.01 * H[0, 0], 1)
    assert st == 0
    bi = _info(h)
    Hinv = np.array(bi.Hinv[: dim * dim]).reshape(dim, dim)
    assert np.array_equal(Hinv, oracle.box_inverse(H))  # same written definition, bit for bit
    w, V = oracle.box_widths(H)
    assert np.allclose(bi.widths[:dim], w, rtol=1e-13)
    assert math.isclose(bi.volume, V, rel_tol=1e-13)
    L.lib().clm_box_destroy(h)


@pytest.mark.parametrize("k", range(len(BOXES)))
@pytest.mark.parametrize("lcell", [1, 2, 3])
def test_grid_covers_the_cutoff(k, lcell):
    H = BOXES[k]
    dim = H.shape[0]
    w, _ = oracle.box_widths(H)
    for rc in (w.min() / 3.5, w.min() / 7.3, w.min() / 20.0):
        st, h = _box(dim, H, rc, lcell)
        assert st == 0
        bi = _info(h)
        assert not bi.small_box
        lc = bi.lcell
        assert 1 <= lc <= lcell
        for d in range(dim):
            n = bi.grid[d]
            assert n >= 2 * lc + 1
            assert w[d] / n >= rc / lc  # cell width along every face normal >= rc / lcell
        assert bi.guard_band > 0 and bi.guard_band < 1e-4 * bi.rc2
        assert bi.rc2 == rc * rc
        L.lib().clm_box_destroy(h)


@pytest.mark.parametrize("k", range(len(BOXES)))
@pytest.mark.parametrize("lcell,lcell_x", [(1, 2), (2, 3), (2, 4), (3, 1)])
def test_grid_covers_the_cutoff_row_axis_refined(k, lcell, lcell_x):
    """A separate reach along the row axis: every axis d still has cells of
    width >= rc / l_d and at least 2 l_d + 1 of them."""
    H = np.ascontiguousarray(BOXES[k], dtype=np.float64)
    dim = H.shape[0]
    w, _ = oracle.box_widths(H)
    for rc in (w.min() / 3.5, w.min() / 7.3, w.min() / 20.0):
        h = ctypes.c_void_p()
        st = L.lib().clm_box_create_ex(dim, H.ctypes.data_as(_dp), rc, lcell, lcell_x, ctypes.byref(h))
        assert st == 0
        bi = _info(h)
        if bi.small_box:
            L.lib().clm_box_destroy(h)
            continue
        lds = [bi.lcell_x] + [bi.lcell] * (dim - 1)
        assert 1 <= bi.lcell <= lcell and 1 <= bi.lcell_x <= lcell_x
        for d in range(dim):
            n = bi.grid[d]
            assert n >= 2 * lds[d] + 1
            assert w[d] / n >= rc / lds[d]
        L.lib().clm_box_destroy(h)
    h = ctypes.c_void_p()
    assert L.lib().clm_box_create_ex(dim, H.ctypes.data_as(_dp), 1.0, 2, 9, ctypes.byref(h)) == 3


def test_small_box_flag_and_lcell_fallback():
    st, h = _box(3, np.eye(3) * 10.0, 4.0, 1)  # 2 cells per axis: brute force
    assert st == 0 and _info(h).small_box == 1
    L.lib().clm_box_destroy(h)
    # 2l+1 cells of side >= rc/l fit when rc <= L l / (2l+1): rc 4.1 needs l = 3
    st, h = _box(3, np.eye(3) * 10.0, 4.1, 1)
    assert st == 0 and _info(h).small_box == 1
    L.lib().clm_box_destroy(h)
    st, h = _box(3, np.eye(3) * 10.0, 4.1, 3)
    bi = _info(h)
    assert st == 0 and bi.small_box == 0 and bi.lcell == 3 and list(bi.grid) == [7, 7, 7]
    L.lib().clm_box_destroy(h)


def test_lengths_angles_constructor():
    la = np.array([215.4, 215.4, 215.4])
    an = np.array([80.0, 95.0, 100.0])
    h = ctypes.c_void_p()
    assert L.lib().clm_box_from_lengths_angles(la.ctypes.data_as(_dp), an.ctypes.data_as(_dp), 12.0, 2,
                                               ctypes.byref(h)) == 0
    bi = _info(h)
    H = np.array(bi.H[:9]).reshape(3, 3)
    assert np.allclose(H, oracle.box_from_lengths_angles(la, an), rtol=1e-14, atol=1e-12)
    assert list(bi.grid) == [35, 34, 35] and bi.lcell == 2
    L.lib().clm_box_destroy(h)
    bad = np.array([80.0, 80.0, 170.0])
    assert L.lib().clm_box_from_lengths_angles(la.ctypes.data_as(_dp), bad.ctypes.data_as(_dp), 12.0, 2,
                                               ctypes.byref(h)) == 2


def test_workspace_bytes():
    st, h = _box(3, BOXES[1], 12.0, 2)
    sizes = []
    for n in (0, 1, 1000, 1_000_000):
        b = ctypes.c_size_t(0)
        assert L.lib().clm_celllist_workspace_bytes(h, n, 0, L.CLM_FP32_GUARD, ctypes.byref(b)) == 0
        sizes.append(b.value)
    assert sizes == sorted(sizes) and sizes[-1] > 1_000_000 * 64
    b = ctypes.c_size_t(0)
    assert L.lib().clm_celllist_workspace_bytes(h, -1, 0, 1, ctypes.byref(b)) == 1
    assert L.lib().clm_celllist_workspace_bytes(h, 10, 0, 7, ctypes.byref(b)) == 1
    assert L.lib().clm_celllist_workspace_bytes(None, 10, 0, 1, ctypes.byref(b)) == 1
    L.lib().clm_box_destroy(h)


def test_null_arguments_are_rejected_not_crashed():
    lib = L.lib()
    assert lib.clm_map(None, 0, None, None) == 1
    assert lib.clm_celllist_build(None, None, None) == 1
    assert lib.clm_celllist_info_get(None, None) == 1
    assert lib.clm_synchronize(None) == 1
    assert lib.clm_box_info_get(None, None) == 1
    assert lib.clm_status_string(4) == b"CLM_E_CAPACITY"


def test_md_workspace_sizes_and_validation():
    lib = L.lib()
    b = ctypes.c_size_t(0)
    assert lib.clm_md_workspace_bytes(1000, ctypes.byref(b)) == 0
    # block partials of ceil(1000/256) blocks (8 doubles each) and one double
    assert b.value >= 4 * 8 * 8 + 8
    assert lib.clm_md_workspace_bytes(-1, ctypes.byref(b)) == 1
    assert lib.clm_md_workspace_bytes(10, None) == 1
    h = ctypes.c_void_p()
    assert lib.clm_md_create(None, 3, 10, 1.0, 0.001, None, 0, ctypes.byref(h)) == 1
    assert lib.clm_vlist_workspace_bytes(None, 100, ctypes.byref(b)) == 1
    assert lib.clm_vlist_update(None, None) == 1
    assert lib.clm_vlist_lj(None, 1.0, 1.0, None, None, None, None, None, None, None) == 1


def test_calibration_arguments():
    """The device-rate microbenchmarks (include/clmap_calib.h): scratch sizes
    and argument validation before any device call."""
    lib = L.lib()
    nb = ctypes.c_size_t(0)
    assert lib.clm_calibrate_scratch_bytes(0, ctypes.byref(nb)) == 0 and nb.value == 4096 * 256 * 4
    assert lib.clm_calibrate_scratch_bytes(1, ctypes.byref(nb)) == 0 and nb.value == 4096 * 256 * 8
    assert lib.clm_calibrate_scratch_bytes(2, ctypes.byref(nb)) == 0 and nb.value == 0
    assert lib.clm_calibrate_scratch_bytes(3, ctypes.byref(nb)) == L.STATUS_CODES["CLM_E_INVALID_ARG"]
    assert lib.clm_calibrate_scratch_bytes(0, None) == L.STATUS_CODES["CLM_E_INVALID_ARG"]
    ms, work = ctypes.c_double(0.0), ctypes.c_double(0.0)
    assert lib.clm_calibrate(None, 0, None, None, 0, 1, ctypes.byref(ms), ctypes.byref(work)) \
        == L.STATUS_CODES["CLM_E_INVALID_ARG"]


def test_pairs_sort_workspace_and_validation():
    """Neighbour-list sort: workspace sizes (a key buffer, a distance buffer,
    the digit table) and argument checks before any device call."""
    lib = L.lib()
    b = ctypes.c_size_t(0)
    assert lib.clm_pairs_sort_workspace_bytes(10**6, 1, ctypes.byref(b)) == 0
    with_d = b.value
    assert with_d >= 10**6 * 16 + 256 * (10**6 // 2048) * 4
    assert lib.clm_pairs_sort_workspace_bytes(10**6, 0, ctypes.byref(b)) == 0
    assert with_d - b.value >= 10**6 * 8
    assert lib.clm_pairs_sort_workspace_bytes(0, 0, ctypes.byref(b)) == 0
    bad = L.STATUS_CODES["CLM_E_INVALID_ARG"]
    assert lib.clm_pairs_sort_workspace_bytes(-1, 0, ctypes.byref(b)) == bad
    assert lib.clm_pairs_sort_workspace_bytes(1 << 31, 0, ctypes.byref(b)) == bad
    assert lib.clm_pairs_sort_workspace_bytes(10, 0, None) == bad
    assert lib.clm_pairs_sort(None, 10, 10, None, None, None, 10, None, 0) == bad


def test_md_kinetic_and_rescale_validation():
    lib = L.lib()
    bad = L.STATUS_CODES["CLM_E_INVALID_ARG"]
    assert lib.clm_md_kinetic(None, None, None) == bad
    assert lib.clm_md_rescale(None, None, 1.0) == bad
