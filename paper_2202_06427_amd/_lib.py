"""ctypes mirror of include/clmap.h (argument marshalling only).

Loads libclmap.so from this package directory and raises if it is missing:
there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclmap.so")

# clm_status
CLM_OK = 0
STATUS_NAMES = {0: "CLM_OK", 1: "CLM_E_INVALID_ARG", 2: "CLM_E_BAD_BOX", 3: "CLM_E_BAD_CUTOFF",
                4: "CLM_E_CAPACITY", 5: "CLM_E_WORKSPACE", 6: "CLM_E_DEVICE", 7: "CLM_E_UNSUPPORTED"}
STATUS_CODES = {v: k for k, v in STATUS_NAMES.items()}

# clm_precision
CLM_FP64 = 0
CLM_FP32_GUARD = 1

# clm_map_kind
MAP_KINDS = {
    "count": 0, "sum_d": 1, "sum_inv_d": 2, "lj_e": 3, "lj_ef": 4, "lj_adjoint": 5,
    "hist_dist": 6, "hist_relspeed": 7, "neighbor_list": 8, "sum_w_inv_d": 9, "hist_dist_vel": 10,
}

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class BoxInfo(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("lcell_requested", ctypes.c_int), ("lcell", ctypes.c_int),
        ("small_box", ctypes.c_int), ("grid", ctypes.c_int * 3), ("ncells", ctypes.c_int64),
        ("H", ctypes.c_double * 9), ("Hinv", ctypes.c_double * 9), ("widths", ctypes.c_double * 3),
        ("volume", ctypes.c_double), ("cutoff", ctypes.c_double), ("rc2", ctypes.c_double),
        ("guard_band", ctypes.c_double), ("lcell_x", ctypes.c_int), ("pad", ctypes.c_int),
    ]


class CellListInfo(ctypes.Structure):
    _fields_ = [
        ("n_x", ctypes.c_int64), ("n_y", ctypes.c_int64), ("ncells", ctypes.c_int64),
        ("ntiles", ctypes.c_int64), ("nonempty_cells", ctypes.c_int64),
        ("max_occupancy", ctypes.c_int64), ("candidate_pairs", ctypes.c_int64),
        ("guard_retests", ctypes.c_int64), ("near_evaluations", ctypes.c_int64),
        ("half_pairs_tested", ctypes.c_int64), ("half_pairs_kept", ctypes.c_int64),
    ]


class MapParams(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double), ("epsilon", ctypes.c_double), ("near_factor", ctypes.c_double),
        ("want_virial", ctypes.c_int), ("upstream_dev", _vp), ("nbins", ctypes.c_int),
        ("hist_hi", ctypes.c_double), ("vel_x_dev", _vp), ("vel_y_dev", _vp),
        ("want_sums", ctypes.c_int), ("capacity", ctypes.c_int64), ("with_distances", ctypes.c_int),
        ("cutoff", ctypes.c_double), ("weights_x_dev", _vp), ("weights_y_dev", _vp),
        ("scratch_dev", _vp), ("scratch_bytes", ctypes.c_size_t),
        ("no_prune", ctypes.c_int), ("sorted", ctypes.c_int), ("check_capacity", ctypes.c_int),
        ("half_shell", ctypes.c_int),
    ]


class MapOut(ctypes.Structure):
    _fields_ = [
        ("energy_dev", _vp), ("forces_dev", _vp), ("virial_dev", _vp), ("grad_box_dev", _vp),
        ("hist_dev", _vp), ("hist_sums_dev", _vp), ("pairs_dev", _vp), ("dist_dev", _vp),
        ("count_dev", _vp),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("builds", ctypes.c_int64), ("sweeps", ctypes.c_int64), ("build_ms", ctypes.c_double),
        ("sweep_ms", ctypes.c_double), ("last_sweep_ms", ctypes.c_double),
    ]


class VlistInfo(ctypes.Structure):
    _fields_ = [
        ("updates", ctypes.c_int64), ("rebuilds", ctypes.c_int64), ("entries", ctypes.c_int64),
        ("max_row", ctypes.c_int64), ("row_capacity", ctypes.c_int64), ("skin", ctypes.c_double),
        ("overflow", ctypes.c_int), ("pad", ctypes.c_int),
    ]


EXPORTS = [
    "clm_context_create", "clm_context_set_stream", "clm_context_destroy", "clm_box_create",
    "clm_box_create_ex",
    "clm_box_from_lengths_angles", "clm_box_info_get", "clm_box_destroy",
    "clm_celllist_workspace_bytes", "clm_celllist_create", "clm_celllist_build", "clm_map",
    "clm_celllist_info_get", "clm_celllist_destroy", "clm_synchronize", "clm_last_error",
    "clm_status_string", "clm_context_set_timing", "clm_stats_get", "clm_map_batch_workspace_bytes",
    "clm_map_batch", "clm_box_nonperiodic", "clm_extrema_workspace_bytes", "clm_extrema",
    "clm_map_static_max_bytes", "clm_map_static", "clm_map_scratch_bytes",
    "clm_pairs_sort_workspace_bytes", "clm_pairs_sort",
    # include/clmap_md.h
    "clm_md_workspace_bytes", "clm_md_create", "clm_md_kick_drift", "clm_md_kick", "clm_md_kinetic",
    "clm_md_rescale", "clm_md_destroy",
    "clm_vlist_workspace_bytes", "clm_vlist_create", "clm_vlist_update", "clm_vlist_lj",
    "clm_vlist_info_get", "clm_vlist_destroy",
    # include/clmap_kclosest.h
    "clm_kclosest_workspace_bytes", "clm_kclosest",
    # include/clmap_calib.h
    "clm_calibrate_scratch_bytes", "clm_calibrate",
]

CALIB_KINDS = {"fma_f32": 0, "fma_f64": 1, "copy": 2}

_lib = None


class ClmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libclmap.so not built: {LIB_PATH} (run paper_2202_06427_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_i64, c_d = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pvp = ctypes.POINTER(_vp)
    L.clm_context_create.argtypes = [c_int, _vp, pvp]
    L.clm_context_set_stream.argtypes = [_vp, _vp]
    L.clm_context_destroy.argtypes = [_vp]
    L.clm_box_create.argtypes = [c_int, _dp, c_d, c_int, pvp]
    L.clm_box_create_ex.argtypes = [c_int, _dp, c_d, c_int, c_int, pvp]
    L.clm_box_from_lengths_angles.argtypes = [_dp, _dp, c_d, c_int, pvp]
    L.clm_box_info_get.argtypes = [_vp, ctypes.POINTER(BoxInfo)]
    L.clm_box_destroy.argtypes = [_vp]
    L.clm_celllist_workspace_bytes.argtypes = [_vp, c_i64, c_i64, c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.clm_celllist_create.argtypes = [_vp, _vp, c_i64, c_i64, c_int, _vp, ctypes.c_size_t, pvp]
    L.clm_celllist_build.argtypes = [_vp, _vp, _vp]
    L.clm_map.argtypes = [_vp, c_int, ctypes.POINTER(MapParams), ctypes.POINTER(MapOut)]
    L.clm_celllist_info_get.argtypes = [_vp, ctypes.POINTER(CellListInfo)]
    L.clm_celllist_destroy.argtypes = [_vp]
    L.clm_synchronize.argtypes = [_vp]
    L.clm_context_set_timing.argtypes = [_vp, c_int]
    L.clm_stats_get.argtypes = [_vp, ctypes.POINTER(Stats), c_int]
    L.clm_map_batch_workspace_bytes.argtypes = [c_int, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)]
    L.clm_map_batch.argtypes = [c_int, ctypes.POINTER(_vp), c_int, ctypes.POINTER(MapParams),
                                ctypes.POINTER(MapOut), _vp, ctypes.c_size_t]
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.clm_map_static_max_bytes.argtypes = [szp]
    L.clm_map_scratch_bytes.argtypes = [_vp, c_int, szp]
    L.clm_pairs_sort_workspace_bytes.argtypes = [c_i64, c_int, szp]
    L.clm_pairs_sort.argtypes = [_vp, c_i64, c_i64, _vp, _vp, _vp, c_i64, _vp, ctypes.c_size_t]
    L.clm_map_static.argtypes = [_vp, _vp, _vp, c_i64, _vp, c_i64, c_int, c_int,
                                 ctypes.POINTER(MapParams), ctypes.POINTER(MapOut)]
    L.clm_md_workspace_bytes.argtypes = [c_i64, szp]
    L.clm_md_create.argtypes = [_vp, c_int, c_i64, c_d, c_d, _vp, ctypes.c_size_t, pvp]
    L.clm_md_kick_drift.argtypes = [_vp, _vp, _vp, _vp, c_d]
    L.clm_md_kick.argtypes = [_vp, _vp, _vp, _vp]
    L.clm_md_kinetic.argtypes = [_vp, _vp, _vp]
    L.clm_md_rescale.argtypes = [_vp, _vp, c_d]
    L.clm_md_destroy.argtypes = [_vp]
    L.clm_vlist_workspace_bytes.argtypes = [_vp, c_i64, szp]
    L.clm_vlist_create.argtypes = [_vp, c_d, c_i64, _vp, ctypes.c_size_t, pvp]
    L.clm_vlist_update.argtypes = [_vp, _vp]
    L.clm_vlist_lj.argtypes = [_vp, c_d, c_d, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.clm_vlist_info_get.argtypes = [_vp, ctypes.POINTER(VlistInfo)]
    L.clm_vlist_destroy.argtypes = [_vp]
    L.clm_box_nonperiodic.argtypes = [c_int, _dp, _dp, c_d, c_int, pvp]
    L.clm_extrema_workspace_bytes.argtypes = [c_i64, szp]
    L.clm_extrema.argtypes = [_vp, c_int, _vp, c_i64, _vp, ctypes.c_size_t, _dp, _dp]
    L.clm_kclosest_workspace_bytes.argtypes = [_vp, c_i64, c_i64, szp]
    L.clm_kclosest.argtypes = [_vp, c_i64, c_i64, _vp, ctypes.c_size_t, _vp, _vp, _vp,
                               ctypes.POINTER(c_i64)]
    L.clm_calibrate_scratch_bytes.argtypes = [c_int, szp]
    L.clm_calibrate.argtypes = [_vp, c_int, _vp, _vp, ctypes.c_size_t, c_int, _dp, _dp]
    L.clm_last_error.restype = ctypes.c_char_p
    L.clm_status_string.restype = ctypes.c_char_p
    L.clm_status_string.argtypes = [c_int]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype if name in ("clm_last_error", "clm_status_string") else c_int
    _lib = L
    return L


def check(status):
    if status != CLM_OK:
        raise ClmError(status, lib().clm_last_error().decode(errors="replace"))
