"""ctypes declarations of libp3t.so (the C ABI in include/p3t.h).

Loading fails loudly if the library has not been built: there is no fallback
path of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp3t.so")
HEADER = os.path.join(HERE, "..", "include", "p3t.h")

P3T_OK, P3T_ERR_ARG, P3T_ERR_CAPACITY, P3T_ERR_HIP, P3T_ERR_STATE, P3T_ERR_NUMERIC, P3T_ERR_CLUSTER = range(7)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_CAPACITY", 3: "ERR_HIP", 4: "ERR_STATE", 5: "ERR_NUMERIC",
                6: "ERR_CLUSTER"}

FLAG_COINCIDENT = 0x01
FLAG_NAN = 0x02
FLAG_LIST_OVERFLOW = 0x04
FLAG_STACK_OVERFLOW = 0x08
FLAG_PAIR_OVERFLOW = 0x10
FLAG_KMAX = 0x20
FLAG_NSTEPS = 0x40
FLAG_BIG_CLUSTER = 0x80
FLAG_UNBOUND = 0x100
FLAG_GROUP_BOUND = 0x200
FLAG_COLL_UNCHECKED = 0x400


class CParams(C.Structure):
    _fields_ = [
        ("G", C.c_double), ("m_star", C.c_double), ("gamma", C.c_double),
        ("r_cut0", C.c_double), ("r_cut1", C.c_double),
        ("r_search0", C.c_double), ("r_search1", C.c_double), ("r_search2", C.c_double), ("r_search3", C.c_double),
        ("dt_soft", C.c_double), ("theta", C.c_double), ("eta", C.c_double), ("eta0", C.c_double),
        ("multipole", C.c_int32), ("precision", C.c_int32), ("cutoff_mode", C.c_int32), ("hill_length", C.c_int32),
        ("n_group_max", C.c_int32), ("n_leaf_max", C.c_int32), ("vran_bins", C.c_int32),
        ("vran_min_count", C.c_int32), ("k_max", C.c_int32), ("cluster_cap", C.c_int32),
        ("isolated", C.c_int32),
    ]


class CStats(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_nodes", C.c_int64), ("n_groups", C.c_int64), ("n_near", C.c_int64),
        ("n_far", C.c_int64), ("n_cell", C.c_int64), ("n_pairs", C.c_int64), ("list_entries", C.c_int64),
        ("ms_cutoffs", C.c_double), ("ms_tree", C.c_double), ("ms_walk", C.c_double), ("ms_force", C.c_double),
        ("ms_neighbour", C.c_double), ("ms_hermite", C.c_double),
        ("ms_near", C.c_double), ("ms_far", C.c_double), ("ms_cell", C.c_double), ("ms_cand", C.c_double),
        ("timing", C.c_int32), ("n_slow", C.c_int32), ("ms_direct", C.c_double),
        ("n_heval", C.c_int64), ("n_hpair", C.c_int64), ("ms_sort", C.c_double), ("ms_clusters", C.c_double),
    ]


class CKernelConfig(C.Structure):
    _fields_ = [
        ("force_split", C.c_int32), ("force_unroll", C.c_int32), ("force_persistent", C.c_int32),
        ("waves_per_cu", C.c_int32), ("walk_waves_per_cu", C.c_int32), ("direct_pair_cap", C.c_int32),
        ("top_slots", C.c_int32), ("reserved", C.c_int32 * 1),
    ]


# name -> (restype, argtypes)
_vp, _i64, _i32, _d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
SIGNATURES = {
    "p3t_default_params": (None, [C.POINTER(CParams)]),
    "p3t_create": (C.c_int, [C.POINTER(CParams), _vp, C.POINTER(_vp)]),
    "p3t_destroy": (C.c_int, [_vp]),
    "p3t_set_stream": (C.c_int, [_vp, _vp]),
    "p3t_set_params": (C.c_int, [_vp, C.POINTER(CParams)]),
    "p3t_get_params": (C.c_int, [_vp, C.POINTER(CParams)]),
    "p3t_reserve": (C.c_int, [_vp, _i64, _i64]),
    "p3t_compute_cutoffs": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "p3t_build_tree": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "p3t_compute_soft_force": (C.c_int, [_vp, _vp]),
    "p3t_neighbour_list": (C.c_int, [_vp, _vp, _vp, _i64, C.POINTER(_i64), _vp]),
    "p3t_clusters": (C.c_int, [_vp, _i64, _vp, _vp, _vp, C.POINTER(_i64)]),
    "p3t_hermite_cluster_step": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "p3t_kick": (C.c_int, [_vp, _i64, _d, _vp, _vp]),
    "p3t_kepler_drift": (C.c_int, [_vp, _i64, _d, _vp, _vp, _vp, _i64, _vp, C.POINTER(_i64)]),
    "p3t_evaluate": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i32]),
    "p3t_hard_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_i64)]),
    "p3t_hard_step_collide": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _vp, C.POINTER(_d),
                                        C.POINTER(_i64), C.POINTER(_i64)]),
    "p3t_merge_bodies": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_i64)]),
    "p3t_hermite_collide": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp,
                                      _vp, C.POINTER(_i64)]),
    "p3t_hard_evaluate": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32,
                                    C.POINTER(_i64), C.POINTER(_i64)]),
    "p3t_soft_force_frozen": (C.c_int, [_vp, _vp, _vp, _vp]),
    "p3t_total_energy": (C.c_int, [_vp, _i64, _vp, _vp, _vp, C.POINTER(_d)]),
    "p3t_soft_kick_adjoint": (C.c_int, [_vp, _d, _vp, _vp, _vp]),
    "p3t_set_timing": (C.c_int, [_vp, _i32]),
    "p3t_set_kernel_config": (C.c_int, [_vp, C.POINTER(CKernelConfig)]),
    "p3t_get_kernel_config": (C.c_int, [_vp, C.POINTER(CKernelConfig)]),
    "p3t_get_stats": (C.c_int, [_vp, C.POINTER(CStats)]),
    "p3t_get_status": (C.c_int, [_vp, C.POINTER(C.c_uint32)]),
    "p3t_last_error": (C.c_char_p, [_vp]),
    "p3t_compute_cutoffs_noalloc": (C.c_int, [C.POINTER(CParams), _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
}

_lib = None


def load(path: str | None = None):
    """Load libp3t.so (built by paper_2007_15432_amd.build).  Raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libp3t.so not found at {p}: build it first (python -m paper_2007_15432_amd.build)")
    L = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = L
    return L
