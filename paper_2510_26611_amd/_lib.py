"""ctypes declarations of librsdock's C ABI (include/rsdock.h).  Loads the in-tree library.

The library must have been built (``python -m paper_2510_26611_amd.build_lib`` or
``__graft_entry__.build()``); there is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsdock.so")

RSD_OK = 0
RSD_E_INVALID = -1
RSD_E_OOM = -2
RSD_E_HIP = -3
RSD_E_NUMERIC = -4
RSD_E_UNSUPPORTED = -5
RSD_E_IO = -6
RSD_DEVICE_PTRS = 1
FLAG_ACCEPT = 1
FLAG_IN_DOMAIN = 2
FLAG_INVALID = 4

EXPORTED = [
    "rsd_version", "rsd_last_error", "rsd_context_create", "rsd_context_set_stream",
    "rsd_context_memory", "rsd_context_free", "rsd_build_rs_tensor", "rsd_tensor_import",
    "rsd_score_poses", "rsd_tensor_query", "rsd_tensor_export", "rsd_tensor_save",
    "rsd_tensor_load", "rsd_tensor_free", "rsd_context_set_timing", "rsd_kernel_time",
    "rsd_context_set_option", "rsd_batch_create", "rsd_batch_run", "rsd_batch_free", "rsd_autotune",
    "rsd_tensor_restrict", "rsd_tensor_grid", "rsd_tensor_combine",
    "rsd_tensor_centre", "rsd_contact_poses", "rsd_orbit_minima",
    "rsd_self_energy", "rsd_pose_order", "rsd_score_poses_noalloc",
    "rsd_tensor_layout", "rsd_probe_gather", "rsd_autotune_cells",
]


class SincParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("K_long", C.c_int32), ("h_M", C.c_double), ("L_s", C.c_double),
                ("r_cut", C.c_double), ("eps", C.c_double)]


class Request(C.Structure):
    _fields_ = [("tensor", C.c_void_p), ("lig_charges", C.c_void_p), ("lig_positions", C.c_void_p),
                ("L", C.c_int64), ("quats", C.c_void_p), ("trans", C.c_void_p), ("P", C.c_int64),
                ("vdw_min", C.c_double), ("energies", C.c_void_p), ("energies_long", C.c_void_p),
                ("flags", C.c_void_p), ("counts", C.c_void_p)]


class TuneReport(C.Structure):
    _fields_ = [("score_mode", C.c_int32), ("poses_per_wave", C.c_int32), ("short_waves", C.c_int32),
                ("candidates", C.c_int32), ("best_ms", C.c_double), ("default_ms", C.c_double)]


_P = C.c_void_p
_D = C.c_double
_I32 = C.c_int32
_I64 = C.c_int64
_U32 = C.c_uint32
_SZ = C.c_size_t


def _declare(lib: C.CDLL) -> C.CDLL:
    st = C.c_int
    sig = {
        "rsd_version": (st, [C.POINTER(_I32), C.POINTER(_I32)]),
        "rsd_last_error": (C.c_char_p, []),
        "rsd_context_create": (st, [_I32, _P, _SZ, C.POINTER(_P)]),
        "rsd_context_set_stream": (st, [_P, _P]),
        "rsd_context_memory": (st, [_P, C.POINTER(_SZ), C.POINTER(_SZ)]),
        "rsd_context_free": (None, [_P]),
        "rsd_build_rs_tensor": (st, [_P, _P, _P, _I64, _I32, _D, C.POINTER(SincParams), _U32, C.POINTER(_P)]),
        "rsd_pose_order": (st, [_P, _P, _P, _P, _I64, _P, _P, _P, C.POINTER(_I32)]),
        "rsd_tensor_import": (st, [_P, _P, _P, _P, _I64, _I32, _D, C.POINTER(SincParams), _P, _P, _I64, _U32,
                                   C.POINTER(_P)]),
        "rsd_score_poses": (st, [_P, _P, _P, _P, _I64, _P, _P, _I64, _D, _U32, _P, _P, _P, _P, _P]),
        "rsd_score_poses_noalloc": (st, [_P, _P, _P, _P, _I64, _P, _P, _I64, _D, _U32, _P, _P, _P, _P, _P]),
        "rsd_tensor_layout": (st, [_P, _P, _P]),
        "rsd_probe_gather": (st, [_P, _I32, _I32, _P, _P]),
        "rsd_autotune_cells": (st, [_P, _P, _P, _P, _I64, _P, _P, _I64, _D, _I32, _P, _P]),
        "rsd_tensor_query": (st, [_P, C.POINTER(_I32), C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_SZ)]),
        "rsd_tensor_export": (st, [_P, _P, _P, _P]),
        "rsd_tensor_save": (st, [_P, C.c_char_p]),
        "rsd_tensor_load": (st, [_P, C.c_char_p, C.POINTER(_P)]),
        "rsd_tensor_free": (None, [_P]),
        "rsd_context_set_timing": (st, [_P, _I32]),
        "rsd_context_set_option": (st, [_P, C.c_char_p, _I64]),
        "rsd_kernel_time": (st, [_P, C.c_char_p, C.POINTER(_I64), C.POINTER(_D)]),
        "rsd_batch_create": (st, [_P, C.POINTER(Request), _I32, C.POINTER(_P)]),
        "rsd_batch_run": (st, [_P]),
        "rsd_batch_free": (None, [_P]),
        "rsd_autotune": (st, [_P, _P, _P, _P, _I64, _P, _P, _I64, _D, _I32, C.POINTER(TuneReport)]),
        "rsd_tensor_restrict": (st, [_P, _P, C.POINTER(_D), C.POINTER(_D), _D, C.POINTER(_P)]),
        "rsd_tensor_combine": (st, [_P, _P, C.c_int32, _D, C.POINTER(_P)]),
        "rsd_tensor_centre": (st, [_P, C.POINTER(_D)]),
        "rsd_self_energy": (st, [_P, _P, C.POINTER(_D), C.POINTER(_D)]),
        "rsd_contact_poses": (st, [_P, _P, _P, C.c_int64, _P, C.c_int64, _P, C.c_int64, C.POINTER(_D), _D, _D, _P,
                                   _P, _P]),
        "rsd_orbit_minima": (st, [_P, _P, _P, C.c_int64, C.c_int64, _P, _P, _P, _P, _P]),
        "rsd_tensor_grid": (st, [_P, C.POINTER(_D), C.POINTER(_I32), C.POINTER(_D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librsdock.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib
