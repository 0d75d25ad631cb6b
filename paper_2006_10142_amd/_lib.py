"""ctypes declarations of libadiwave.so (the C ABI in include/adiwave.h).

The shared library is loaded from this package directory only; there is no
fallback: if it is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libadiwave.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "adiwave.h")

ADI_F32, ADI_F64 = 0, 1
ADI_OK, ADI_EINVAL, ADI_ENOMEM, ADI_EHIP, ADI_EUNSUPPORTED = 0, -1, -2, -3, -4
ADI_START_PAPER, ADI_START_GHOST = 0, 1
ADI_MAX_SOURCES = 1024

_vp = ctypes.c_void_p


class AdiSource(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("idx", _vp), ("amp", _vp)]


class AdiReceivers(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("idx", _vp), ("traces", _vp)]


class AdiWaveInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dtype", ctypes.c_int),
                ("x_threads_per_line", ctypes.c_int), ("x_rows_per_strip", ctypes.c_int),
                ("y_fused", ctypes.c_int), ("y_chunk_rows", ctypes.c_int),
                ("y_chunks", ctypes.c_int), ("kernels_per_step", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("fused_step", ctypes.c_int),
                ("fused_allowed", ctypes.c_int), ("r_max", ctypes.c_double),
                ("line_solver", ctypes.c_int), ("fused_tile_cols", ctypes.c_int),
                ("fused_tiles", ctypes.c_int), ("fused_lane_nodes", ctypes.c_int),
                ("fused_segment_rows", ctypes.c_int), ("fused_strips_wide", ctypes.c_int)]


class AdiTuning(ctypes.Structure):
    _fields_ = [("x_threads_per_line", ctypes.c_int), ("x_rows_per_strip", ctypes.c_int),
                ("y_fused", ctypes.c_int), ("y_chunk_rows", ctypes.c_int),
                ("fused_step", ctypes.c_int), ("line_solver", ctypes.c_int),
                ("fused_tile_cols", ctypes.c_int), ("fused_lane_nodes", ctypes.c_int),
                ("fused_segment_rows", ctypes.c_int)]


class AdiBatchPlan(ctypes.Structure):
    _fields_ = [("x_threads_per_line", ctypes.c_int), ("x_grid", ctypes.c_int),
                ("yscan_grid", ctypes.c_int), ("ysolve_grid", ctypes.c_int),
                ("graph", ctypes.c_int), ("count", ctypes.c_int), ("nodes", ctypes.c_longlong),
                ("workspace_bytes", ctypes.c_size_t), ("x_items", ctypes.c_int),
                ("yscan_items", ctypes.c_int), ("ysolve_items", ctypes.c_int),
                ("fused_step", ctypes.c_int), ("fused_allowed", ctypes.c_int),
                ("fused_items", ctypes.c_int), ("fused_lane_nodes", ctypes.c_int),
                ("fused_strips", ctypes.c_int)]


_SIGNATURES = {
    "adi_wave_create": [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                        ctypes.c_double, _vp, ctypes.c_double, ctypes.c_int, _vp],
    "adi_wave_set_kappa": [_vp, _vp, ctypes.c_double],
    "adi_wave_set_stream": [_vp, _vp],
    "adi_wave_start": [_vp, _vp, _vp, ctypes.POINTER(AdiSource), ctypes.c_int, _vp],
    "adi_wave_step": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(AdiSource),
                      ctypes.POINTER(AdiReceivers), ctypes.c_int],
    "adi_wave_step_tdc": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp,
                          ctypes.POINTER(AdiSource), ctypes.POINTER(AdiReceivers)],
    "adi_wave_step_split": [_vp, ctypes.c_int, _vp, _vp, ctypes.POINTER(AdiSource),
                            ctypes.POINTER(AdiSource), ctypes.POINTER(AdiReceivers)],
    "adi_wave_destroy": [_vp],
    "tridiag_solve_batched": [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                              ctypes.c_longlong, ctypes.c_longlong, _vp],
    "tridiag_solve_batched_noalloc": [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                                      ctypes.c_longlong, ctypes.c_longlong, _vp],
    "adi_wave_get_info": [_vp, ctypes.POINTER(AdiWaveInfo)],
    "adi_wave_set_tuning": [_vp, ctypes.POINTER(AdiTuning)],
    "adi_wave_profile": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(AdiSource),
                         ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int)],
    "adi_stream_copy": [_vp, _vp, ctypes.c_size_t, _vp],
    "adi_last_error": [],
    "adi_batch_create": [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp),
                         ctypes.POINTER(ctypes.c_double), ctypes.c_int, _vp],
    "adi_batch_bind": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "adi_batch_start": [_vp, ctypes.c_int],
    "adi_batch_step": [_vp, ctypes.c_int],
    "adi_batch_levels": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "adi_batch_graph": [_vp, ctypes.c_int],
    "adi_batch_get_plan": [_vp, ctypes.POINTER(AdiBatchPlan)],
    "adi_batch_set_plan": [_vp, ctypes.POINTER(AdiBatchPlan)],
    "adi_batch_autotune": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
    "adi_batch_destroy": [_vp],
    "adi_adjoint_forward": [_vp, _vp, _vp, ctypes.POINTER(AdiSource), ctypes.POINTER(AdiReceivers),
                            ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_ulonglong)],
    "adi_adjoint_backward": [_vp, ctypes.c_ulonglong, ctypes.POINTER(AdiSource),
                             ctypes.POINTER(AdiReceivers), _vp, _vp, _vp],
}

_lib = None


class AdiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"adiwave status {status}: {msg}")
        self.status = status


def header_functions() -> list:
    """Names of the functions declared in include/adiwave.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:adi_status|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def load():
    """Load libadiwave.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2006_10142_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, argtypes in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = ctypes.c_char_p if name == "adi_last_error" else ctypes.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != ADI_OK:
        raise AdiError(status, load().adi_last_error().decode(errors="replace"))
