"""ctypes view of libgm.so (the C ABI in include/gm.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

GM_OK = 0
GM_ERR_INVALID_ARG = 1
GM_ERR_OUT_OF_MEMORY = 2
GM_ERR_DEVICE = 3
GM_ERR_UNSUPPORTED = 4

GM_FORM_FASTGM = 0
GM_FORM_PLAIN = 1

GM_K_MAX = 4096

OPTIONS = {"pos_bits": 0, "t0_scale_ppm": 1, "map_load": 2, "republish": 3, "stats": 4,
           "seg_rest": 5, "small_waves": 6, "timing": 7, "wave_lim": 8}
STATS = ["vectors", "iterations", "arrivals", "kept", "elements", "heavy", "heavy_batches",
         "passes", "resolves", "cyc_prep", "cyc_walk", "cyc_seg", "cyc_extra", "cyc_out"]

_lib = None


class TuneResult(ctypes.Structure):
    _fields_ = [("small_waves", ctypes.c_int32), ("map_load", ctypes.c_int32),
                ("seg_rest", ctypes.c_int32), ("republish", ctypes.c_int32),
                ("ms", ctypes.c_double), ("from_cache", ctypes.c_int32),
                ("wave_lim", ctypes.c_int32)]


class GMError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


def path() -> str:
    return _build.LIB


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        raise ImportError(
            f"libgm.so not found at {_build.LIB}; build it with "
            "`python -m paper_2302_05176_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(_build.LIB)
    p, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_double)
    st = ctypes.c_int
    L.gm_sketch.argtypes = [p, p, p, i64, i32, u64, p, p, p]
    L.gm_sketch_plain.argtypes = [p, p, p, i64, i32, u64, p, p, p]
    L.gm_sketch_plain_noalloc.argtypes = [p, p, p, i64, i32, u64, p, p, p]
    L.gm_sketch_update.argtypes = [p, p, p, i64, i32, u64, p, p, p]
    L.gm_sketch_batched.argtypes = [p, p, p, i64, p, p, i32, u64, ctypes.c_int, p, p, p]
    L.gm_jaccard_est.argtypes = [p, p, i64, i32, p, p]
    L.gm_jaccard_est_pairs.argtypes = [p, i64, i32, p, p, i64, p, p]
    L.gm_wcard_est.argtypes = [p, i64, i32, p, p]
    L.gm_merge.argtypes = [p, p, i64, i32, p, p, p]
    L.gm_setops.argtypes = [p, p, p, p, i64, i32, p, p]
    L.gm_rate_probe.argtypes = [i32, i64, i32, u64, p, p]
    L.gm_lsh_build.argtypes = [p, i64, i32, i32, i32, ctypes.POINTER(p), p]
    L.gm_lsh_query.argtypes = [p, p, i64, i32, p, p, p]
    L.gm_lsh_info.argtypes = [p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.gm_lsh_free.argtypes = [p]
    L.gm_lsh_free.restype = None
    L.gm_get_data_errors.argtypes = [ctypes.POINTER(ctypes.c_int64), p]
    L.gm_reset_data_errors.argtypes = [p]
    L.gm_set_option.argtypes = [ctypes.c_int, i64]
    L.gm_status_string.argtypes = [ctypes.c_int]
    L.gm_status_string.restype = ctypes.c_char_p
    L.gm_reserve.argtypes = [i64, p]
    L.gm_workspace_bytes.argtypes = [i64, ctypes.POINTER(ctypes.c_int64)]
    L.gm_serve_run.argtypes = [p, p, i64, p, p, p, i64, p, p, p, p, p]
    L.gm_autotune.argtypes = [p, p, p, i64, p, p, i32, u64, p, p, i32, i32,
                              ctypes.POINTER(TuneResult), p]
    L.gm_get_stats.argtypes = [ctypes.POINTER(ctypes.c_int64), i32, p]
    L.gm_reset_stats.argtypes = [p]
    L.gm_get_timing.argtypes = [i32, p, p, p]
    L.gm_get_timing.restype = i32
    L.gm_reset_timing.argtypes = []
    L.gm_reset_timing.restype = None
    L.gm_release_stream.argtypes = [p]
    L.gm_release_stream.restype = None
    L.gm_release.argtypes = []
    L.gm_release.restype = None
    for name in ("gm_sketch", "gm_sketch_plain", "gm_sketch_plain_noalloc", "gm_sketch_batched", "gm_jaccard_est",
                 "gm_jaccard_est_pairs", "gm_wcard_est", "gm_merge", "gm_setops", "gm_get_data_errors",
                 "gm_reset_data_errors", "gm_set_option", "gm_get_stats", "gm_reset_stats", "gm_reserve", "gm_workspace_bytes", "gm_autotune",
                 "gm_serve_run", "gm_lsh_build", "gm_lsh_query", "gm_lsh_info"):
        getattr(L, name).restype = st
    _lib = L
    return L


def status_string(status: int) -> str:
    try:
        return load().gm_status_string(int(status)).decode()
    except ImportError:
        return "unknown"


def check(status: int, what: str) -> None:
    if status != GM_OK:
        raise GMError(status, what)
