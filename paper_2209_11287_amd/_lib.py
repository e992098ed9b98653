"""ctypes declarations of the C ABI in include/selfjoin.h (argument marshalling
only; every step of the self-join runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libselfjoin.so")

SJ_OK = 0
SJ_ERR_INVALID = 1
SJ_ERR_OOM = 2
SJ_ERR_HIP = 3
SJ_ERR_CAPACITY = 4
SJ_ERR_UNSUPPORTED = 5

PATHS = {"fp64_valu": 0, "fp64_mfma": 1, "fp32_mfma": 2, "bf16_mfma": 3, "bf16x3_mfma": 4, "fp8_mfma": 5}
PATH_NAMES = {v: k for k, v in PATHS.items()}

# Every symbol include/selfjoin.h declares.
EXPORTS = [
    "selfjoin_build_grid",
    "selfjoin_count",
    "selfjoin_core_points",
    "selfjoin_knn",
    "selfjoin_pairs",
    "selfjoin_measure_error",
    "selfjoin_grid_info",
    "selfjoin_free_grid",
    "selfjoin_status_string",
    "selfjoin_last_error",
    "selfjoin_version",
    "selfjoin_batch_build",
    "selfjoin_batch_count",
    "selfjoin_batch_pairs",
    "selfjoin_batch_info",
    "selfjoin_batch_free",
    "selfjoin_count_noalloc",
    "selfjoin_probe_peaks",
]


# sj_opts.alloc / sj_opts.free
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class sj_opts(ctypes.Structure):
    _fields_ = [("index_dims", ctypes.c_int32), ("tune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("short_circuit", ctypes.c_int32), ("dim_order", ctypes.c_int32),
                ("symmetric", ctypes.c_int32), ("reserved32", ctypes.c_int32),
                ("reserved", ctypes.c_int64 * 2)]


class sj_stats(ctypes.Structure):
    _fields_ = [
        ("cand_ref", ctypes.c_int64),
        ("cand_eval", ctypes.c_int64),
        ("pairs", ctypes.c_int64),
        ("rechecked", ctypes.c_int64),
        ("rechecked_in", ctypes.c_int64),
        ("band_rel", ctypes.c_double),
        ("ms", ctypes.c_double),
        ("ms_build", ctypes.c_double),
        ("ms_refine", ctypes.c_double),
        ("ms_emit", ctypes.c_double),
        ("tiles_pruned", ctypes.c_int64),
        ("path_run", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["path_run"] = PATH_NAMES.get(d["path_run"], d["path_run"])
        return d


class sj_grid_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("cells", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("eps", ctypes.c_double),
        ("eps2", ctypes.c_double),
        ("cell_side", ctypes.c_double),
        ("cand_ref", ctypes.c_int64),
        ("cand_items", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class sj_peaks(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "fp64_mfma_tflops", "fp32_mfma_tflops", "bf16_mfma_tflops", "fp8_mfma_tflops", "fp64_valu_tflops",
        "hbm_read_gbs", "hbm_copy_gbs")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)

_lib = None


class LibraryMissing(ImportError):
    pass


def load():
    """Loads libselfjoin.so; raises LibraryMissing (no fallback) if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is not built; run `python -m paper_2209_11287_amd.build` "
            "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    lib.selfjoin_build_grid.restype = ctypes.c_int
    lib.selfjoin_build_grid.argtypes = [_vp, _i64, ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(sj_opts), _vp, ctypes.POINTER(_vp)]
    lib.selfjoin_count.restype = ctypes.c_int
    lib.selfjoin_count.argtypes = [_vp, ctypes.c_int, _vp, _i64p, ctypes.POINTER(sj_stats), _vp]
    lib.selfjoin_core_points.restype = ctypes.c_int
    lib.selfjoin_core_points.argtypes = [_vp, ctypes.c_int, ctypes.c_int32, _vp, _i64p, _vp]
    lib.selfjoin_knn.restype = ctypes.c_int
    lib.selfjoin_knn.argtypes = [_vp, ctypes.c_int, ctypes.c_int32, _i64, _vp, _vp, _vp, _vp]
    lib.selfjoin_pairs.restype = ctypes.c_int
    lib.selfjoin_pairs.argtypes = [_vp, ctypes.c_int, _i64, _vp, _vp, _i64, _i64p, _i64p,
                                   ctypes.POINTER(sj_stats), _vp]
    lib.selfjoin_measure_error.restype = ctypes.c_int
    lib.selfjoin_measure_error.argtypes = [_vp, ctypes.c_int, _dp, _dp, _i64p, _vp]
    lib.selfjoin_grid_info.restype = ctypes.c_int
    lib.selfjoin_grid_info.argtypes = [_vp, ctypes.POINTER(sj_grid_info), _vp]
    lib.selfjoin_free_grid.restype = None
    lib.selfjoin_free_grid.argtypes = [_vp, _vp]
    lib.selfjoin_status_string.restype = ctypes.c_char_p
    lib.selfjoin_status_string.argtypes = [ctypes.c_int]
    lib.selfjoin_last_error.restype = ctypes.c_char_p
    lib.selfjoin_last_error.argtypes = []
    lib.selfjoin_version.restype = ctypes.c_char_p
    lib.selfjoin_version.argtypes = []
    lib.selfjoin_batch_build.restype = ctypes.c_int
    lib.selfjoin_batch_build.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp), _i64p, ctypes.POINTER(ctypes.c_int32),
                                         _dp, ctypes.POINTER(sj_opts), _vp, ctypes.POINTER(_vp)]
    lib.selfjoin_batch_count.restype = ctypes.c_int
    lib.selfjoin_batch_count.argtypes = [_vp, ctypes.c_int, _i64p, ctypes.POINTER(sj_stats), _vp]
    lib.selfjoin_batch_pairs.restype = ctypes.c_int
    lib.selfjoin_batch_pairs.argtypes = [_vp, ctypes.c_int, _vp, _i64, _i64p, ctypes.POINTER(sj_stats), _vp]
    lib.selfjoin_batch_info.restype = ctypes.c_int
    lib.selfjoin_batch_info.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _i64p]
    lib.selfjoin_batch_free.restype = None
    lib.selfjoin_batch_free.argtypes = [_vp, _vp]
    lib.selfjoin_count_noalloc.restype = ctypes.c_int
    lib.selfjoin_count_noalloc.argtypes = [_vp, _i64, ctypes.c_int32, ctypes.c_double, ctypes.c_int, _vp, _i64p,
                                           _vp]
    lib.selfjoin_probe_peaks.restype = ctypes.c_int
    lib.selfjoin_probe_peaks.argtypes = [_i64, ctypes.POINTER(sj_peaks), _vp]
    _lib = lib
    return lib


class SelfJoinError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.selfjoin_status_string(status).decode()
        detail = lib.selfjoin_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def check(status: int, where: str):
    if status != SJ_OK:
        raise SelfJoinError(status, where)
