"""The C-ABI library without a GPU: it loads, exports every function that
include/selfjoin.h declares, and rejects invalid arguments on the host before
any device call."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_2209_11287_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "selfjoin.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(selfjoin_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libselfjoin.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declarations_match_binding_list():
    assert _declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, flags=re.M))
    for name in _declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_status_strings_and_version(lib):
    for s in range(6):
        assert lib.selfjoin_status_string(s)
    assert b"gfx950" in lib.selfjoin_version()
    assert lib.selfjoin_status_string(99) == b"unknown status"


def _build(lib, ptr, n, d, eps, index_dims=0, out=True):
    opts = _lib.sj_opts()
    opts.index_dims = index_dims
    h = ctypes.c_void_p()
    return lib.selfjoin_build_grid(ptr, n, d, eps, ctypes.byref(opts), None,
                                   ctypes.byref(h) if out else None)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("n,d,eps", [(-1, 2, 0.1), (1 << 31, 2, 0.1), (2_000_000_001, 2, 0.1), (10, 0, 0.1), (10, 257, 0.1),
                                     (10, 2, 0.0), (10, 2, -1.0), (10, 2, math.nan), (10, 2, math.inf)])
def test_build_rejects_invalid_arguments(lib, n, d, eps):
    assert _build(lib, FAKE, n, d, eps) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_last_error()


def test_build_rejects_null_pointers_and_bad_options(lib):
    assert _build(lib, None, 10, 2, 0.1) == _lib.SJ_ERR_INVALID
    assert _build(lib, FAKE, 10, 2, 0.1, out=False) == _lib.SJ_ERR_INVALID
    assert _build(lib, FAKE, 10, 2, 0.1, index_dims=5) == _lib.SJ_ERR_INVALID
    assert _build(lib, FAKE, 10, 2, 0.1, index_dims=-2) == _lib.SJ_ERR_INVALID  # -1 = no index


def test_calls_on_null_grid_rejected(lib):
    total = ctypes.c_int64(0)
    assert lib.selfjoin_count(None, 1, None, ctypes.byref(total), None, None) == _lib.SJ_ERR_INVALID
    w = ctypes.c_int64(0)
    nx = ctypes.c_int64(0)
    assert lib.selfjoin_pairs(None, 1, 0, None, None, 0, ctypes.byref(w), ctypes.byref(nx), None,
                              None) == _lib.SJ_ERR_INVALID
    e = ctypes.c_double()
    assert lib.selfjoin_measure_error(None, 1, ctypes.byref(e), ctypes.byref(e), ctypes.byref(w),
                                      None) == _lib.SJ_ERR_INVALID
    info = _lib.sj_grid_info()
    assert lib.selfjoin_grid_info(None, ctypes.byref(info), None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_core_points(None, 1, 4, None, ctypes.byref(w), None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_knn(None, 1, 4, 0, None, None, None, None) == _lib.SJ_ERR_INVALID
    lib.selfjoin_free_grid(None, None)  # accepted


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2209_11287_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
                assert "liboracle" not in src and "selfjoin_oracle" not in src, f


def test_batch_calls_reject_invalid_arguments(lib):
    h = ctypes.c_void_p()
    opts = _lib.sj_opts()
    # B < 0, NULL out
    assert lib.selfjoin_batch_build(-1, None, None, None, None, None, None, ctypes.byref(h)) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_batch_build(0, None, None, None, None, None, None, None) == _lib.SJ_ERR_INVALID
    # a bad problem in the list
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    ns = (ctypes.c_int64 * 2)(10, 10)
    ds = (ctypes.c_int32 * 2)(2, 0)
    es = (ctypes.c_double * 2)(0.1, 0.1)
    assert lib.selfjoin_batch_build(2, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), ns, ds, es,
                                    ctypes.byref(opts), None, ctypes.byref(h)) == _lib.SJ_ERR_INVALID
    ds[1] = 2
    es[0] = float("nan")
    assert lib.selfjoin_batch_build(2, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), ns, ds, es,
                                    ctypes.byref(opts), None, ctypes.byref(h)) == _lib.SJ_ERR_INVALID
    # symmetric outside {0, 1} (every problem valid)
    es[0] = 0.1
    opts.symmetric = 2
    assert lib.selfjoin_batch_build(2, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), ns, ds, es,
                                    ctypes.byref(opts), None, ctypes.byref(h)) == _lib.SJ_ERR_INVALID
    assert b"symmetric" in lib.selfjoin_last_error()
    opts.symmetric = 0
    tot = (ctypes.c_int64 * 1)()
    assert lib.selfjoin_batch_count(None, 1, tot, None, None) == _lib.SJ_ERR_INVALID
    offs = (ctypes.c_int64 * 2)()
    assert lib.selfjoin_batch_pairs(None, 1, None, 0, offs, None, None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_batch_info(None, 0, None, None) == _lib.SJ_ERR_INVALID
    lib.selfjoin_batch_free(None, None)


def test_peak_probe_rejects_invalid_arguments(lib):
    out = _lib.sj_peaks()
    assert lib.selfjoin_probe_peaks(1 << 20, None, None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_probe_peaks(-1, ctypes.byref(out), None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_probe_peaks(8, ctypes.byref(out), None) == _lib.SJ_ERR_INVALID
    assert lib.selfjoin_last_error()


@pytest.mark.parametrize("field,value", [("short_circuit", -2), ("short_circuit", 65), ("dim_order", 2),
                                         ("dim_order", -1), ("symmetric", 2), ("symmetric", -1)])
def test_build_rejects_out_of_range_options(lib, field, value):
    opts = _lib.sj_opts()
    setattr(opts, field, value)
    h = ctypes.c_void_p()
    assert lib.selfjoin_build_grid(FAKE, 10, 2, 0.1, ctypes.byref(opts), None, ctypes.byref(h)) == _lib.SJ_ERR_INVALID
    assert field in lib.selfjoin_last_error().decode()
