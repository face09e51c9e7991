"""The C-ABI library without a GPU: it loads, exports every entry point that
include/mf.h declares, and rejects invalid arguments before touching the
device (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_1406_1717_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mf_median_filter", "mf_median_filter_i32", "mf_median_filter_batched",
                     "mf_median_filter_backward", "mf_plan_create_batched", "mf_plan_execute",
                     "mf_plan_destroy", "mf_output_length", "mf_status_string", "mf_last_error"):
        assert required in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports(name):
    L = lib.load()
    assert hasattr(L, name), name


def test_output_length():
    assert lib.mf_output_length(10, 3) == 8
    assert lib.mf_output_length(10, 10) == -1     # even
    assert lib.mf_output_length(9, 9) == 1
    assert lib.mf_output_length(5, 7) == -1
    assert lib.mf_output_length(5, 0) == -1
    assert lib.mf_output_length(1, 1) == 1


def test_status_strings():
    for s in range(6):
        assert isinstance(lib.status_string(s), str) and lib.status_string(s)


FAKE = ctypes.c_void_p(256)   # never dereferenced: every call below fails validation


@pytest.mark.parametrize("n,k,code", [
    (10, 4, 1), (10, 0, 1), (10, -3, 1), (10, 11, 1), (0, 1, 1),
    (2**31, 3, 2), (100000, 32769, 2),
])
def test_forward_validation(n, k, code):
    L = lib.load()
    assert L.mf_median_filter(FAKE, n, k, FAKE, None, None) == code
    assert L.mf_median_filter_i32(FAKE, n, k, FAKE, None, None) == code
    assert L.mf_median_filter_noalloc(FAKE, n, k, FAKE, None, None) == code
    assert L.mf_median_filter_f64(FAKE, n, k, FAKE, None, None) == code
    assert L.mf_median_filter_i64(FAKE, n, k, FAKE, None, None) == code
    assert lib.last_error()


def test_null_pointers_rejected():
    L = lib.load()
    assert L.mf_median_filter(None, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter(FAKE, 10, 3, None, None, None) == 1
    assert L.mf_median_filter_noalloc(None, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_f64(None, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_i64(FAKE, 10, 3, None, None, None) == 1
    assert L.mf_median_filter_backward(None, FAKE, 10, 3, FAKE, None) == 1
    assert L.mf_median_filter_backward_f64(FAKE, None, 10, 3, FAKE, None) == 1
    assert L.mf_median_filter_backward_f64(FAKE, FAKE, 10, 4, FAKE, None) == 1
    assert L.mf_median_filter_backward_rows_f64(FAKE, FAKE, 0, 10, 3, FAKE, None) == 1
    assert L.mf_median_filter_rows(FAKE, 0, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_rows_i32(FAKE, 0, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_rows_i32(None, 2, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_rows_f64(FAKE, 0, 10, 3, FAKE, None, None) == 1
    assert L.mf_median_filter_rows_i64(FAKE, 2, 10, 4, FAKE, None, None) == 1
    h = ctypes.c_void_p()
    assert L.mf_plan_create_batched(None, None, 1, ctypes.byref(h)) == 1
    assert L.mf_plan_execute(None, FAKE, FAKE, None, None) == 1


def test_batched_plan_validation():
    import numpy as np
    L = lib.load()
    h = ctypes.c_void_p()
    off = np.array([0, 10, 15], dtype=np.int64)
    for ks in ([3, 7], [4, 3], [3, 0]):        # window above length, even, zero
        k = np.array(ks, dtype=np.int32)
        rc = L.mf_plan_create_batched(off.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                                      2, ctypes.byref(h))
        assert rc == 1, ks
        assert "signal" in lib.last_error()
    bad = np.array([1, 10, 15], dtype=np.int64)
    k = np.array([3, 3], dtype=np.int32)
    assert L.mf_plan_create_batched(bad.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                                    2, ctypes.byref(h)) == 1


def test_binding_refuses_without_the_library(monkeypatch, tmp_path):
    """No fallback: without libmf.so every call fails loudly."""
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "missing" / "libmf.so"))
    with pytest.raises(ImportError):
        lib.load()
    with pytest.raises(ImportError):
        lib.mf_output_length(10, 3)
