"""The C-ABI library loads and exports every entry point include/kslb.h declares.

CPU only: no kernel is launched here.
"""
import ctypes
import os
import re

import pytest

from paper_1711_03540_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kslb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(kslb_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("kslb_create", "kslb_set_physical", "kslb_set_coefficients", "kslb_init_rho",
                 "kslb_advance", "kslb_read_rho", "kslb_read_f", "kslb_destroy",
                 "kslb_ensemble_create", "kslb_ensemble_advance", "kslb_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_state_bytes_and_bad_shapes():
    f = _lib.fn("kslb_state_bytes")
    assert f(4096, 7, 0) == 2 * 4096 * 7 * 8 + 4096
    assert f(4096, 5, 1) == 2 * 4096 * 5 * 4 + 4096
    # rows are padded to a pitch of n rounded up to 64 sites
    assert f(1000, 7, 2) == 2 * (1024 * 8 + 1024 * 7 * 4) + 4096
    assert f(1000, 7, 0) == 2 * 1024 * 7 * 8 + 4096
    assert f(0, 7, 0) == 0
    assert f(16, 6, 0) == 0
    assert f(16, 7, 3) == 2 * 64 * 8 + 4096          # rho only: one row
    assert f(16, 7, 4) == 0


def test_errors_are_reported_without_device_work():
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.kslb_create(ctypes.byref(h), 0, 7, 0, None, 0, None)
    assert st == _lib.KSLB_EINVAL
    assert "shape" in _lib.last_error()
    st = lib.kslb_create(ctypes.byref(h), 64, 7, 0, None, 0, None)
    assert st == _lib.KSLB_EINVAL
    st = lib.kslb_advance(None, 1)
    assert st == _lib.KSLB_EINVAL


def test_ensemble_bytes_per_instance_shapes():
    import numpy as np
    f = _lib.fn("kslb_ensemble_bytes")
    one = _lib.fn("kslb_state_bytes")
    sizes = np.array([1000, 64, 4096, 7], dtype=np.int64)
    qs = np.array([7, 5, 7, 5], dtype=np.int32)
    precs = np.array([0, 1, 2, 3], dtype=np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    # each instance's ping-pong state as a lattice of its own, one diagnostics block
    want = sum(one(int(n), int(q), int(p)) - 4096 for n, q, p in zip(sizes, qs, precs)) + 4096
    assert f(4, ptr(sizes), ptr(qs), ptr(precs)) == want
    bad = qs.copy()
    bad[2] = 6
    assert f(4, ptr(sizes), ptr(bad), ptr(precs)) == 0
    assert f(4, ptr(sizes), None, ptr(precs)) == 0
    h = ctypes.c_void_p()
    lib = _lib.load()
    assert lib.kslb_ensemble_create(ctypes.byref(h), 4, ptr(sizes), ptr(bad), ptr(precs), None, 0, None) \
        == _lib.KSLB_EINVAL
    assert "instance 2" in _lib.last_error()
