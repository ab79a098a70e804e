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


# ---------------------------------------------------------------- kernel planning (host only)

from paper_1711_03540_amd.lattice import plan_kernel  # noqa: E402

LDS = 160 * 1024   # one gfx950 workgroup may use the CU's 160 KiB


def test_plan_takes_span_when_every_owner_fits():
    # N = 4096 D1Q7: 128 single-wave owners of 32 sites (128-site windows of
    # 2 sites per lane, 16 steps between exchanges) on a device that keeps
    # 2048 owners resident
    p = plan_kernel(4096, 7, "fp64", span_owners=2048, lds_bytes=LDS)
    assert p == {"kernel": "span", "steps_per_launch": p["steps_per_launch"], "exchange_steps": 16,
                 "workgroups": 128, "lanes": 64}
    assert p["steps_per_launch"] % 16 == 0 and p["steps_per_launch"] > 5_000
    # the rho-only state keeps 3 sites per lane (densities move one lane per step)
    assert plan_kernel(4096, 7, "rho", span_owners=2048, lds_bytes=LDS)["exchange_steps"] == 24


def test_plan_refuses_span_beyond_half_the_resident_owners():
    # a plan uses at most half the owners the device keeps resident: 128
    # owners need 256
    assert plan_kernel(4096, 7, "fp64", span_owners=256, lds_bytes=LDS)["workgroups"] == 128
    # with fewer, AUTO shortens the exchange interval so that wider owners fit
    # (200 resident: at most 100 owners of 128 - 6 s >= 41 sites, s = 14) ...
    p = plan_kernel(4096, 7, "fp64", span_owners=200, lds_bytes=LDS)
    assert p["kernel"] == "span" and p["exchange_steps"] == 14 and p["workgroups"] == 94
    # ... but not below 12 steps between exchanges: then the one-workgroup
    # kernel takes the lattice (4096 = 8 sites x 512 lanes) ...
    p = plan_kernel(4096, 7, "fp64", span_owners=60, lds_bytes=LDS)
    assert p["kernel"] == "resident" and p["workgroups"] == 1 and p["lanes"] == 512
    # ... or tiles, where it does not fit one workgroup
    p = plan_kernel(12345, 7, "fp64", span_owners=64, lds_bytes=LDS)
    assert p["kernel"] == "tiled" and p["steps_per_launch"] == 80
    # an explicit SPAN request that cannot fit is refused
    with pytest.raises(_lib.KslbError) as e:
        plan_kernel(4096, 7, "fp64", kernel="span", steps_per_launch=16, span_owners=255, lds_bytes=LDS)
    assert e.value.status == _lib.KSLB_EINVAL and "resident" in str(e.value)


def test_plan_fixed_ends_and_small_lds():
    # fixed ends run on SPAN or PLAIN only
    assert plan_kernel(301, 5, "fp64", fixed_ends=True, span_owners=2048, lds_bytes=LDS)["kernel"] == "span"
    assert plan_kernel(1201, 7, "fp64", fixed_ends=True, span_owners=8, lds_bytes=LDS)["kernel"] == "plain"
    with pytest.raises(_lib.KslbError):
        plan_kernel(1201, 7, "fp64", fixed_ends=True, kernel="tiled", span_owners=8, lds_bytes=LDS)
    # without room for the one-workgroup kernel's 96 KiB exchange area AUTO tiles instead
    assert plan_kernel(4096, 7, "fp64", span_owners=8, lds_bytes=64 * 1024)["kernel"] == "tiled"
    with pytest.raises(_lib.KslbError):
        plan_kernel(4096, 7, "fp64", kernel="resident", span_owners=8, lds_bytes=64 * 1024)


def test_host_functions_from_many_threads():
    # distinct calls share no unsynchronised state: host-only entry points
    # give the same answers from 8 threads at once as from one
    import threading

    import numpy as np
    from paper_1711_03540_amd.lattice import scheme_coefficients, stability_check
    cases = [(q, dX, dT, tau) for q in (5, 7) for dX in (0.1, 0.2) for dT in (1e-4, 1e-5) for tau in (1.0, 1.3)]
    want = []
    for q, dX, dT, tau in cases:
        _, E, G = scheme_coefficients(q, dX, dT, tau)
        want.append((E, stability_check(q, E, G, 1 / tau, dX, dT, 3.0),
                     plan_kernel(4096 + 97 * q, q, "fp64", span_owners=2048, lds_bytes=LDS)))
    errors = []

    def work():
        try:
            for _ in range(5):
                for (q, dX, dT, tau), (E0, s0, p0) in zip(cases, want):
                    _, E, G = scheme_coefficients(q, dX, dT, tau)
                    assert np.array_equal(E, E0)
                    assert stability_check(q, E, G, 1 / tau, dX, dT, 3.0) == s0
                    assert plan_kernel(4096 + 97 * q, q, "fp64", span_owners=2048, lds_bytes=LDS) == p0
        except Exception as e:   # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=work) for _ in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


def test_probe_library_exports_its_header():
    # the measurement kernels (device peaks) sit in a library of their own
    from paper_1711_03540_amd import probe
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "kslb_probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(kslb_probe_[a-z0-9_]+)\s*\(", text)))
    assert names == sorted(probe.SIGNATURES)
    lib = probe.load()
    for name in names:
        assert hasattr(lib, name)
    assert lib.kslb_probe_copy(None, None, 16, None) != 0      # refused without device work
    assert lib.kslb_probe_lds(None, 1, 1, None) != 0
