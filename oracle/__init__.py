"""FP64 CPU oracle for the lattice Boltzmann scheme for the Kuramoto-Sivashinsky
equation (Otomo, Boghosian & Dubois, arXiv:1711.03540).

TEST INFRASTRUCTURE ONLY: this package checks the GPU library.  Only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark may
import it; the GPU library and its Python binding never do.  It shares no code
with the GPU path: the arithmetic lives in ``ks_oracle.c`` and this module only
builds that file and marshals arrays through ctypes.

Every function names the passage of the paper it follows; see ``ks_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "libks_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile ``ks_oracle.c`` with gcc, FP64, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        p = ctypes.c_void_p
        lib.ko_T.restype = d
        lib.ko_T.argtypes = [i, d]
        lib.ko_coefficients.restype = i
        lib.ko_coefficients.argtypes = [i, d, d, d, i, p]
        lib.ko_tau_fit.restype = d
        lib.ko_tau_fit.argtypes = [i, d, d]
        lib.ko_feq.restype = None
        lib.ko_feq.argtypes = [i, p, d, p]
        lib.ko_weights.restype = i
        lib.ko_weights.argtypes = [p]
        lib.ko_velocities.restype = i
        lib.ko_velocities.argtypes = [i, p]
        lib.ko_collide.restype = i
        lib.ko_collide.argtypes = [i, l, p, d, p, p]
        lib.ko_density.restype = i
        lib.ko_density.argtypes = [i, l, p, p]
        lib.ko_init.restype = i
        lib.ko_init.argtypes = [i, l, p, p, p]
        lib.ko_advance_periodic.restype = i
        lib.ko_advance_periodic.argtypes = [i, l, p, d, p, l]
        lib.ko_solve_periodic.restype = i
        lib.ko_solve_periodic.argtypes = [i, l, d, d, d, i, p, l, p, p]
        lib.ko_tanh_solution.restype = d
        lib.ko_tanh_solution.argtypes = [d, d]
        lib.ko_tanh_left.restype = d
        lib.ko_tanh_left.argtypes = []
        lib.ko_tanh_right.restype = d
        lib.ko_tanh_right.argtypes = []
        lib.ko_solve_tanh_fixed.restype = i
        lib.ko_solve_tanh_fixed.argtypes = [i, d, d, d, i, l, p, ctypes.POINTER(l)]
        lib.ko_global_error.restype = d
        lib.ko_global_error.argtypes = [l, p, p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def velocities(q: int) -> np.ndarray:
    """Lattice velocities in the oracle's order (appendix A)."""
    c = np.zeros(q, dtype=np.int32)
    if _load().ko_velocities(q, _ptr(c)):
        raise ValueError("q must be 5 or 7")
    return c


def weights() -> np.ndarray:
    """7x7 array, row l = w(l)_i (appendix A; rows 0-4 zero at c = +-3)."""
    w = np.zeros((7, 7))
    _load().ko_weights(_ptr(w))
    return w


def T(i: int, tau: float) -> float:
    """Closed form of T_i, section 2, Eq. (T_form)."""
    return _load().ko_T(i, tau)


def coefficients(q: int, dX: float, dT: float, tau: float, dm_variant: int = 0) -> np.ndarray:
    """[J, K, M, dM, C6] (Table 2; the delta f_eq and delta M corrections of section 2.2)."""
    out = np.zeros(5)
    if _load().ko_coefficients(q, dX, dT, tau, dm_variant, _ptr(out)):
        raise ValueError("bad scheme")
    return out


def tau_fit(q: int, dX: float, dT: float) -> float:
    """Minimum stable tau, Eq. (general_tau_formula) with the fitted A, B."""
    return _load().ko_tau_fit(q, dX, dT)


def feq(q: int, coef, rho: float) -> np.ndarray:
    """Equilibrium populations of one site, section 2.3."""
    c = _f64(coef)
    out = np.zeros(q)
    _load().ko_feq(q, _ptr(c), float(rho), _ptr(out))
    return out


def init(q: int, coef, rho0) -> np.ndarray:
    """Populations at equilibrium with rho0 (Q x N)."""
    c, r = _f64(coef), _f64(rho0)
    f = np.zeros((q, r.size))
    _load().ko_init(q, r.size, _ptr(c), _ptr(r), _ptr(f))
    return f


def advance(q: int, coef, tau: float, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance pre-collision populations f (Q x N) by nsteps periodic LB steps, Eq. (2)."""
    c = _f64(coef)
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    rc = _load().ko_advance_periodic(q, g.shape[1], _ptr(c), float(tau), _ptr(g), int(nsteps))
    if rc:
        raise RuntimeError("oracle advance failed (%d)" % rc)
    return g


def collide(q: int, coef, tau: float, f: np.ndarray) -> np.ndarray:
    """Post-collision populations of f (no streaming)."""
    c = _f64(coef)
    f = _f64(f)
    post = np.zeros_like(f)
    _load().ko_collide(q, f.shape[1], _ptr(c), float(tau), _ptr(f), _ptr(post))
    return post


def density(f: np.ndarray) -> np.ndarray:
    f = _f64(f)
    rho = np.zeros(f.shape[1])
    _load().ko_density(f.shape[0], f.shape[1], _ptr(f), _ptr(rho))
    return rho


def solve_periodic(q: int, rho0, dX: float, dT: float, tau: float, nsteps: int,
                   dm_variant: int = 0, want_f: bool = False):
    """Periodic solve from rho0; returns rho (and the pre-collision f if asked)."""
    r0 = _f64(rho0)
    n = r0.size
    rho = np.zeros(n)
    f = np.zeros((q, n)) if want_f else None
    rc = _load().ko_solve_periodic(q, n, dX, dT, tau, dm_variant, _ptr(r0), int(nsteps),
                                   _ptr(rho), _ptr(f) if want_f else None)
    if rc:
        raise RuntimeError("oracle solve failed (%d)" % rc)
    return (rho, f) if want_f else rho


def tanh_solution(X, t: float) -> np.ndarray:
    """Table 3 analytic solution rho(X, t)."""
    lib = _load()
    X = np.atleast_1d(np.asarray(X, dtype=np.float64))
    return np.array([lib.ko_tanh_solution(float(x), float(t)) for x in X])


def tanh_ends():
    lib = _load()
    return lib.ko_tanh_left(), lib.ko_tanh_right()


def solve_tanh_fixed(q: int, dX: float, dT: float, tau: float, nsteps: int, dm_variant: int = 0):
    """Table 3 problem with fixed ends; returns rho at X_j = j dX, j = 0..60/dX."""
    n = int(round(60.0 / dX)) + 1
    rho = np.zeros(n)
    n_out = ctypes.c_long(0)
    rc = _load().ko_solve_tanh_fixed(q, dX, dT, tau, dm_variant, int(nsteps), _ptr(rho),
                                     ctypes.byref(n_out))
    if rc or n_out.value != n:
        raise RuntimeError("oracle fixed-end solve failed (%d)" % rc)
    return rho


def global_error(rho_num, rho_ana) -> float:
    """G of section 3."""
    a, b = _f64(rho_num), _f64(rho_ana)
    return _load().ko_global_error(a.size, _ptr(a), _ptr(b))
