"""Python front end of one periodic KS lattice (thin wrapper over libkslb).

PyTorch provides the device memory and the stream; every step of the method
runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import call, fn


def _dptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.c_void_p)


def scheme_coefficients(q: int, dX: float, dT: float, tau: float, dm_variant: int = 0):
    """(jkm[5], E[q], G[q]) from the host parameter code of the library."""
    jkm = np.zeros(5)
    E = np.zeros(q)
    G = np.zeros(q)
    call("kslb_scheme_coefficients", q, dX, dT, tau, dm_variant, _dptr(jkm), _dptr(E), _dptr(G))
    return jkm, E, G


def tau_fit(q: int, dX: float, dT: float) -> float:
    return fn("kslb_tau_fit")(q, dX, dT)


def spectral_radius(q: int, E, G, omega: float, rho_bar: float, k: float) -> float:
    E = np.ascontiguousarray(E, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    r = ctypes.c_double(0.0)
    call("kslb_spectral_radius", q, _dptr(E), _dptr(G), omega, rho_bar, k, ctypes.byref(r))
    return r.value


def stability_check(q: int, E, G, omega: float, dX: float, dT: float, rho_max: float) -> bool:
    E = np.ascontiguousarray(E, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    s = ctypes.c_int(0)
    call("kslb_stability_check", q, _dptr(E), _dptr(G), omega, dX, dT, rho_max, ctypes.byref(s))
    return bool(s.value)


def _prec(p) -> int:
    return _lib.PRECISIONS[p] if isinstance(p, str) else int(p)


def plan_kernel(n: int, q: int = 7, precision="fp64", fixed_ends: bool = False, kernel="auto",
                steps_per_launch: int = 0, span_owners: int = 0, lds_bytes: int = 0) -> dict:
    """Kernel class and launch shape an advance would take (host only; 0 for a
    limit queries the current device)."""
    k = _lib.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    ko, spl, ex, wg, ln = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
    call("kslb_plan_kernel", int(n), int(q), _prec(precision), int(bool(fixed_ends)), k, int(steps_per_launch),
         int(span_owners), int(lds_bytes), ctypes.byref(ko), ctypes.byref(spl), ctypes.byref(ex), ctypes.byref(wg),
         ctypes.byref(ln))
    name = {v: nm for nm, v in _lib.KERNELS.items()}[ko.value]
    return {"kernel": name, "steps_per_launch": spl.value, "exchange_steps": ex.value,
            "workgroups": wg.value, "lanes": ln.value}


class Lattice:
    """One periodic lattice of ``n`` sites, scheme D1Q``q``, on a GPU."""

    def __init__(self, n: int, q: int = 7, precision="fp64", device=None, stream=None):
        import torch
        self.n, self.q, self.precision = int(n), int(q), _prec(precision)
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = fn("kslb_state_bytes")(self.n, self.q, self.precision)
        if nbytes == 0:
            raise ValueError("bad lattice shape n=%d q=%d precision=%r" % (n, q, precision))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            call("kslb_create", ctypes.byref(h), self.n, self.q, self.precision,
                 ctypes.c_void_p(self.buf.data_ptr()), nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        self._h = h

    # -- parameters -------------------------------------------------------
    def set_physical(self, dX: float, dT: float, tau: float = 0.0, dm_variant: int = 0,
                     guard: str = "refuse", rho_max: float = 3.0) -> "Lattice":
        g = {"refuse": _lib.GUARD_REFUSE, "raise": _lib.GUARD_RAISE_TAU, "off": _lib.GUARD_OFF}[guard]
        call("kslb_set_physical", self._h, dX, dT, tau, dm_variant, g, rho_max)
        self._phys = (dX, dT, dm_variant, guard, rho_max)
        return self

    def set_coefficients(self, E, G, omega: float) -> "Lattice":
        E = np.ascontiguousarray(E, dtype=np.float64)
        G = np.ascontiguousarray(G, dtype=np.float64)
        call("kslb_set_coefficients", self._h, _dptr(E), _dptr(G), omega)
        return self

    def coefficients(self) -> dict:
        E, G, jkm = np.zeros(self.q), np.zeros(self.q), np.zeros(5)
        om, tau = ctypes.c_double(), ctypes.c_double()
        call("kslb_get_coefficients", self._h, _dptr(E), _dptr(G), ctypes.byref(om), ctypes.byref(tau),
             _dptr(jkm))
        return {"E": E, "G": G, "omega": om.value, "tau": tau.value, "J": jkm[0], "K": jkm[1],
                "M": jkm[2], "dM": jkm[3], "C6": jkm[4]}

    def set_kernel(self, kind="auto", steps_per_launch: int = 0) -> "Lattice":
        k = _lib.KERNELS[kind] if isinstance(kind, str) else int(kind)
        call("kslb_set_kernel", self._h, k, steps_per_launch)
        return self

    def kernel(self) -> dict:
        """The kernel an advance runs now (AUTO resolved) and its launch shape."""
        k, spl, ex, wg, ln = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
        call("kslb_get_kernel", self._h, ctypes.byref(k), ctypes.byref(spl), ctypes.byref(ex), ctypes.byref(wg),
             ctypes.byref(ln))
        name = {v: n for n, v in _lib.KERNELS.items()}[k.value]
        return {"kernel": name, "steps_per_launch": spl.value, "exchange_steps": ex.value,
                "workgroups": wg.value, "lanes": ln.value}

    def set_fixed_ends(self, rho_left: float, rho_right: float) -> "Lattice":
        """Fixed-end boundary of the paper's Table 3 problem (set before init_rho)."""
        call("kslb_set_boundary", self._h, 1, float(rho_left), float(rho_right))
        return self

    def set_periodic(self) -> "Lattice":
        call("kslb_set_boundary", self._h, 0, 0.0, 0.0)
        return self

    # -- state ------------------------------------------------------------
    def init_rho(self, rho) -> "Lattice":
        import torch
        if isinstance(rho, torch.Tensor) and rho.is_cuda:
            r = rho.to(torch.float64).contiguous()
            assert r.numel() == self.n
            call("kslb_init_rho", self._h, ctypes.c_void_p(r.data_ptr()), 1)
            self._keep = r
        else:
            r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
            assert r.size == self.n
            call("kslb_init_rho", self._h, _dptr(r), 0)
        return self

    def advance(self, steps: int) -> "Lattice":
        call("kslb_advance", self._h, int(steps))
        return self

    def solve(self, rho0, steps: int, out=None):
        """init_rho(rho0) + advance(steps) + read_rho(out) as one enqueued call
        (kslb_solve: fused into the first and last launches of the tiled
        kernel); rho0 a float64 device tensor of n sites; out may be rho0
        itself.  Returns out."""
        import torch
        if not (isinstance(rho0, torch.Tensor) and rho0.is_cuda):
            raise TypeError("solve takes the initial density as a device tensor")
        r = rho0.to(torch.float64).contiguous()
        assert r.numel() == self.n
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        assert out.numel() == self.n and out.dtype == torch.float64 and out.is_contiguous()
        call("kslb_solve", self._h, ctypes.c_void_p(r.data_ptr()), int(steps), ctypes.c_void_p(out.data_ptr()))
        self._keep = r
        return out

    def advance_guarded(self, steps: int, chunk: int = 1000, tau_step: float = 0.02, max_raises: int = 50,
                        bound: float = None) -> "Lattice":
        """Advance `steps` steps in chunks, saving the state before each chunk.  A
        chunk that ends with a non-finite state (the library's flag) or, if
        `bound` is given, with max |rho| above it, is rolled back and run again
        with tau raised by `tau_step` (the minimum stable tau of section 3 grows
        with dT; raising tau is how its scans restore stability).  Each recovery
        is recorded as (step, old tau, new tau) in `self.recoveries`.  FP64 and
        FP32 storage (split storage encodes the state against the coefficients;
        the rho-only storage is tied to tau = 1)."""
        if self.precision not in (_lib.PRECISIONS["fp64"], _lib.PRECISIONS["fp32"]):
            raise ValueError("advance_guarded needs fp64 or fp32 storage")
        if getattr(self, "_phys", None) is None:
            raise ValueError("set_physical first")
        dX, dT, dm, guard, rho_max = self._phys
        self.recoveries = []
        left = int(steps)
        raises = 0
        while left > 0:
            n = min(int(chunk), left)
            ckpt, step0 = self.save_state(), self.step
            self.advance(n)
            _, bad = self.diagnostics()
            if not bad and bound is not None:
                bad = not (np.max(np.abs(self.rho())) <= bound)
            if not bad:
                left -= n
                continue
            if raises >= max_raises:
                raise FloatingPointError("unstable after %d raises of tau" % raises)
            old = self.coefficients()["tau"]
            self.load_state(ckpt, step0)
            call("kslb_set_physical", self._h, dX, dT, old + tau_step, dm, _lib.GUARD_OFF, rho_max)
            self.recoveries.append((step0, old, self.coefficients()["tau"]))
            raises += 1
        return self

    def read_rho(self, out=None):
        """Density as a float64 device tensor (enqueued on the lattice stream)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        call("kslb_read_rho", self._h, ctypes.c_void_p(out.data_ptr()), 1)
        return out

    def rho(self) -> np.ndarray:
        out = np.zeros(self.n)
        call("kslb_read_rho", self._h, _dptr(out), 0)
        return out

    def f(self, pre_collision: bool = False) -> np.ndarray:
        out = np.zeros((self.q, self.n))
        call("kslb_read_f", self._h, _dptr(out), 0, int(bool(pre_collision)))
        return out

    def write_f(self, f, step: int = 0) -> "Lattice":
        a = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        assert a.shape == (self.q, self.n)
        call("kslb_write_f", self._h, _dptr(a), 0, int(step))
        return self

    def save_state(self):
        import torch
        size = fn("kslb_state_size")(self._h)
        out = torch.empty(size, dtype=torch.uint8, device=self.device)
        call("kslb_save_state", self._h, ctypes.c_void_p(out.data_ptr()))
        return out

    def load_state(self, blob, step: int) -> "Lattice":
        call("kslb_load_state", self._h, ctypes.c_void_p(blob.data_ptr()), int(step))
        self._keep = blob
        return self

    @property
    def step(self) -> int:
        s = ctypes.c_int64()
        call("kslb_step_count", self._h, ctypes.byref(s))
        return s.value

    def diagnostics(self):
        m, f = ctypes.c_double(), ctypes.c_int()
        call("kslb_diagnostics", self._h, ctypes.byref(m), ctypes.byref(f))
        return m.value, bool(f.value)

    def aborted_launches(self) -> int:
        """Multi-workgroup launches of this lattice that stopped early (synchronises)."""
        c = ctypes.c_int64()
        call("kslb_aborted_launches", self._h, ctypes.byref(c))
        return c.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            fn("kslb_destroy")(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
