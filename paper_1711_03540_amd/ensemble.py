"""Python front end of a ragged ensemble of periodic KS lattices (libkslb)."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np

from . import _lib
from ._lib import call, fn
from .lattice import _dptr, _prec


class Ensemble:
    """``len(sizes)`` independent periodic lattices.

    Instance i has capacity ``sizes[i]`` sites, scheme ``q[i]`` and storage
    ``precision[i]`` (either may be one value for all) and its own
    coefficients (``set_physical``, for one instance or all).
    ``advance(steps)`` moves instance i by ``steps[i]`` steps, one kernel
    launch per chunk of steps for each (scheme, storage) present.
    """

    def __init__(self, sizes: Sequence[int], q=7, precision="fp64", device=None, stream=None):
        import torch
        self.sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
        self.count = int(self.sizes.size)
        self.qs = np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.int32), (self.count,)))
        precs = [precision] * self.count if isinstance(precision, (str, int)) else list(precision)
        if len(precs) != self.count:
            raise ValueError("one precision per instance, or one for all")
        self.precs = np.ascontiguousarray(np.asarray([_prec(p) for p in precs], dtype=np.int32))
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = fn("kslb_ensemble_bytes")(self.count, _dptr(self.sizes), _dptr(self.qs), _dptr(self.precs))
        if nbytes == 0:
            raise ValueError("bad ensemble shape")
        self.nbytes = nbytes
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            call("kslb_ensemble_create", ctypes.byref(h), self.count, _dptr(self.sizes), _dptr(self.qs),
                 _dptr(self.precs), ctypes.c_void_p(self.buf.data_ptr()), nbytes,
                 ctypes.c_void_p(self.stream.cuda_stream))
        self._h = h
        self.n = self.sizes.copy()
        self.chunk = 64

    def set_physical(self, dX: float, dT: float, tau: float = 0.0, dm_variant: int = 0,
                     guard: str = "refuse", rho_max: float = 3.0, idx: int = -1) -> "Ensemble":
        """Coefficients of instance idx, or of every instance (idx = -1)."""
        g = {"refuse": _lib.GUARD_REFUSE, "raise": _lib.GUARD_RAISE_TAU, "off": _lib.GUARD_OFF}[guard]
        call("kslb_ensemble_set_physical", self._h, int(idx), dX, dT, tau, dm_variant, g, rho_max)
        return self

    def tau_of(self, idx: int) -> float:
        t = ctypes.c_double()
        call("kslb_ensemble_get_tau", self._h, int(idx), ctypes.byref(t))
        return t.value

    @property
    def tau(self) -> float:
        """tau of instance 0 (the tau of every instance after set_physical for all
        instances of one scheme)."""
        return self.tau_of(0)

    def tiling(self) -> dict:
        """The tiling in effect: sites per lane, instance tiles per window, steps per launch."""
        b, m, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        call("kslb_ensemble_get_tiling", self._h, ctypes.byref(b), ctypes.byref(m), ctypes.byref(c))
        return {"sites_per_lane": b.value, "max_segments": m.value, "steps_per_chunk": c.value}

    def set_tiling(self, sites_per_lane: int = 0, max_segments: int = 0, steps_per_chunk: int = 0) -> "Ensemble":
        """Sites per lane (4/8; 10 with FP32, 12 with FP64 and 16 with the rho-only storage throughout),
        instance tiles per workgroup window, steps per launch (0 = keep)."""
        call("kslb_ensemble_set_tiling", self._h, sites_per_lane, max_segments, steps_per_chunk)
        self.chunk = steps_per_chunk or getattr(self, "chunk", 64)
        return self

    def set_graphs(self, enable: bool = True) -> "Ensemble":
        """Replay steady-state chunk pairs from a captured HIP graph (default on)."""
        call("kslb_ensemble_set_graphs", self._h, int(bool(enable)))
        return self

    def resize(self, idx: int, n: int) -> "Ensemble":
        call("kslb_ensemble_resize", self._h, int(idx), int(n))
        self.n[idx] = n
        return self

    def bind(self, idx: int, n: int, dev_ptr: int, nbytes: int) -> "Ensemble":
        """Rebind instance idx to n sites whose state lives at device address
        dev_ptr (nbytes >= kslb_instance_bytes, 256-byte aligned, owned by the
        caller); its state is dropped."""
        call("kslb_ensemble_bind", self._h, int(idx), int(n), ctypes.c_void_p(int(dev_ptr)), int(nbytes))
        self.n[idx] = n
        return self

    def init_rho(self, idx: int, rho) -> "Ensemble":
        import torch
        if isinstance(rho, torch.Tensor) and rho.is_cuda:
            r = rho.to(torch.float64).contiguous()
            call("kslb_ensemble_init_rho", self._h, int(idx), ctypes.c_void_p(r.data_ptr()), 1)
        else:
            r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
            assert r.size == self.n[idx]
            call("kslb_ensemble_init_rho", self._h, int(idx), _dptr(r), 0)
        return self

    def init_rho_all(self, rho) -> "Ensemble":
        """Initialise every instance from the densities of all instances back to
        back in instance order (one launch per scheme and storage present)."""
        import torch
        total = int(np.sum(self.n))
        if isinstance(rho, torch.Tensor) and rho.is_cuda:
            r = rho.to(torch.float64).contiguous()
            assert r.numel() == total
            call("kslb_ensemble_init_rho_all", self._h, ctypes.c_void_p(r.data_ptr()), 1)
        else:
            r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
            assert r.size == total
            call("kslb_ensemble_init_rho_all", self._h, _dptr(r), 0)
        return self

    def advance(self, steps) -> "Ensemble":
        s = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.int64), (self.count,)))
        call("kslb_ensemble_advance", self._h, _dptr(s))
        return self

    def rho(self, idx: int) -> np.ndarray:
        out = np.zeros(int(self.n[idx]))
        call("kslb_ensemble_read_rho", self._h, int(idx), _dptr(out), 0)
        return out

    def read_rho(self, idx: int, out):
        call("kslb_ensemble_read_rho", self._h, int(idx), ctypes.c_void_p(out.data_ptr()), 1)
        return out

    def rho_all(self, out=None):
        """Densities of every instance back to back in instance order: into the
        float64 device tensor `out` (enqueued), or returned as a host array."""
        import torch
        total = int(np.sum(self.n))
        if out is not None:
            assert out.is_cuda and out.numel() >= total and out.dtype == torch.float64 and out.is_contiguous()
            call("kslb_ensemble_read_rho_all", self._h, ctypes.c_void_p(out.data_ptr()), 1)
            return out
        host = np.zeros(total)
        call("kslb_ensemble_read_rho_all", self._h, _dptr(host), 0)
        return host

    def status(self, idx: int):
        s, f = ctypes.c_int64(), ctypes.c_int()
        call("kslb_ensemble_status", self._h, int(idx), ctypes.byref(s), ctypes.byref(f))
        return s.value, bool(f.value)

    def renormalize(self, ref, pert, delta: float, log_accum):
        """Benettin step on trajectory pairs (ref[p], pert[p]); adds ln(d / delta)
        to log_accum[p], a float64 device tensor of len(ref) entries."""
        import numpy as np
        r = np.ascontiguousarray(np.asarray(ref, dtype=np.int32))
        p = np.ascontiguousarray(np.asarray(pert, dtype=np.int32))
        assert r.size == p.size and log_accum.numel() >= r.size and log_accum.is_cuda
        call("kslb_ensemble_renormalize", self._h, int(r.size), r.ctypes.data_as(ctypes.c_void_p),
             p.ctypes.data_as(ctypes.c_void_p), float(delta), ctypes.c_void_p(log_accum.data_ptr()))
        return self

    def orthonormalize(self, ref, pert, delta: float, log_accum):
        """Lyapunov-spectrum step on groups (ref[g], pert[g][0..k-1]): QR of the
        perturbations, each rescaled to delta; adds ln(R_mm / delta) to
        log_accum[g * k + m], a float64 device tensor."""
        r = np.ascontiguousarray(np.asarray(ref, dtype=np.int32))
        p = np.ascontiguousarray(np.asarray(pert, dtype=np.int32).reshape(r.size, -1))
        k = p.shape[1]
        assert log_accum.numel() >= r.size * k and log_accum.is_cuda
        call("kslb_ensemble_orthonormalize", self._h, int(r.size), int(k), r.ctypes.data_as(ctypes.c_void_p),
             p.ctypes.data_as(ctypes.c_void_p), float(delta), ctypes.c_void_p(log_accum.data_ptr()))
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            fn("kslb_ensemble_destroy")(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
