"""ctypes binding of libkslb.so (argument marshalling only).

Every entry point of include/kslb.h is declared here with the same name.  The
library is loaded from this package's directory; there is no fallback: if it
is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkslb.so")

KSLB_OK, KSLB_EINVAL, KSLB_ENOMEM, KSLB_EDEVICE, KSLB_ESTATE, KSLB_EUNSTABLE, KSLB_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6
FP64, FP32, SPLIT, RHO = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "split": SPLIT, "rho": RHO}
DM_DERIVED, DM_LITERAL = 0, 1
GUARD_REFUSE, GUARD_RAISE_TAU, GUARD_OFF = 0, 1, 2
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_RESIDENT, KERNEL_TILED, KERNEL_SPAN = 0, 1, 2, 3, 4
KERNELS = {"auto": KERNEL_AUTO, "plain": KERNEL_PLAIN, "resident": KERNEL_RESIDENT,
           "tiled": KERNEL_TILED, "span": KERNEL_SPAN}

_ERRNAMES = {KSLB_EINVAL: "EINVAL", KSLB_ENOMEM: "ENOMEM", KSLB_EDEVICE: "EDEVICE",
             KSLB_ESTATE: "ESTATE", KSLB_EUNSTABLE: "EUNSTABLE", KSLB_ENONFINITE: "ENONFINITE"}


class KslbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(status, "?"), status, message))
        self.status = status


_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_sz = ctypes.c_size_t
_st = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "kslb_scheme_coefficients": (_st, [_i, _d, _d, _d, _i, _vp, _vp, _vp]),
    "kslb_tau_fit": (_d, [_i, _d, _d]),
    "kslb_spectral_radius": (_st, [_i, _vp, _vp, _d, _d, _d, _vp]),
    "kslb_stability_check": (_st, [_i, _vp, _vp, _d, _d, _d, _d, _vp]),
    "kslb_state_bytes": (_sz, [_i64, _i, _i]),
    "kslb_create": (_st, [_vp, _i64, _i, _i, _vp, _sz, _vp]),
    "kslb_set_physical": (_st, [_vp, _d, _d, _d, _i, _i, _d]),
    "kslb_set_coefficients": (_st, [_vp, _vp, _vp, _d]),
    "kslb_get_coefficients": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "kslb_set_kernel": (_st, [_vp, _i, _i]),
    "kslb_get_kernel": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "kslb_plan_kernel": (_st, [_i64, _i, _i, _i, _i, _i, _i64, _i, _vp, _vp, _vp, _vp, _vp]),
    "kslb_set_boundary": (_st, [_vp, _i, _d, _d]),
    "kslb_init_rho": (_st, [_vp, _vp, _i]),
    "kslb_advance": (_st, [_vp, _i64]),
    "kslb_solve": (_st, [_vp, _vp, _i64, _vp]),
    "kslb_advance_noalloc": (_st, [_vp, _i64]),
    "kslb_read_rho": (_st, [_vp, _vp, _i]),
    "kslb_read_f": (_st, [_vp, _vp, _i, _i]),
    "kslb_write_f": (_st, [_vp, _vp, _i, _i64]),
    "kslb_state_size": (_sz, [_vp]),
    "kslb_save_state": (_st, [_vp, _vp]),
    "kslb_load_state": (_st, [_vp, _vp, _i64]),
    "kslb_step_count": (_st, [_vp, _vp]),
    "kslb_diagnostics": (_st, [_vp, _vp, _vp]),
    "kslb_aborted_launches": (_st, [_vp, _vp]),
    "kslb_destroy": (_st, [_vp]),
    "kslb_ensemble_bytes": (_sz, [_i, _vp, _vp, _vp]),
    "kslb_ensemble_create": (_st, [_vp, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "kslb_ensemble_set_physical": (_st, [_vp, _i, _d, _d, _d, _i, _i, _d]),
    "kslb_ensemble_get_tau": (_st, [_vp, _i, _vp]),
    "kslb_ensemble_set_tiling": (_st, [_vp, _i, _i, _i]),
    "kslb_ensemble_get_tiling": (_st, [_vp, _vp, _vp, _vp]),
    "kslb_ensemble_set_graphs": (_st, [_vp, _i]),
    "kslb_ensemble_resize": (_st, [_vp, _i, _i64]),
    "kslb_instance_bytes": (_sz, [_i64, _i, _i]),
    "kslb_ensemble_bind": (_st, [_vp, _i, _i64, _vp, _sz]),
    "kslb_ensemble_init_rho": (_st, [_vp, _i, _vp, _i]),
    "kslb_ensemble_init_rho_all": (_st, [_vp, _vp, _i]),
    "kslb_ensemble_read_rho_all": (_st, [_vp, _vp, _i]),
    "kslb_ensemble_orthonormalize": (_st, [_vp, _i, _i, _vp, _vp, _d, _vp]),
    "kslb_ensemble_advance": (_st, [_vp, _vp]),
    "kslb_ensemble_read_rho": (_st, [_vp, _i, _vp, _i]),
    "kslb_ensemble_status": (_st, [_vp, _i, _vp, _vp]),
    "kslb_ensemble_renormalize": (_st, [_vp, _i, _vp, _vp, _d, _vp]),
    "kslb_ensemble_destroy": (_st, [_vp]),
    "kslb_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libkslb.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkslb.so not found at %s: build it first (python -c "
                              "'import __graft_entry__ as g; g.build()')" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error() -> str:
    msg = load().kslb_last_error()
    return msg.decode() if msg else ""


def check(status: int) -> None:
    if status != KSLB_OK:
        raise KslbError(status, last_error())


def call(name: str, *args) -> int:
    """Call an entry point that returns kslb_status; raise on error."""
    st = getattr(load(), name)(*args)
    check(st)
    return st


def fn(name: str):
    return getattr(load(), name)
