"""MI355X (gfx950) lattice Boltzmann solver for the Kuramoto-Sivashinsky equation.

The method is the BGK lattice Boltzmann scheme of Otomo, Boghosian & Dubois
(arXiv:1711.03540) on periodic D1Q5 ("basic") and D1Q7 ("improved") lattices.
The compute path is the HIP library libkslb.so (C ABI in include/kslb.h);
this package only marshals arguments and supplies PyTorch device memory and
streams.  Importing the package loads nothing; the first object created loads
the library and raises if it was not built.
"""
from ._lib import KslbError  # noqa: F401


def __getattr__(name):
    if name in ("Lattice", "scheme_coefficients", "tau_fit", "spectral_radius", "stability_check"):
        from . import lattice
        return getattr(lattice, name)
    if name == "Ensemble":
        from .ensemble import Ensemble
        return Ensemble
    raise AttributeError(name)
