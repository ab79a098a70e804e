"""The no-allocation advance (kslb_advance_noalloc) against kslb_advance.

Two calls in a row through the C ABI, the second with a smaller lattice: each
must leave bitwise the state the allocating advance leaves.  The SPAN kernel's
edge slots then come from the library's static device array (longer advances
split into more launches); other kernel classes use no scratch.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_1711_03540_amd import _lib
from paper_1711_03540_amd.inputs import random_modes_ic
from paper_1711_03540_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def pair(n, q, kernel, prec="fp64", dX=math.pi / 16, dT=1e-4):
    rho0 = random_modes_ic(n, n * dX, seed=n + q)
    out = []
    for _ in range(2):
        lat = Lattice(n, q, prec).set_physical(dX, dT, 0.0).set_kernel(kernel)
        out.append(lat.init_rho(rho0))
    return out, rho0


@pytest.mark.parametrize("first,second", [((4096, 7, "span", 12000), (1000, 5, "span", 700)),
                                          ((70001, 7, "tiled", 130), (3000, 7, "span", 50))])
def test_noalloc_advance_equals_advance_twice(first, second):
    for n, q, kernel, steps in (first, second):
        say("case noalloc: n=%d q=%d kernel=%s steps=%d" % (n, q, kernel, steps))
        (a, b), rho0 = pair(n, q, kernel)
        assert a.kernel()["kernel"] == kernel
        _lib.call("kslb_advance", a._h, ctypes.c_int64(steps))
        _lib.call("kslb_advance_noalloc", b._h, ctypes.c_int64(steps))
        assert b.step == a.step == steps
        assert np.array_equal(a.f(), b.f())
        assert np.array_equal(a.rho(), b.rho())
        assert b.aborted_launches() == 0
        if kernel == "span" and n == 4096:
            # a SPAN advance of 12000 steps needs more launches from the 64 MiB
            # static area than from the lattice's own, so a mix of the two in
            # one lattice must also agree; and both match the oracle
            _lib.call("kslb_advance_noalloc", a._h, ctypes.c_int64(250))
            _lib.call("kslb_advance", b._h, ctypes.c_int64(250))
            assert np.array_equal(a.f(), b.f())
            tau = a.coefficients()["tau"]
            ref = oracle.solve_periodic(q, rho0, math.pi / 16, 1e-4, tau, steps + 250)
            assert np.max(np.abs(a.rho() - ref)) <= 1e-12 * np.max(np.abs(ref))
        a.close()
        b.close()
