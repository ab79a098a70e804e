"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar: FP64 results within 1e-12 norm-wise relative error of the oracle,
max|x - x_oracle| / max|x_oracle|, for rho and for every population; every
kernel class bitwise identical to every other.  FP32 and split-precision
errors are measured and bounded loosely.
"""
import functools
import math

import numpy as np
import pytest

import oracle
from paper_1711_03540_amd.ensemble import Ensemble
from paper_1711_03540_amd.inputs import (CFG_LARGE_Q7, CFG_RESIDENT_Q7, CFG_SMALL_Q5, kassam_trefethen_ic,
                                         random_modes_ic)
from paper_1711_03540_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def say(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=64)
def oracle_run(q, n, dX, dT, tau, steps, seed, amp=0.3):
    rho0 = ic(n, dX, seed, amp)
    return oracle.solve_periodic(q, rho0, dX, dT, tau, steps, want_f=True)


def ic(n, dX, seed, amp=0.3):
    return 1.0 + random_modes_ic(n, n * dX, seed=seed, n_modes=min(16, max(1, n // 2)), amplitude=amp)


def make(q, n, prec="fp64", kernel="auto", dX=0.2, dT=1e-4, tau=1.1, steps_per_launch=0):
    lat = Lattice(n, q, prec)
    lat.set_physical(dX, dT, tau)
    lat.set_kernel(kernel, steps_per_launch)
    return lat


SIZES = [1, 2, 3, 7, 64, 256, 1000, 1001, 4096, 70001]


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kernel", ["plain", "tiled", "resident", "span", "auto"])
def test_fp64_parity(q, n, kernel):
    dX, dT, tau, steps = 0.2, 1e-4, 1.1, 700
    say("case fp64 parity q=%d n=%d kernel=%s" % (q, n, kernel))
    lat = make(q, n, kernel="plain", dX=dX, dT=dT, tau=tau)
    if kernel in ("resident", "span"):
        try:
            lat.set_kernel(kernel)
        except Exception:
            pytest.skip("n=%d cannot use the %s kernel" % (n, kernel))
    else:
        lat.set_kernel(kernel)
    coef = oracle.coefficients(q, dX, dT, tau)
    rho_ref, f_ref = oracle_run(q, n, dX, dT, tau, steps, 5)
    lat.init_rho(ic(n, dX, 5)).advance(steps)
    assert lat.step == steps
    assert rel(lat.rho(), rho_ref) < TOL64
    # stored state: the collided populations at time `steps`
    assert rel(lat.f(pre_collision=False), oracle.collide(q, coef, tau, f_ref)) < TOL64
    # streamed one link: the oracle's (pre-collision) f one step later
    assert rel(lat.f(pre_collision=True), oracle.advance(q, coef, tau, f_ref, 1)) < TOL64


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("n", [256, 1000, 4096, 12345])
def test_kernel_classes_bitwise_identical(q, n):
    say("case bitwise q=%d n=%d" % (q, n))
    rho0 = ic(n, 0.2, 9)
    outs = []
    for kernel, spl in (("plain", 0), ("tiled", 0), ("tiled", 7), ("tiled", 1), ("resident", 0), ("span", 0),
                        ("span", 5), ("span", 24)):
        lat = make(q, n, kernel="plain")
        try:
            lat.set_kernel(kernel, spl)
        except Exception:
            continue
        lat.init_rho(rho0).advance(333)
        outs.append((kernel, spl, lat.f()))
    assert len(outs) >= 4
    for k, s, f in outs[1:]:
        assert np.array_equal(f, outs[0][2]), (k, s)


@pytest.mark.parametrize("prec", ["fp32", "split"])
@pytest.mark.parametrize("kernel", ["plain", "tiled", "resident", "span"])
def test_reduced_precision_kernels_bitwise_identical(prec, kernel):
    say("case bitwise %s %s" % (prec, kernel))
    n = 4096
    rho0 = ic(n, 0.2, 4)
    ref = make(7, n, prec, "plain").init_rho(rho0).advance(250).f()
    got = make(7, n, prec, kernel).init_rho(rho0).advance(250).f()
    assert np.array_equal(got, ref)


def test_small_config_full_length():
    # D1Q5, N = 256 on L = 32 pi, cos(x/16)(1 + sin(x/16)), dT = (pi/8)^4/90, tau = 1, 10^4 steps
    w = CFG_SMALL_Q5
    say("case %s" % w.name)
    rho0 = w.rho0()
    lat = Lattice(w.n, w.q, "fp64")
    lat.set_physical(w.dX, w.dT, 0.0)
    tau = lat.coefficients()["tau"]
    assert tau == 1.0
    lat.init_rho(rho0).advance(w.steps)
    ref = oracle.solve_periodic(w.q, rho0, w.dX, w.dT, tau, w.steps)
    assert rel(lat.rho(), ref) < TOL64


def test_resident_config_in_bench_launch():
    # D1Q7, N = 4096, 16 random modes, dT = 1e-4, fitted tau, resident kernel as timed
    w = CFG_RESIDENT_Q7
    say("case %s 2000 steps" % w.name)
    rho0 = w.rho0()
    lat = Lattice(w.n, w.q, "fp64")
    lat.set_physical(w.dX, w.dT, 0.0)
    lat.set_kernel("resident")
    tau = lat.coefficients()["tau"]
    assert abs(tau - oracle.tau_fit(7, w.dX, w.dT)) < 1e-15
    lat.init_rho(rho0).advance(2000)
    rho_ref, f_ref = oracle.solve_periodic(w.q, rho0, w.dX, w.dT, tau, 2000, want_f=True)
    assert rel(lat.rho(), rho_ref) < TOL64
    coef = oracle.coefficients(w.q, w.dX, w.dT, tau)
    assert rel(lat.f(), oracle.collide(w.q, coef, tau, f_ref)) < TOL64


@pytest.mark.parametrize("spl", [8, 16, 0])
def test_span_kernel_in_bench_shape(spl):
    # D1Q7, N = 4096, the multi-workgroup kernel with s steps between edge exchanges
    w = CFG_RESIDENT_Q7
    say("case span n=4096 s=%d" % spl)
    rho0 = w.rho0()
    lat = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("span", spl)
    tau = lat.coefficients()["tau"]
    lat.init_rho(rho0).advance(2001)
    mass, bad = lat.diagnostics()          # raises if a workgroup timed out
    assert not bad
    ref = oracle.solve_periodic(w.q, rho0, w.dX, w.dT, tau, 2001)
    assert rel(lat.rho(), ref) < TOL64
    plain = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("plain")
    plain.init_rho(rho0).advance(2001)
    assert np.array_equal(lat.f(), plain.f())


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("n,spl", [(1000, 0), (4096, 0), (4096, 17), (12345, 0), (70001, 0)])
def test_span_exchange_slots(q, n, spl):
    # SPAN owners trade edges through write-once slots polled for a sentinel:
    # bitwise equal to the one-step kernel and to the oracle, over several
    # advances that reuse the slots
    dX, dT, tau, steps = 0.2, 1e-4, 1.1, 700
    rho0 = ic(n, dX, 17)
    lat = make(q, n, dX=dX, dT=dT, tau=tau)
    lat.set_kernel("span", spl)
    k = lat.kernel()
    say("case span slots q=%d n=%d s=%d: %s" % (q, n, spl, k))
    assert k["kernel"] == "span" and k["lanes"] == 64 and k["workgroups"] >= 2
    assert spl == 0 or k["exchange_steps"] == spl
    assert k["steps_per_launch"] % k["exchange_steps"] == 0
    lat.init_rho(rho0).advance(steps)
    mass, bad = lat.diagnostics()          # raises if a workgroup timed out
    assert not bad
    ref = make(q, n, kernel="plain", dX=dX, dT=dT, tau=tau).init_rho(rho0).advance(steps)
    assert np.array_equal(lat.f(), ref.f())
    if n <= 4096:
        assert rel(lat.rho(), oracle_run(q, n, dX, dT, tau, steps, 17)[0]) < TOL64
    for extra in (steps // 3, 1, k["exchange_steps"], 2 * k["exchange_steps"] + 1):
        lat.advance(extra)
        ref.advance(extra)
        assert np.array_equal(lat.f(), ref.f()), extra
    lat.diagnostics()


def test_span_advance_longer_than_one_launch():
    # an advance split over several launches (the exchange slots of one launch
    # cover steps_per_launch steps) equals the one-step kernel
    w = CFG_RESIDENT_Q7
    lat = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("span")
    per = lat.kernel()["steps_per_launch"]
    steps = 2 * per + 57
    say("case span %d steps over launches of %d" % (steps, per))
    rho0 = w.rho0()
    lat.init_rho(rho0).advance(steps)
    lat.diagnostics()
    ref = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("tiled").init_rho(rho0).advance(steps)
    assert np.array_equal(lat.f(), ref.f())


@pytest.mark.parametrize("prec", ["fp32", "split", "rho"])
def test_span_reduced_storage_bitwise(prec):
    n, dX, dT = 4096, 0.3, 2e-4
    tau = 1.0
    rho0 = ic(n, dX, 23)
    say("case span storage %s" % prec)
    outs = []
    for kernel in ("plain", "span"):
        lat = Lattice(n, 7, prec).set_physical(dX, dT, tau).set_kernel(kernel)
        lat.init_rho(rho0).advance(900)
        outs.append(lat.f())
    assert np.array_equal(outs[0], outs[1])


def test_resident_config_full_length():
    w = CFG_RESIDENT_Q7
    say("case %s full %d steps" % (w.name, w.steps))
    rho0 = w.rho0()
    lat = Lattice(w.n, w.q, "fp64")
    lat.set_physical(w.dX, w.dT, 0.0)
    tau = lat.coefficients()["tau"]
    lat.init_rho(rho0)
    m0, bad0 = lat.diagnostics()
    lat.advance(w.steps)
    m1, bad1 = lat.diagnostics()
    assert not bad0 and not bad1
    assert abs(m1 - m0) < 1e-11 * np.abs(rho0).sum()
    ref = oracle.solve_periodic(w.q, rho0, w.dX, w.dT, tau, w.steps)
    err = rel(lat.rho(), ref)
    say("full-length rel err vs oracle %.3e" % err)
    assert err < 1e-10


def test_large_config_sampled_sites():
    # D1Q7, N = 2^24, dT = 2e-8, tau = 1, 10^3 steps, tiled kernel: sampled sites
    # checked against the oracle on the light cone of each site (a periodic
    # window of 2*3*steps + 1 sites or more gives the centre site exactly).
    w = CFG_LARGE_Q7
    say("case %s" % w.name)
    rho0 = w.rho0()
    lat = Lattice(w.n, w.q, "fp64")
    lat.set_physical(w.dX, w.dT, 0.0)
    tau = lat.coefficients()["tau"]
    assert tau == 1.0
    lat.set_kernel("tiled")
    lat.init_rho(rho0)
    m0, _ = lat.diagnostics()
    lat.advance(w.steps)
    m1, bad = lat.diagnostics()
    rho = lat.rho()
    assert not bad
    assert abs(m1 - m0) < 1e-12 * np.abs(rho0).sum()
    # the benchmark's launch: one kslb_solve (init and readout fused into the
    # first and last tiled launches) gives the same densities bit for bit
    import torch
    fused = lat.solve(torch.tensor(rho0, device="cuda"), w.steps).cpu().numpy()
    assert np.array_equal(fused, rho)
    half = 3 * w.steps + 8
    rng = np.random.default_rng(0)
    sites = [0, 1, w.n - 1, w.n // 2] + list(rng.integers(0, w.n, 4))
    for j in sites:
        idx = (np.arange(j - half, j + half + 1)) % w.n
        r = oracle.solve_periodic(w.q, rho0[idx], w.dX, w.dT, tau, w.steps)
        ref = r[half]
        assert abs(rho[j] - ref) <= TOL64 * np.max(np.abs(r)), (j, rho[j], ref)


def test_plain_and_tiled_agree_at_large_size():
    w = CFG_LARGE_Q7
    say("case large plain vs tiled 50 steps")
    rho0 = w.rho0()
    a = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("plain")
    b = Lattice(w.n, w.q, "fp64").set_physical(w.dX, w.dT, 0.0).set_kernel("tiled")
    a.init_rho(rho0).advance(50)
    b.init_rho(rho0).advance(50)
    import torch
    assert torch.equal(a.read_rho(), b.read_rho())
    assert torch.equal(a.save_state(), b.save_state())


# measured on MI355X: split 1.8e-10 / 2.6e-10, fp32 6.3e-7 / 8.8e-7 at 1000 / 2000 steps
@pytest.mark.parametrize("prec,bound", [("split", 2e-9), ("fp32", 3e-6)])
def test_reduced_precision_error(prec, bound):
    w = CFG_RESIDENT_Q7
    rho0 = w.rho0()
    tau = oracle.tau_fit(7, w.dX, w.dT)
    for steps in (1000, 2000):
        lat = Lattice(w.n, w.q, prec).set_physical(w.dX, w.dT, 0.0)
        lat.init_rho(rho0).advance(steps)
        err = rel(lat.rho(), oracle.solve_periodic(7, rho0, w.dX, w.dT, tau, steps))
        say("%s error vs FP64 oracle at %d steps: %.3e" % (prec, steps, err))
        assert err < bound


def _fma64(a, b, c):
    """Fused multiply-add in double, correctly rounded (exact rational arithmetic)."""
    from fractions import Fraction
    return float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def _round_f32(x):
    """Round an exact rational to the nearest float32, ties to even."""
    from fractions import Fraction
    c0 = np.float32(float(x))                 # within one float32 ulp of the answer
    cands = [c0, np.nextafter(c0, np.float32(np.inf)), np.nextafter(c0, np.float32(-np.inf))]
    key = lambda c: (abs(Fraction(float(c)) - x), int(np.array(c, dtype=np.float32).view(np.uint32)) & 1)
    return min(cands, key=key)


def _fmaf(a, b, c):
    from fractions import Fraction
    return _round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_fp32_step_keeps_density_and_rho2_in_double():
    # One step of the FP32 storage mode against a numpy emulation of its
    # stated arithmetic: populations widened to double, the density summed in
    # double in the kernel's fixed pairwise order, rho^2 and the equilibrium in
    # double (fused multiply-adds, correctly rounded), then the relaxation
    # (1 - omega) g + feq as one single-precision fused multiply-add.  Every
    # stored value must match bitwise.  The same step evaluated entirely in
    # float32 is further from the exact FP64 step (the oracle's collision).
    say("case fp32 step emulation")
    q, n, dX, dT, tau = 7, 301, 0.2, 1e-4, 1.3
    c = np.array([0, 1, -1, 2, -2, 3, -3])
    coef = oracle.coefficients(q, dX, dT, tau)
    rng = np.random.default_rng(42)
    f0 = oracle.init(q, coef, 1.0 + 0.3 * random_modes_ic(n, n * dX, seed=6))
    S = (f0 + 1e-2 * rng.standard_normal(f0.shape)).astype(np.float32).astype(np.float64)
    lat = make(q, n, "fp32", "plain", dX, dT, tau).write_f(S, step=0)
    assert np.array_equal(lat.f(), S)
    lat.advance(1)
    got = lat.f()
    cf = lat.coefficients()
    A, B, om = cf["omega"] * cf["E"], cf["omega"] * cf["G"], cf["omega"]
    a1mw_f = np.float32(1.0 - om)
    g = np.stack([np.roll(S[i], int(c[i])) for i in range(q)])      # streamed, widened floats
    want = np.empty_like(S)
    for j in range(n):
        x = g[:, j]
        rho = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + x[6])
        r2 = rho * rho
        eq = np.empty(q)
        eq[0] = A[0] * rho
        for ip, im in ((1, 2), (3, 4), (5, 6)):
            a = A[ip] * rho
            eq[ip] = _fma64(B[ip], r2, a) if ip < 5 else a
            eq[im] = _fma64(B[im], r2, a) if im < 5 else a
        for i in range(q):
            want[i, j] = float(_fmaf(a1mw_f, np.float32(x[i]), np.float32(eq[i])))
    mism = int(np.sum(got != want))
    say("fp32 step: %d of %d stored values differ from the emulation" % (mism, want.size))
    assert mism == 0
    # the same step in float32 throughout (density, rho^2, equilibrium, relaxation)
    g32 = g.astype(np.float32)
    rho32 = ((g32[0] + g32[1]) + (g32[2] + g32[3])) + ((g32[4] + g32[5]) + g32[6])
    r232 = rho32 * rho32
    pure = np.float32(1.0 - om) * g32 + (A.astype(np.float32)[:, None] * rho32 + B.astype(np.float32)[:, None] * r232)
    exact = oracle.collide(q, coef, tau, g)
    e_lib, e_pure = float(np.max(np.abs(got - exact))), float(np.max(np.abs(pure - exact)))
    say("one fp32 step: max error vs the exact FP64 step %.3e (library) vs %.3e (all float32)" % (e_lib, e_pure))
    assert e_lib < e_pure
    # rounding feq to single, then the single-precision fused step: at most about one ulp
    assert e_lib <= 1.5 * float(np.spacing(np.float32(np.max(np.abs(exact)))))


def test_ensemble_matches_oracle_and_single_lattices():
    say("case ensemble ragged")
    sizes = [1, 2, 3, 64, 500, 777, 1024, 2049, 4096, 5000, 9999, 20000]
    steps = [5, 9, 0, 1, 17, 64, 100, 333, 250, 16, 170, 50]
    dX, dT = math.pi / 16, 1e-4
    ens = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 0.0)
    tau = ens.tau
    rho0s = [random_modes_ic(n, n * dX, seed=1000 + i, n_modes=min(16, max(1, n // 2))) for i, n in enumerate(sizes)]
    for i, r in enumerate(rho0s):
        ens.init_rho(i, r)
    ens.advance(steps)
    for i, n in enumerate(sizes):
        got = ens.rho(i)
        ref = oracle.solve_periodic(7, rho0s[i], dX, dT, tau, steps[i])
        assert rel(got, ref) < TOL64, i
        lat = Lattice(n, 7, "fp64").set_physical(dX, dT, 0.0).set_kernel("plain")
        lat.init_rho(rho0s[i]).advance(steps[i])
        assert np.array_equal(got, lat.rho()), i
        assert ens.status(i) == (steps[i], False)


def test_ensemble_graph_replays_match_eager_launches():
    # steady-state chunk pairs replayed from a captured graph, several advance
    # calls with host synchronisation and eager work in between, each checked
    # against the launch-per-chunk path
    import torch
    say("case ensemble graphs")
    sizes = [700, 2500, 5000, 9000, 64]
    dX, dT = 0.2, 1e-4
    rho0s = [ic(n, dX, 70 + i) for i, n in enumerate(sizes)]
    a = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 1.1).set_tiling(8, 16, 16).set_graphs(True)
    b = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 1.1).set_tiling(8, 16, 16).set_graphs(False)
    for e in (a, b):
        for i, r in enumerate(rho0s):
            e.init_rho(i, r)
    # chunk pairs: 6 replays (recorded), 2 (launched directly), 4 (recorded),
    # then 2 twice (the same pair recurs: recorded on the second call)
    for rnd, steps in enumerate(([200] * 5, [160, 96, 300, 0, 64], [128] * 5, [64] * 5, [64] * 5)):
        a.advance(steps)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        b.advance(steps)
        for i in range(len(sizes)):
            assert np.array_equal(a.rho(i), b.rho(i)), (rnd, i)
            assert a.status(i)[0] == b.status(i)[0]


@pytest.mark.parametrize("q,n,prec,kernel,steps_per_launch,steps", [
    (7, 12345, "fp64", "tiled", 0, 1), (7, 12345, "fp64", "tiled", 0, 80), (7, 12345, "fp64", "tiled", 0, 81),
    (7, 12345, "fp64", "tiled", 0, 250), (7, 70001, "fp64", "tiled", 7, 30), (5, 7001, "fp64", "tiled", 0, 150),
    (7, 9000, "fp32", "tiled", 0, 100), (5, 9000, "split", "tiled", 0, 100), (7, 9000, "rho", "tiled", 0, 100),
    (7, 4096, "fp64", "auto", 0, 100), (7, 5000, "fp64", "plain", 0, 20), (7, 12345, "fp64", "tiled", 0, 0),
    (7, 1, "fp64", "tiled", 0, 5), (7, 100, "fp64", "tiled", 0, 90), (5, 301, "rho", "tiled", 0, 200)])
def test_solve_matches_separate_calls(q, n, prec, kernel, steps_per_launch, steps):
    # kslb_solve (initialisation and readout fused into the first and last
    # tiled launches) against init_rho + advance + read_rho: density, stored
    # populations and step count bitwise (the state rows' padding sites past
    # n hold whatever the buffer held, so states are compared site by site)
    import torch
    say("case solve q=%d n=%d %s %s s=%d steps=%d" % (q, n, prec, kernel, steps_per_launch, steps))
    tau = 1.0 if prec == "rho" else 1.1
    rho0 = torch.tensor(ic(n, 0.2, 11), device="cuda")
    a = make(q, n, prec, kernel, tau=tau, steps_per_launch=steps_per_launch)
    b = make(q, n, prec, kernel, tau=tau, steps_per_launch=steps_per_launch)
    got = a.solve(rho0, steps)
    want = b.init_rho(rho0).advance(steps).read_rho()
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    state = b.f()
    assert np.array_equal(a.f(), state)
    assert a.step == b.step == steps
    # the lattice continues from the solved state like any other
    a.advance(7)
    b.advance(7)
    assert np.array_equal(a.rho(), b.rho())
    # unaligned device pointers take the unfused path, with the same result
    big = torch.empty(n + 1, dtype=torch.float64, device="cuda")
    big[1:] = rho0
    out = torch.empty(n + 1, dtype=torch.float64, device="cuda")
    c = make(q, n, prec, kernel, tau=tau, steps_per_launch=steps_per_launch)
    from paper_1711_03540_amd._lib import call
    import ctypes
    call("kslb_solve", c._h, ctypes.c_void_p(big[1:].data_ptr()), steps, ctypes.c_void_p(out[1:].data_ptr()))
    torch.cuda.synchronize()
    assert torch.equal(out[1:], want)
    assert np.array_equal(c.f(), state)
    # in place (the density written over rho0), in one launch or several
    d = make(q, n, prec, kernel, tau=tau, steps_per_launch=steps_per_launch)
    r = rho0.clone()
    assert d.solve(r, steps, out=r) is r
    torch.cuda.synchronize()
    assert torch.equal(r, want)
    assert np.array_equal(d.f(), state)
    assert d.step == steps


def test_ensemble_graphs_replaced_without_waiting():
    # every call advances a different subset of instances by five chunk pairs,
    # so each call records a new graph and retires the previous one while its
    # replays may still run; no host synchronisation between the calls
    say("case ensemble graphs replaced")
    sizes = [700, 2500, 5000, 9000, 64, 3001]
    dX, dT = 0.2, 1e-4
    rho0s = [ic(n, dX, 80 + i) for i, n in enumerate(sizes)]
    a = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 1.1).set_tiling(8, 16, 16).set_graphs(True)
    b = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 1.1).set_tiling(8, 16, 16).set_graphs(False)
    for e in (a, b):
        for i, r in enumerate(rho0s):
            e.init_rho(i, r)
    for k in range(9):
        steps = [160] * len(sizes)
        steps[k % len(sizes)] = 0
        a.advance(steps)
        b.advance(steps)
    for i in range(len(sizes)):
        assert np.array_equal(a.rho(i), b.rho(i)), i
        assert a.status(i) == b.status(i)


@pytest.mark.parametrize("q,prec", [(7, "fp64"), (5, "fp64"), (7, "split"), (5, "fp32")])
def test_ensemble_packing_and_chunking_bitwise(q, prec):
    # packed windows (several instance tiles per workgroup), one tile per
    # workgroup, 4, 8 (or, FP64, 12) sites per lane and any chunk length give
    # the same bits
    say("case ensemble packing q=%d %s" % (q, prec))
    sizes = [5, 100, 333, 640, 1500, 2048, 3001, 7777]
    steps = [40, 77, 64, 5, 100, 31, 64, 90]
    dX, dT = 0.2, 1e-4
    rho0s = [ic(n, dX, 50 + i) for i, n in enumerate(sizes)]
    outs = []
    tilings = [(8, 16, 32), (8, 1, 32), (4, 16, 16), (8, 256, 7), (8, 3, 40)]
    if prec == "fp64":
        tilings += [(12, 16, 32), (12, 1, 41), (12, 5, 96)]
    if prec == "fp32":
        tilings += [(10, 16, 32), (10, 1, 41), (10, 5, 80)]
    default = Ensemble(sizes, q, prec).tiling()
    assert default == {"sites_per_lane": {"fp64": 12, "fp32": 10}.get(prec, 8), "max_segments": 16,
                       "steps_per_chunk": {"fp32": 48, "split": 40}.get(prec, 64)}
    for B, segs, chunk in tilings:
        ens = Ensemble(sizes, q, prec).set_physical(dX, dT, 1.1).set_tiling(B, segs, chunk)
        assert ens.tiling() == {"sites_per_lane": B, "max_segments": segs, "steps_per_chunk": chunk}
        for i, r in enumerate(rho0s):
            ens.init_rho(i, r)
        ens.advance(steps)
        outs.append([ens.rho(i) for i in range(len(sizes))])
    for o in outs[1:]:
        for i in range(len(sizes)):
            assert np.array_equal(o[i], outs[0][i]), i
    if prec == "fp64":
        for i, n in enumerate(sizes):
            ref = oracle.solve_periodic(q, rho0s[i], dX, dT, 1.1, steps[i])
            assert rel(outs[0][i], ref) < TOL64


# (sites, scheme, storage, coefficient set, steps) of a mixed ensemble; the
# sets are (dX, dT, tau), tau = 0 taking the fit; the rho-only storage needs tau = 1
MIXED_SETS = {"a": (0.2, 1e-4, 1.1), "b": (math.pi / 16, 1e-4, 0.0), "c": (0.3, 2e-4, 1.0)}
MIXED = [(64, 7, "fp64", "a", 100), (300, 5, "fp64", "a", 77), (1000, 7, "fp32", "b", 64),
         (2500, 5, "split", "a", 130), (777, 7, "rho", "c", 90), (4096, 7, "fp64", "b", 200),
         (5000, 5, "rho", "c", 33), (128, 5, "fp32", "c", 64), (3000, 7, "split", "c", 150),
         (640, 7, "fp64", "c", 0), (2049, 7, "fp64", "a", 257)]


def mixed_ensemble(graphs):
    from paper_1711_03540_amd import KslbError
    sizes = [m[0] for m in MIXED]
    ens = Ensemble(sizes, [m[1] for m in MIXED], [m[2] for m in MIXED]).set_tiling(8, 16, 8).set_graphs(graphs)
    with pytest.raises(KslbError):                 # tau 1.1 for every instance: the rho-only ones refuse
        ens.set_physical(*MIXED_SETS["a"])
    with pytest.raises(KslbError):                 # so nothing was assigned
        ens.tau_of(0)
    for i, m in enumerate(MIXED):
        ens.set_physical(*MIXED_SETS[m[3]], idx=i)
    for i, m in enumerate(MIXED):
        ens.init_rho(i, ic(m[0], MIXED_SETS[m[3]][0], 90 + i))
    return ens


def test_mixed_ensemble_matches_single_lattices():
    # one ensemble holding both schemes, all four storage modes and three
    # coefficient sets: every instance equals the same solve on a lattice of
    # its own (bitwise) and, in FP64, the oracle; graph replay and
    # launch-per-chunk agree bitwise
    say("case ensemble mixed schemes, storage and coefficients")
    a, b = mixed_ensemble(True), mixed_ensemble(False)
    steps = [m[4] for m in MIXED]
    a.advance(steps)
    b.advance(steps)
    for i, (n, q, prec, cs, st) in enumerate(MIXED):
        dX, dT, tau = MIXED_SETS[cs]
        got = a.rho(i)
        assert np.array_equal(got, b.rho(i)), i
        lat = Lattice(n, q, prec).set_physical(dX, dT, tau).set_kernel("plain")
        assert a.tau_of(i) == lat.coefficients()["tau"], i
        lat.init_rho(ic(n, dX, 90 + i)).advance(st)
        assert np.array_equal(got, lat.rho()), i
        assert a.status(i) == (st, False), i
        if prec == "fp64":
            ref = oracle.solve_periodic(q, ic(n, dX, 90 + i), dX, dT, a.tau_of(i), st)
            assert rel(got, ref) < TOL64, i
    # new coefficients for one instance apply from its next step, its state kept
    a.set_physical(*MIXED_SETS["a"], idx=9)
    a.advance([0] * 9 + [40, 0])
    rho0 = ic(640, MIXED_SETS["c"][0], 99)
    # the stored state is feq_c(rho0); one oracle step with set c (tau = 1:
    # its collision leaves an equilibrium as it is) streams it, 39 with set a follow
    coef_c = oracle.coefficients(7, *MIXED_SETS["c"])
    g1 = oracle.advance(7, coef_c, 1.0, oracle.init(7, coef_c, rho0), 1)
    g40 = oracle.advance(7, oracle.coefficients(7, *MIXED_SETS["a"]), MIXED_SETS["a"][2], g1, 39)
    assert rel(a.rho(9), oracle.density(g40)) < TOL64
    assert a.status(9) == (40, False)


def test_ensemble_per_instance_errors():
    from paper_1711_03540_amd import KslbError
    say("case ensemble per-instance errors")
    ens = Ensemble([64, 128, 256], [5, 7, 7], ["fp64", "rho", "split"])
    with pytest.raises(KslbError):
        ens.set_physical(0.3, 2e-4, 1.1, idx=3)            # no such instance
    with pytest.raises(KslbError):
        ens.set_physical(0.3, 2e-4, 1.1, idx=1)            # rho-only storage needs tau = 1
    with pytest.raises(KslbError):
        ens.tau_of(1)                                      # nothing assigned yet
    with pytest.raises(KslbError):
        ens.init_rho(0, np.ones(64))                       # coefficients first
    with pytest.raises(KslbError):
        ens.set_tiling(16, 0, 0)                           # 16 sites per lane: rho-only throughout
    with pytest.raises(KslbError):
        ens.set_tiling(12, 0, 0)                           # 12 sites per lane: FP64 throughout
    ens.set_physical(0.3, 2e-4, 1.0)                       # every instance, one set per scheme
    assert ens.tau_of(0) == ens.tau_of(1) == ens.tau_of(2) == 1.0
    ens.set_physical(0.3, 2e-4, 1.1, idx=2)
    assert ens.tau_of(2) == 1.1 and ens.tau_of(1) == 1.0
    import torch
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    for i, n in enumerate((64, 128, 256)):
        ens.init_rho(i, ic(n, 0.3, 3 + i))
    with pytest.raises(KslbError):
        ens.renormalize([1], [2], 1e-6, acc)               # not FP64, and sizes differ
    ens.advance([10, 0, 5])
    assert [ens.status(i)[0] for i in range(3)] == [10, 0, 5]


def test_ensemble_init_all_equals_per_instance_init():
    # one launch per (scheme, storage) gives the states per-instance inits give,
    # from device and from host densities, after a resize too; the batched
    # readout returns the per-instance densities
    import torch
    say("case ensemble init all")
    sizes = [m[0] for m in MIXED]
    qs, precs = [m[1] for m in MIXED], [m[2] for m in MIXED]

    def make_one():
        ens = Ensemble(sizes, qs, precs)
        for i, m in enumerate(MIXED):
            ens.set_physical(*MIXED_SETS[m[3]], idx=i)
        return ens
    a, b, c = make_one(), make_one(), make_one()
    a.resize(3, 1234)
    b.resize(3, 1234)
    c.resize(3, 1234)
    rhos = [ic(int(a.n[i]), MIXED_SETS[m[3]][0], 40 + i) for i, m in enumerate(MIXED)]
    for i, r in enumerate(rhos):
        a.init_rho(i, r)
    b.init_rho_all(torch.tensor(np.concatenate(rhos), device="cuda"))
    c.init_rho_all(np.concatenate(rhos))
    steps = [m[4] for m in MIXED]
    for e in (a, b, c):
        e.advance(steps)
    for i in range(len(MIXED)):
        ra = a.rho(i)
        assert np.array_equal(ra, b.rho(i)) and np.array_equal(ra, c.rho(i)), i
        assert b.status(i) == (steps[i], False)
    # batched readout, to the device and to the host: the per-instance densities back to back
    want = np.concatenate([a.rho(i) for i in range(len(MIXED))])
    dev = torch.full((want.size + 5,), -1.0, dtype=torch.float64, device="cuda")
    b.rho_all(dev)
    assert np.array_equal(dev[: want.size].cpu().numpy(), want) and float(dev[-1]) == -1.0
    assert np.array_equal(c.rho_all(), want)


def test_renormalize_pairs_of_both_schemes_in_one_call():
    # pairs given D1Q7 first: results land in each pair's own accumulator slot
    import torch
    say("case renormalise mixed schemes")
    n, dX, dT, tau, steps, delta = 200, 0.2, 1e-4, 1.1, 150, 1e-7
    base = [1.0 + random_modes_ic(n, n * dX, seed=s, amplitude=0.3) for s in (1, 2)]
    pert = [r + 1e-6 * random_modes_ic(n, n * dX, seed=s, amplitude=1.0) for r, s in zip(base, (3, 4))]
    mixed = Ensemble([n] * 4, [7, 7, 5, 5], "fp64").set_physical(dX, dT, tau)
    for i, r in enumerate((base[0], pert[0], base[1], pert[1])):
        mixed.init_rho(i, r)
    mixed.advance(steps)
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    mixed.renormalize([0, 2], [1, 3], delta, acc)
    for q, (r, p), slot in ((7, (base[0], pert[0]), 0), (5, (base[1], pert[1]), 1)):
        one = Ensemble([n, n], q, "fp64").set_physical(dX, dT, tau).init_rho(0, r).init_rho(1, p).advance(steps)
        acc1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        one.renormalize([0], [1], delta, acc1)
        assert float(acc.cpu()[slot]) == float(acc1.cpu()[0]), q
        assert np.array_equal(mixed.rho(2 * slot + 1), one.rho(1)), q


@pytest.mark.parametrize("q", [5, 7])
def test_rho_only_ensemble_16_sites_per_lane(q):
    # the rho-only storage (tau = 1) in ensembles, 16 and 8 sites per lane:
    # each instance equals a rho-only lattice on the plain kernel bitwise
    say("case rho-only ensemble q=%d" % q)
    sizes = [1, 5, 100, 777, 2048, 3001, 9000]
    steps = [7, 64, 90, 33, 128, 16, 200]
    dX, dT = 0.3, 2e-4
    rho0s = [ic(n, dX, 60 + i) for i, n in enumerate(sizes)]
    outs = []
    for B, segs, chunk in ((16, 16, 32), (16, 1, 80), (8, 16, 32)):
        ens = Ensemble(sizes, q, "rho").set_physical(dX, dT, 1.0).set_tiling(B, segs, chunk)
        ens.init_rho_all(np.concatenate(rho0s))
        ens.advance(steps)
        outs.append([ens.rho(i) for i in range(len(sizes))])
    for i, n in enumerate(sizes):
        lat = Lattice(n, q, "rho").set_physical(dX, dT, 1.0).set_kernel("plain")
        lat.init_rho(rho0s[i]).advance(steps[i])
        want = lat.rho()
        for o in outs:
            assert np.array_equal(o[i], want), (i, n)


def test_ensemble_instances_bound_to_caller_memory():
    # instances rebound to device memory outside the ensemble's buffer (one
    # block allocated before it, one after, so offsets from its base have
    # either sign) compute bitwise what single lattices compute; rebinding to
    # another size drops the state; bad memory is refused
    import torch

    from paper_1711_03540_amd import KslbError
    from paper_1711_03540_amd.serve import instance_bytes
    say("case ensemble bind")
    dX, dT = math.pi / 16, 1e-4
    shapes = [(5000, 7, "fp64"), (777, 5, "fp32"), (3000, 7, "split")]
    before = [torch.empty(instance_bytes(n, q, p), dtype=torch.uint8, device="cuda") for n, q, p in shapes]
    ens = Ensemble([1, 1, 1], [q for _, q, _ in shapes], [p for _, _, p in shapes]).set_physical(dX, dT, 0.0)
    after = [torch.empty(instance_bytes(n, q, p), dtype=torch.uint8, device="cuda") for n, q, p in shapes]
    mem = [before[0], after[1], before[2]]
    for k, (n, q, p) in enumerate(shapes):
        ens.bind(k, n, mem[k].data_ptr(), mem[k].numel())
        ens.init_rho(k, ic(n, dX, 40 + k, 0.1))
    ens.advance([300, 500, 200])
    for k, (n, q, p) in enumerate(shapes):
        lat = Lattice(n, q, p).set_physical(dX, dT, 0.0).set_kernel("plain").init_rho(ic(n, dX, 40 + k, 0.1))
        lat.advance([300, 500, 200][k])
        assert np.array_equal(ens.rho(k), lat.rho()), k
    # rebind instance 0 to a smaller lattice in the other block
    ens.bind(0, 1234, after[0].data_ptr(), after[0].numel())
    with pytest.raises(KslbError):
        ens.advance([10, 0, 0])                              # no state until init
    ens.init_rho(0, ic(1234, dX, 9, 0.1)).advance([64, 0, 0])
    lat = Lattice(1234, 7, "fp64").set_physical(dX, dT, 0.0).set_kernel("plain").init_rho(ic(1234, dX, 9, 0.1))
    assert np.array_equal(ens.rho(0), lat.advance(64).rho())
    with pytest.raises(KslbError) as e:
        ens.bind(1, 777, after[1].data_ptr() + 8, after[1].numel() - 8)
    assert e.value.status == -1                              # EINVAL: not 256-byte aligned
    with pytest.raises(KslbError) as e:
        ens.bind(1, 5000, after[1].data_ptr(), after[1].numel())
    assert e.value.status == -2                              # ENOMEM: the block is too small


def test_served_results_equal_solo_solves():
    # continuous batching: requests of both schemes and precisions arrive while
    # others run; each result equals the same solve run alone (bitwise)
    say("case serving alone vs mix")
    import torch
    from paper_1711_03540_amd.inputs import request_stream
    from paper_1711_03540_amd.serve import SolveServer
    dX, dT = math.pi / 16, 1e-4
    reqs = request_stream(40, seed=17, rate=20000.0, n_lo=64, n_hi=6000, steps_lo=50, steps_hi=1500)
    init = [torch.tensor(random_modes_ic(r.n, r.n * dX, seed=r.seed % 1000003, n_modes=min(16, r.n // 2)),
                         device="cuda") for r in reqs]
    # one request blows up (density ~1e300 overflows): it must be flagged and
    # must not disturb the requests sharing its launches
    bad = 7
    init[bad] = init[bad] * 1e300
    for fp32_storage in ("fp32", "split"):
        # a budget of 1 MiB holds only a few of these requests at once, so
        # most wait for memory and are admitted while others run
        srv = SolveServer(dX, dT, budget_bytes=1 << 20, slots=64, chunk=24, round_steps=100,
                          fp32_storage=fp32_storage)
        stats = srv.serve(reqs, init, realtime=True)
        summ = stats.summary()
        say("serve summary (fp32 requests in %s storage)" % fp32_storage, summ)
        assert summ["completed"] == len(reqs)
        assert summ["p99_ms"] >= summ["p50_ms"] > 0
        assert summ["arena_peak_bytes"] <= 1 << 20 and summ["queue_depth_max"] > 0 and summ["active_max"] >= 2
        assert srv.arena.used == 0 and srv.arena.largest_free() == srv.arena.size   # every block returned
        assert stats.results[bad].finite is False
        for i, r in enumerate(reqs):
            if i == bad:
                continue
            assert stats.results[i].finite
            lat = Lattice(r.n, r.q, srv.storage[r.precision]).set_physical(dX, dT, 0.0).set_kernel("plain")
            lat.init_rho(init[i]).advance(r.steps)
            assert torch.equal(stats.results[i].rho, lat.read_rho()), (fp32_storage, i)


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("dX", [0.2, 0.1])
def test_fixed_ends_table3_parity(q, dX):
    # the Table 3 travelling wave with fixed ends: GPU (plain and
    # multi-workgroup kernels) against the oracle's fixed-end solve
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    say("case fixed ends q=%d dX=%g" % (q, dX))
    dT = dX ** 4 / 100
    tau = 1.0 if q == 5 else 1.3
    steps = 3000
    n = table3_sites(dX)
    X = np.arange(n) * dX
    lo, hi = table3_ends()
    ref = oracle.solve_tanh_fixed(q, dX, dT, tau, steps)
    outs = []
    for kernel, spl in (("plain", 0), ("span", 0), ("span", 7)):
        lat = Lattice(n, q, "fp64").set_physical(dX, dT, tau).set_kernel(kernel, spl).set_fixed_ends(lo, hi)
        say("  kernel %s: %s" % (kernel, lat.kernel()))
        lat.init_rho(table3_profile(X, 0.0)).advance(steps)
        rho = lat.rho()
        assert rel(rho, ref) < TOL64, (kernel, spl)
        assert rho[0] == pytest.approx(lo, abs=1e-14) and rho[-1] == pytest.approx(hi, abs=1e-14)
        outs.append(lat.f())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    G = oracle.global_error(ref, oracle.tanh_solution(X, steps * dT))
    assert G < 1e-3


@pytest.mark.parametrize("kernel", ["plain", "span"])
def test_solve_with_fixed_ends(kernel):
    # kslb_solve on the Table 3 problem (fixed ends run unfused): the result of
    # init_rho + advance + read_rho bitwise, also written over its input
    import torch
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    say("case solve fixed ends %s" % kernel)
    dX, q = 0.1, 7
    dT, tau, steps = dX ** 4 / 100, 1.3, 700
    n = table3_sites(dX)
    lo, hi = table3_ends()
    rho0 = torch.tensor(table3_profile(np.arange(n) * dX, 0.0), device="cuda")
    mk = lambda: Lattice(n, q, "fp64").set_physical(dX, dT, tau).set_kernel(kernel).set_fixed_ends(lo, hi)
    a, b, c = mk(), mk(), mk()
    got = a.solve(rho0, steps)
    want = b.init_rho(rho0).advance(steps).read_rho()
    r = rho0.clone()
    c.solve(r, steps, out=r)
    torch.cuda.synchronize()
    assert torch.equal(got, want) and torch.equal(r, want)
    assert np.array_equal(a.f(), b.f()) and a.step == b.step == c.step == steps
    assert float(got[0]) == pytest.approx(lo, abs=1e-14) and float(got[-1]) == pytest.approx(hi, abs=1e-14)


@pytest.mark.parametrize("prec", ["fp32", "split", "rho"])
def test_fixed_ends_reduced_storage_bitwise(prec):
    # the fixed-end boundary in the reduced storage modes: the plain and
    # multi-workgroup kernels give the same bits
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    say("case fixed ends %s" % prec)
    q, dX, dT, tau, steps = 7, 0.1, 2e-6, 1.0, 1500
    n = table3_sites(dX)
    X = np.arange(n) * dX
    lo, hi = table3_ends()
    outs = []
    for kernel in ("plain", "span"):
        lat = Lattice(n, q, prec).set_physical(dX, dT, tau).set_kernel(kernel).set_fixed_ends(lo, hi)
        lat.init_rho(table3_profile(X, 0.0)).advance(steps)
        outs.append(lat.rho())
    assert np.array_equal(outs[0], outs[1])
    assert np.all(np.isfinite(outs[0]))


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("n", [3, 256, 1000, 4096, 70001])
def test_rho_only_mode_at_tau1(q, n):
    # tau = 1: the rho-only storage evolves exactly as FP64 on every kernel
    # class: its populations feq(rho) are FP64's post-collision state bit for
    # bit.  The density readouts differ by rounding only: FP64 sums its stored
    # populations, the rho-only state holds rho itself.
    say("case rho-only q=%d n=%d" % (q, n))
    dX, dT = 0.3, 2e-4
    rho0 = ic(n, dX, 31)
    ref = make(q, n, "fp64", "plain", dX, dT, 1.0).init_rho(rho0).advance(500)
    rr = ref.rho()
    assert rel(rr, oracle.solve_periodic(q, rho0, dX, dT, 1.0, 500)) < TOL64
    for kernel in ("plain", "tiled", "resident", "span"):
        lat = Lattice(n, q, "rho").set_physical(dX, dT, 1.0)
        try:
            lat.set_kernel(kernel)
        except Exception:
            continue
        lat.init_rho(rho0).advance(500)
        assert np.array_equal(lat.f(), ref.f()), kernel
        assert rel(lat.rho(), rr) < 1e-15, kernel
    with pytest.raises(Exception):
        Lattice(n, q, "rho").set_physical(dX, dT, 1.1)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split"])
def test_checkpoint_resume_bitwise(prec):
    say("case resume %s" % prec)
    n = 3000
    rho0 = ic(n, 0.2, 12)
    a = make(7, n, prec).init_rho(rho0).advance(400)
    b = make(7, n, prec).init_rho(rho0).advance(200)
    blob = b.save_state()
    c = make(7, n, prec).load_state(blob, 200).advance(200)
    assert c.step == 400
    assert np.array_equal(a.f(), c.f())


def test_pre_and_post_collision_populations():
    say("case f conventions")
    q, n, dX, dT, tau = 7, 300, 0.2, 1e-4, 1.3
    coef = oracle.coefficients(q, dX, dT, tau)
    rho0 = ic(n, dX, 21)
    lat = make(q, n, "fp64", "plain", dX, dT, tau).init_rho(rho0)
    f = oracle.init(q, coef, rho0)
    for s in range(3):
        assert rel(lat.f(pre_collision=False), oracle.collide(q, coef, tau, f)) < TOL64
        nxt = oracle.advance(q, coef, tau, f, 1)
        assert rel(lat.f(pre_collision=True), nxt) < TOL64
        lat.advance(1)
        f = nxt


def test_write_f_roundtrip_and_nonfinite_flag():
    say("case write_f / nonfinite")
    n = 500
    lat = make(7, n).init_rho(ic(n, 0.2, 2)).advance(10)
    f = lat.f()
    lat2 = make(7, n).write_f(f, step=10)
    assert np.array_equal(lat2.f(), f)
    assert lat2.step == 10
    mass, bad = lat2.diagnostics()
    assert not bad and abs(mass - lat.rho().sum()) < 1e-12 * n
    f[3, 17] = np.nan
    lat2.write_f(f, step=10)
    assert lat2.diagnostics()[1]


@pytest.mark.parametrize("prec", ["fp32", "split", "rho"])
def test_populations_io_reduced_storage(prec):
    # write_f / read_f through the reduced storage modes: FP32 rounds each
    # population to single; split keeps rho in double and rounds only the
    # non-equilibrium part; the rho-only state (tau = 1) keeps rho, and at
    # tau = 1 the stored populations are exactly feq(rho)
    say("case populations io %s" % prec)
    n, dX, dT, tau = 400, 0.3, 2e-4, 1.0
    ref = make(7, n, "fp64", "plain", dX, dT, tau).init_rho(ic(n, dX, 8)).advance(30)
    f = ref.f()
    lat = make(7, n, prec, "plain", dX, dT, tau).write_f(f, step=30)
    g = lat.f()
    assert lat.step == 30
    if prec == "fp32":
        assert np.array_equal(g, f.astype(np.float32).astype(np.float64))
    else:
        assert np.max(np.abs(g - f)) <= 1e-7 * np.max(np.abs(f))
        assert np.max(np.abs(lat.rho() - ref.rho())) <= 1e-14 * np.max(np.abs(ref.rho()))
    # and the state advances as the FP64 one does, to the storage's precision
    lat.advance(20)
    ref.advance(20)
    tol = {"fp32": 1e-5, "split": 1e-9, "rho": 1e-13}[prec]
    assert rel(lat.rho(), ref.rho()) < tol


def test_zero_steps_and_errors():
    say("case errors")
    from paper_1711_03540_amd import KslbError
    lat = Lattice(100, 7, "fp64")
    with pytest.raises(KslbError):
        lat.advance(1)          # coefficients and state not set
    lat.set_physical(0.2, 1e-4, 1.1)
    with pytest.raises(KslbError):
        lat.advance(1)          # no state yet
    lat.init_rho(ic(100, 0.2, 1))
    lat.advance(0)
    assert lat.step == 0
    with pytest.raises(KslbError):
        lat.advance(-1)
    with pytest.raises(KslbError):
        lat.set_kernel("tiled", 100000)
    with pytest.raises(KslbError):
        Lattice(100, 7).set_physical(0.2, 1e-3, 1.0)   # refused by the stability guard


def test_resolved_kernel_and_launch_shape():
    say("case resolved kernel")
    # AUTO: a few thousand sites run on SPAN, larger periodic lattices on TILED
    k = make(7, 4096).kernel()
    assert k["kernel"] == "span" and k["steps_per_launch"] % k["exchange_steps"] == 0
    assert k["exchange_steps"] >= 1 and k["workgroups"] >= 2 and k["lanes"] == 64
    n = 100_000
    for prec, sites, s_default in (("fp64", 12, 80), ("rho", 32, 64), ("fp32", 10, 48), ("split", 8, 32)):
        lat = Lattice(n, 7, prec).set_physical(0.3, 2e-4, 1.0)
        k = lat.kernel()
        s = k["steps_per_launch"]
        assert k["kernel"] == "tiled" and s == s_default
        assert k["workgroups"] == -(-n // (256 * sites - 2 * 3 * s))
        # a tiled advance of s + 1 steps is two launches: same result as s + 1 plain steps
        lat.init_rho(ic(n, 0.3, 5)).advance(s + 1)
        ref = Lattice(n, 7, prec).set_physical(0.3, 2e-4, 1.0).set_kernel("plain")
        ref.init_rho(ic(n, 0.3, 5)).advance(s + 1)
        assert np.array_equal(lat.f(), ref.f())
    k = make(5, 1000, kernel="plain").kernel()
    assert k == {"kernel": "plain", "steps_per_launch": 1, "exchange_steps": 0, "workgroups": 4, "lanes": 256}
    k = make(7, 4096, kernel="resident").kernel()
    assert k["kernel"] == "resident" and k["workgroups"] == 1
    k = make(7, 4096, kernel="tiled", steps_per_launch=24).kernel()
    assert k["steps_per_launch"] == 24 and k["workgroups"] == -(-4096 // (3072 - 144))
    # fixed ends beyond the SPAN size run on PLAIN
    lat = make(7, 70001)
    lat.set_fixed_ends(1.0, 2.0)
    assert lat.kernel()["kernel"] == "plain"


def test_blowup_threshold_matches_oracle():
    # the minimum stable tau of one Table 3 case (section 3's scan), found by
    # bisection on the GPU, also separates bounded from unbounded oracle runs
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    q, dX, dT, steps = 5, 0.2, 1e-3, 500
    n = table3_sites(dX)
    X = np.arange(n) * dX
    lo_end, hi_end = table3_ends()
    say("case blow-up threshold q=%d dX=%g dT=%g" % (q, dX, dT))

    def bounded(rho):
        return bool(np.all(np.isfinite(rho)) and np.max(np.abs(rho)) < 100.0)

    def gpu_stable(tau):
        lat = Lattice(n, q, "fp64").set_physical(dX, dT, tau, guard="off").set_fixed_ends(lo_end, hi_end)
        return bounded(lat.init_rho(table3_profile(X, 0.0)).advance(steps).rho())

    lo, hi = 0.92, 3.0
    assert not gpu_stable(lo) and gpu_stable(hi)
    while hi - lo > 0.01:
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if gpu_stable(mid) else (mid, hi)
    say("  GPU threshold in (%.4f, %.4f]" % (lo, hi))
    with np.errstate(all="ignore"):
        assert bounded(oracle.solve_tanh_fixed(q, dX, dT, hi + 0.01, steps))
        assert not bounded(oracle.solve_tanh_fixed(q, dX, dT, lo - 0.01, steps))


def test_ensemble_full_size_sampled():
    # the 4096-instance ensemble workload (N log-uniform in [512, 8192], 2 x 10^4
    # steps) in the benchmark's launch configuration: the smallest, median and
    # largest instances against the oracle; every instance finite and conserving
    # the sum of rho
    import torch
    from paper_1711_03540_amd.inputs import ensemble_shapes
    sizes = ensemble_shapes(4096, seed=2)
    dX, dT, steps = math.pi / 16, 1e-4, 20_000
    say("case ensemble full size: %d instances, %d sites, %d steps" % (sizes.size, int(sizes.sum()), steps))
    ens = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 0.0)
    ens.set_tiling(0, 0, 0)
    tau = ens.tau
    rho0 = [random_modes_ic(int(n), n * dX, seed=1000 + i) for i, n in enumerate(sizes)]
    ens.init_rho_all(torch.tensor(np.concatenate(rho0), device="cuda"))
    ens.advance(np.full(sizes.size, steps, dtype=np.int64))
    order = np.argsort(sizes, kind="stable")
    for i in (int(order[0]), int(order[sizes.size // 2]), int(order[-1])):
        ref = oracle.solve_periodic(7, rho0[i], dX, dT, tau, steps)
        err = rel(ens.rho(i), ref)
        say("  instance %d (N = %d): rel err vs oracle %.3e" % (i, sizes[i], err))
        assert err < 1e-10
    out = torch.empty(int(sizes.max()), dtype=torch.float64, device="cuda")
    for i, n in enumerate(sizes):
        r = ens.read_rho(i, out[: int(n)])
        s0 = float(np.sum(rho0[i]))
        assert abs(float(r.sum()) - s0) < 1e-10 * np.abs(rho0[i]).sum() + 1e-12, i
    assert not any(ens.status(i)[1] for i in range(0, sizes.size, 97))
    # every 64th instance (64 instances spread over the packing order, windows
    # and launches) equals the same lattice solved alone, bitwise
    for i in range(0, sizes.size, 64):
        lat = Lattice(int(sizes[i]), 7, "fp64").set_physical(dX, dT, 0.0).init_rho(rho0[i]).advance(steps)
        assert torch.equal(ens.read_rho(i, out[: int(sizes[i])]), lat.read_rho()), i
        lat.close()


def test_served_stream_full_size_sampled():
    # the 2000-request serving workload (D1Q5/D1Q7, N in [256, 65536], 10^3..10^5
    # steps, FP32 or FP64): all complete and finite; sampled results equal the
    # same solve run alone, and the smallest FP64 ones match the oracle
    import torch
    from paper_1711_03540_amd.inputs import request_stream
    from paper_1711_03540_amd.serve import SolveServer
    dX, dT = math.pi / 16, 1e-4
    reqs = request_stream(2000, seed=3)
    init = [torch.tensor(random_modes_ic(r.n, r.n * dX, seed=r.seed % (1 << 63)), device="cuda") for r in reqs]
    say("case served stream full size: %d requests" % len(reqs))
    srv = SolveServer(dX, dT, chunk=64, round_steps=256)     # the benchmark's configuration
    stats = srv.serve(reqs, init, realtime=False)
    assert stats.summary()["completed"] == len(reqs)
    assert all(r.finite for r in stats.results)
    # every 29th request (69 of both schemes, both precisions, all sizes and
    # admission times) equals the same solve run alone, bitwise
    for i in range(0, len(reqs), 29):
        r = reqs[i]
        lat = Lattice(r.n, r.q, srv.storage[r.precision]).set_physical(dX, dT, 0.0).set_kernel("auto")
        lat.init_rho(init[i]).advance(r.steps)
        assert torch.equal(stats.results[i].rho, lat.read_rho()), i
        lat.close()
    small = sorted((r.n * r.steps, i) for i, r in enumerate(reqs) if r.precision == "fp64")[:3]
    for _, i in small:
        r = reqs[i]
        lat = Lattice(r.n, r.q, "fp64").set_physical(dX, dT, 0.0)
        tau = lat.coefficients()["tau"]
        ref = oracle.solve_periodic(r.q, init[i].cpu().numpy(), dX, dT, tau, r.steps)
        err = rel(stats.results[i].rho.cpu().numpy(), ref)
        say("  request %d (D1Q%d, N = %d, %d steps): rel err vs oracle %.3e" % (i, r.q, r.n, r.steps, err))
        assert err < 1e-10


def test_tuner_choices_give_identical_results():
    # the autotuner only times candidates: whatever it picks computes the same bits
    from paper_1711_03540_amd import tune
    say("case autotuner")
    n, dX, dT = 1000, math.pi / 16, 1e-4
    t = tune.tune_lattice(n, 7, "fp64", steps=200, cache=None, tile_steps=(0, 32), span_steps=(0,))
    assert t["best"] in t["candidates"] and len(t["candidates"]) >= 2
    rho0 = random_modes_ic(n, n * dX, seed=1)
    lat = tune.apply_lattice(Lattice(n, 7, "fp64").set_physical(dX, dT, 0.0), t)
    lat.init_rho(rho0).advance(300)
    ref = Lattice(n, 7, "fp64").set_physical(dX, dT, 0.0).set_kernel("plain").init_rho(rho0).advance(300)
    assert np.array_equal(lat.f(), ref.f())
    sizes = [300, 700, 1500]
    e = tune.tune_ensemble(sizes, 7, "fp64", steps=64, cache=None, sites_per_lane=(8,), chunks=(16, 32),
                           segments=(1, 16))
    assert e["best"] in e["candidates"] and len(e["candidates"]) == 4
    a = tune.apply_ensemble(Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 0.0), e)
    b = Ensemble(sizes, 7, "fp64").set_physical(dX, dT, 0.0)
    for ens in (a, b):
        for i, m in enumerate(sizes):
            ens.init_rho(i, random_modes_ic(m, m * dX, seed=1000 + i))
        ens.advance([100, 100, 100])
    for i in range(len(sizes)):
        assert np.array_equal(a.rho(i), b.rho(i)), i


def test_guarded_advance_rolls_back_and_raises_tau():
    # the Table 3 case D1Q5, dX = 0.2, dT = 1e-3 at the fitted tau blows up
    # (the guard flags it); the guarded advance rolls each failing chunk back
    # to its checkpoint and reruns it with a larger tau until the run is stable
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    say("case guarded advance")
    q, dX, dT, steps = 5, 0.2, 1e-3, 500
    n = table3_sites(dX)
    X = np.arange(n) * dX
    lo, hi = table3_ends()

    def fresh():
        lat = Lattice(n, q, "fp64").set_physical(dX, dT, 0.0, guard="off").set_fixed_ends(lo, hi)
        return lat.init_rho(table3_profile(X, 0.0))
    plain = fresh().advance(steps)
    rho = plain.rho()
    assert plain.diagnostics()[1] or not np.max(np.abs(rho)) < 1e3      # unguarded: blows up
    tau0 = plain.coefficients()["tau"]
    lat = fresh().advance_guarded(steps, chunk=50, bound=1e3)
    say("  recoveries %s" % lat.recoveries)
    assert lat.recoveries and lat.step == steps
    assert lat.coefficients()["tau"] > tau0
    assert not lat.diagnostics()[1] and np.max(np.abs(lat.rho())) < 1e3
    # the rollback restores the checkpoint exactly: the same run replayed
    # without failures (the fitted tau up to the last rolled-back checkpoint,
    # the final tau after it) gives the same bits
    step0, _, tau_final = lat.recoveries[-1]
    replay = fresh().advance(step0)
    replay.set_physical(dX, dT, tau_final, guard="off").advance(steps - step0)
    assert np.array_equal(replay.f(), lat.f())


def test_span_abort_path_reports_and_recovers(monkeypatch):
    # failure path of the multi-workgroup kernel, forced from the host: every
    # launch starts with its abort word raised (KSLB_SPAN_INJECT_ABORT=1), so
    # every owner stops at its first exchange and the kernel exits normally;
    # until the state is replaced the sticky error word makes every host
    # readout, the checkpoint and the diagnostics report KSLB_EDEVICE and
    # device readouts NaN, and the abort count (never reset) records the
    # launch; once the state is replaced the lattice computes correctly again
    import torch

    from paper_1711_03540_amd import KslbError
    say("case span abort path")
    n, dX, dT = 4096, math.pi / 16, 1e-4
    rho0 = random_modes_ic(n, n * dX, seed=1)
    lat = Lattice(n, 7, "fp64").set_physical(dX, dT, 0.0).set_kernel("span")
    lat.init_rho(rho0)
    assert lat.diagnostics()[1] is False
    assert lat.aborted_launches() == 0
    lat.advance(100)
    assert lat.aborted_launches() == 0
    monkeypatch.setenv("KSLB_SPAN_INJECT_ABORT", "1")
    lat.advance(200)                                   # several exchanges
    monkeypatch.delenv("KSLB_SPAN_INJECT_ABORT")
    for read in (lat.diagnostics, lat.rho, lat.f, lambda: lat.f(pre_collision=True), lat.save_state):
        with pytest.raises(KslbError) as e:
            read()
        assert e.value.status == -3                    # KSLB_EDEVICE, every time (sticky)
    dev = lat.read_rho()                               # device output: enqueued, poisoned
    assert bool(torch.isnan(dev).all())
    lat.advance(50)                                    # later launches leave the error in place
    with pytest.raises(KslbError):
        lat.rho()
    assert lat.aborted_launches() == 1                 # the injected launch; the next returned at once
    lat.init_rho(rho0).advance(200)
    lat.diagnostics()
    assert lat.aborted_launches() == 1                 # replacing the state does not reset the count
    ref = Lattice(n, 7, "fp64").set_physical(dX, dT, 0.0).set_kernel("plain").init_rho(rho0).advance(200)
    assert np.array_equal(lat.f(), ref.f())
    assert np.array_equal(lat.rho(), ref.rho())


def test_lattices_on_several_threads():
    # distinct lattices driven from different threads at once, each on its own
    # stream: the first launches of each kernel set process-wide attributes
    # (under a lock); every result equals the one computed alone
    import threading

    import torch
    say("case lattices on four threads")
    dX, dT = math.pi / 16, 1e-4
    shapes = [(20000, 7, "tiled"), (12345, 5, "tiled"), (4096, 7, "resident"), (3000, 7, "span")]

    def solve(n, q, kernel, stream=None):
        lat = Lattice(n, q, "fp64", stream=stream).set_physical(dX, dT, 0.0).set_kernel(kernel)
        lat.init_rho(random_modes_ic(n, n * dX, seed=n)).advance(500)
        return lat.rho()

    want = [solve(*sh) for sh in shapes]
    got = [None] * len(shapes)
    errors = []

    def work(k):
        try:
            with torch.cuda.stream(torch.cuda.Stream()):
                got[k] = solve(*shapes[k], stream=torch.cuda.current_stream())
        except Exception as e:   # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(shapes))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for w, g in zip(want, got):
        assert np.array_equal(w, g)


def test_beyond_32_bit_offsets():
    # a lattice of 2^29 + 5 sites: population rows start beyond 2^31 elements
    # and 2^34 bytes into the state; plain and tiled kernels agree bit for bit
    # and sampled sites (both ends, the middle, random) match the oracle on
    # their light cones
    import torch
    n, q, dX, dT, steps = (1 << 29) + 5, 7, math.pi / 128, 2e-8, 20
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 100e9:
        pytest.skip("needs about 75 GB of device memory")
    say("case beyond 32-bit offsets: n = %d" % n)
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (2 * math.pi / n)
    rho0 = 1.0 + 0.1 * torch.sin(3 * x) + 0.05 * torch.cos(17 * x + 0.3)
    del x
    outs = []
    for kernel in ("plain", "tiled"):
        lat = Lattice(n, q, "fp64").set_physical(dX, dT, 1.0).set_kernel(kernel)
        lat.init_rho(rho0).advance(steps)
        assert not lat.diagnostics()[1]
        outs.append(lat.read_rho())
        lat.close()
        del lat
        torch.cuda.empty_cache()
    assert torch.equal(outs[0], outs[1])
    half = 3 * steps + 8
    rng = np.random.default_rng(5)
    sites = [0, 1, n - 1, n // 2, (1 << 28) + 3] + [int(v) for v in rng.integers(0, n, 3)]
    for j in sites:
        idx = torch.tensor(np.arange(j - half, j + half + 1) % n, device="cuda")
        window = rho0[idx].cpu().numpy()
        ref = oracle.solve_periodic(q, window, dX, dT, 1.0, steps)[half]
        got = float(outs[1][j])
        assert abs(got - ref) <= TOL64 * np.max(np.abs(window)), (j, got, ref)
