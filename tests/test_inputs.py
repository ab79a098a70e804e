"""Seeded input generators (no arithmetic of the method)."""
import math

import numpy as np

from paper_1711_03540_amd.inputs import (CFG_LARGE_Q7, CFG_RESIDENT_Q7, CFG_SMALL_Q5, SplitMix64,
                                         ensemble_shapes, random_modes_ic, request_stream)


def test_splitmix64_published_outputs():
    # reference outputs of SplitMix64 for seeds 0 and 1234567
    s = SplitMix64(0)
    assert [s.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    s = SplitMix64(1234567)
    assert [s.next_u64() for _ in range(3)] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_random_modes_deterministic_and_in_band():
    a = random_modes_ic(4096, 256 * math.pi, seed=1)
    b = random_modes_ic(4096, 256 * math.pi, seed=1)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, random_modes_ic(4096, 256 * math.pi, seed=2))
    spec = np.abs(np.fft.rfft(a))
    modes = np.nonzero(spec > 1e-6 * spec.max())[0]
    assert len(modes) == 16
    assert modes.max() <= 128      # kappa = 2 pi m / L <= 1: the unstable band
    assert abs(a.mean()) < 1e-12


def test_config_shapes():
    assert CFG_SMALL_Q5.q == 5 and CFG_SMALL_Q5.n == 256
    assert math.isclose(CFG_SMALL_Q5.dX, math.pi / 8)
    assert math.isclose(CFG_SMALL_Q5.dT, (math.pi / 8) ** 4 / 90)
    assert CFG_RESIDENT_Q7.n == 4096 and math.isclose(CFG_RESIDENT_Q7.dX, math.pi / 16)
    assert CFG_LARGE_Q7.n == 1 << 24 and math.isclose(CFG_LARGE_Q7.dX, math.pi / 128)
    r = CFG_SMALL_Q5.rho0()
    x = np.arange(256) * math.pi / 8
    assert np.allclose(r, np.cos(x / 16) * (1 + np.sin(x / 16)))


def test_ensemble_shapes_log_uniform():
    n = ensemble_shapes(4096, seed=2)
    assert n.min() >= 512 and n.max() <= 8192
    assert abs(np.log(n).mean() - np.log(512 * 4)) < 0.1
    assert np.array_equal(n, ensemble_shapes(4096, seed=2))


def test_request_stream():
    reqs = request_stream(2000, seed=3)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(len(reqs) / t[-1] - 2000) < 200
    assert {r.q for r in reqs} == {5, 7}
    assert {r.precision for r in reqs} == {"fp32", "fp64"}
    assert min(r.n for r in reqs) >= 256 and max(r.n for r in reqs) <= 65536
    assert min(r.steps for r in reqs) >= 1000 and max(r.steps for r in reqs) <= 100000


def test_table3_profile_matches_the_oracle():
    # two independent codings of the Table 3 formula
    import oracle
    from paper_1711_03540_amd.inputs import table3_ends, table3_profile, table3_sites
    X = np.linspace(-10, 70, 161)
    for t in (0.0, 0.7):
        assert np.allclose(table3_profile(X, t), oracle.tanh_solution(X, t), rtol=0, atol=1e-14)
    assert np.allclose(table3_ends(), oracle.tanh_ends(), atol=1e-15)
    assert table3_sites(0.05) == 1201 and table3_sites(0.2) == 301
