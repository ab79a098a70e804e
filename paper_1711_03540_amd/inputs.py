"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the lattice Boltzmann method: it only makes
initial densities, ensemble shapes and request streams.  Both the GPU path and
the CPU oracle receive the arrays it returns.

Random numbers come from SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), implemented here from
its published definition; a uniform draw is (next >> 11) * 2**-53.

The paper's only workload is the travelling wave of its Table 3 (built by the
oracle and by the fixed-end tests).  The workloads below are synthetic
stand-ins with the shapes the benchmark configurations name: periodic domains
of N sites on a length L, with initial densities that excite the linearly
unstable band 0 < kappa < 1 of the KS equation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def random_modes_ic(n: int, length: float, seed: int, n_modes: int = 16,
                    amplitude: float = 0.1) -> np.ndarray:
    """Sum of ``n_modes`` cosines with distinct integer wavenumbers and seeded phases.

    Wavenumbers m_j = 1 + floor(u * M_max) with M_max = max(n_modes, floor(L / 2 pi)),
    redrawn on a duplicate, then phases phi_j = 2 pi u; rho0_s = sum_j a cos(2 pi m_j s / n + phi_j).
    """
    sm = SplitMix64(seed)
    m_max = max(n_modes, int(math.floor(length / (2.0 * math.pi))))
    m_max = min(m_max, max(1, n // 2))
    modes: List[int] = []
    while len(modes) < min(n_modes, m_max):
        m = 1 + int(math.floor(sm.uniform() * m_max))
        if m not in modes:
            modes.append(m)
    phases = [2.0 * math.pi * sm.uniform() for _ in modes]
    s = np.arange(n, dtype=np.float64)
    rho = np.zeros(n, dtype=np.float64)
    for m, ph in zip(modes, phases):
        rho += amplitude * np.cos(2.0 * math.pi * m * s / n + ph)
    return rho


def kassam_trefethen_ic(n: int, length: float = 32.0 * math.pi) -> np.ndarray:
    """rho0(x) = cos(x/16) (1 + sin(x/16)) at x_j = j L / n."""
    x = np.arange(n, dtype=np.float64) * (length / n)
    return np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0))


@dataclass
class Workload:
    """One benchmark configuration: scheme, lattice, time step and length of the run."""
    name: str
    q: int
    n: int
    length: float
    dT: float
    steps: int
    precision: str = "fp64"
    tau: float = 0.0          # <= 0: the paper's fitted minimum stable tau
    ic_seed: int = 1
    ic: str = "modes"         # "modes" or "kt"

    @property
    def dX(self) -> float:
        return self.length / self.n

    def rho0(self) -> np.ndarray:
        if self.ic == "kt":
            return kassam_trefethen_ic(self.n, self.length)
        return random_modes_ic(self.n, self.length, self.ic_seed)


_PI = math.pi

# D1Q5, N = 256 on L = 32 pi; dT at equality in the tau = 1 stability bound
# alpha^4/90 >= beta of section 2.2, Eq. (cond_stability); 10^4 steps.
CFG_SMALL_Q5 = Workload("d1q5_n256_kt", 5, 256, 32 * _PI, (_PI / 8) ** 4 / 90.0, 10_000,
                        ic="kt")
# D1Q7, N = 4096 on L = 256 pi (dX = pi/16), 16 random modes, dT = 1e-4, 10^5 steps.
CFG_RESIDENT_Q7 = Workload("d1q7_n4096_modes", 7, 4096, 256 * _PI, 1e-4, 100_000, ic_seed=1)
# D1Q7, N = 2^24 on L = 32 pi 2^12 (dX = pi/128), dT = 2e-8, 10^3 steps.
CFG_LARGE_Q7 = Workload("d1q7_n16m_modes", 7, 1 << 24, 32 * _PI * 4096, 2e-8, 1_000, ic_seed=4)


# The travelling wave of the paper's Table 3 (section 3): b = 3, X0 = 20 on
# [X_m, X_M] = [0, 60], k = sqrt(11/19)/2, with end values b -+ (30/19) sqrt(11/19).
TABLE3_B = 3.0
TABLE3_XM = 60.0


def table3_profile(X, t: float = 0.0) -> np.ndarray:
    """rho(X, t) of the Table 3 solution (its initial condition at t = 0)."""
    X = np.asarray(X, dtype=np.float64)
    k = 0.5 * math.sqrt(11.0 / 19.0)
    a = (15.0 / 19.0) * math.sqrt(11.0 / 19.0)
    th = np.tanh(k * (X - TABLE3_B * t - TABLE3_XM / 3.0))
    return TABLE3_B + a * (-9.0 * th + 11.0 * th ** 3)


def table3_ends():
    left = TABLE3_B - (30.0 / 19.0) * math.sqrt(11.0 / 19.0)
    return left, 2.0 * TABLE3_B - left


def table3_sites(dX: float) -> int:
    """Sites X_j = j dX, j = 0 .. 60/dX."""
    return int(round(TABLE3_XM / dX)) + 1


def ensemble_shapes(count: int = 4096, seed: int = 2, n_lo: int = 512, n_hi: int = 8192) -> np.ndarray:
    """N_i = min(n_hi, floor(n_lo * (n_hi/n_lo)^u)), log-uniform on [n_lo, n_hi]."""
    sm = SplitMix64(seed)
    ratio = n_hi / n_lo
    return np.array([min(n_hi, int(math.floor(n_lo * ratio ** sm.uniform()))) for _ in range(count)],
                    dtype=np.int64)


@dataclass
class Request:
    arrival: float
    q: int
    n: int
    steps: int
    precision: str
    seed: int


def request_stream(count: int, seed: int = 3, rate: float = 2000.0, n_lo: int = 256,
                   n_hi: int = 65536, steps_lo: int = 1000, steps_hi: int = 100_000) -> List[Request]:
    """Poisson arrivals at ``rate``/s; scheme, size, length, precision and IC seed per request."""
    sm = SplitMix64(seed)
    t = 0.0
    out: List[Request] = []
    for _ in range(count):
        t += -math.log(1.0 - sm.uniform()) / rate
        q = 5 if sm.uniform() < 0.5 else 7
        n = min(n_hi, int(math.floor(n_lo * (n_hi / n_lo) ** sm.uniform())))
        steps = steps_lo + int(math.floor(sm.uniform() * (steps_hi - steps_lo + 1)))
        prec = "fp32" if sm.uniform() < 0.5 else "fp64"
        s = sm.next_u64()
        out.append(Request(t, q, n, steps, prec, s))
    return out
