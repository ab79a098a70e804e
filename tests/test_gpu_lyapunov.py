"""GPU: Benettin renormalisation of trajectory pairs (kslb_ensemble_renormalize).

Checked against the FP64 CPU oracle (one renormalisation of a nonlinear pair)
and against linear theory: about the fixed point rho = 0 the largest Lyapunov
exponent of the scheme is ln of the largest |eigenvalue| of the linearised
one-step operator over the lattice's wavenumbers, divided by dT.
"""
import numpy as np
import pytest

import oracle
from paper_1711_03540_amd import KslbError
from paper_1711_03540_amd.ensemble import Ensemble
from paper_1711_03540_amd.inputs import random_modes_ic

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def post_collision(q, coef, tau, rho0, steps):
    """Stored (post-collision) populations after `steps` steps from feq(rho0)."""
    f = oracle.advance(q, coef, tau, oracle.init(q, coef, rho0), steps)
    return oracle.collide(q, coef, tau, f)


@pytest.mark.parametrize("q", [5, 7])
def test_one_renormalisation_matches_oracle(q):
    import torch
    n, dX, dT, tau, steps, delta = 300, 0.2, 1e-4, 1.1, 400, 1e-7
    say("case renormalise q=%d" % q)
    rho_a = 1.0 + random_modes_ic(n, n * dX, seed=3, amplitude=0.3)
    rho_b = rho_a + 1e-6 * random_modes_ic(n, n * dX, seed=4, amplitude=1.0)
    ens = Ensemble([n, n], q, "fp64").set_physical(dX, dT, tau)
    ens.init_rho(0, rho_a).init_rho(1, rho_b).advance(steps)
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    ens.renormalize([0], [1], delta, acc)
    got_log = float(acc.cpu()[0])
    coef = oracle.coefficients(q, dX, dT, tau)
    Sa = post_collision(q, coef, tau, rho_a, steps)
    Sb = post_collision(q, coef, tau, rho_b, steps)
    d = np.sqrt(np.sum((Sb - Sa) ** 2))
    assert abs(got_log - np.log(d / delta)) < 1e-5
    # the perturbed state is now S_a + (S_b - S_a) delta / d; its density difference
    want = (Sb - Sa).sum(axis=0) * (delta / d)
    got = ens.rho(1) - ens.rho(0)
    assert np.max(np.abs(got - want)) < 1e-4 * np.max(np.abs(want))
    # a second call adds to the accumulator
    ens.renormalize([0], [1], delta, acc)
    assert abs(float(acc.cpu()[0]) - got_log) < 1e-6   # d is delta now: ln 1 added


def test_renormalisation_errors():
    import torch
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    e32 = Ensemble([64, 64], 7, "fp32").set_physical(0.4, 1e-3, 1.0)
    e32.init_rho(0, np.ones(64)).init_rho(1, np.ones(64))
    with pytest.raises(KslbError):
        e32.renormalize([0], [1], 1e-6, acc)
    ens = Ensemble([64, 64, 80], 7, "fp64").set_physical(0.4, 1e-3, 1.0)
    for i, n in enumerate((64, 64, 80)):
        ens.init_rho(i, np.ones(n))
    with pytest.raises(KslbError):
        ens.renormalize([0], [2], 1e-6, acc)          # sizes differ
    with pytest.raises(KslbError):
        ens.renormalize([0], [0], 1e-6, acc)          # the same instance
    with pytest.raises(KslbError):
        ens.renormalize([0, 1], [1, 0], 1e-6, acc)    # an instance both reference and perturbed
    with pytest.raises(KslbError):
        ens.renormalize([0], [1], -1.0, acc)
    # identical states: d = 0 -> NaN recorded, states untouched
    ens.renormalize([0], [1], 1e-6, acc)
    assert np.isnan(float(acc.cpu()[0]))
    assert np.array_equal(ens.rho(1), np.ones(64))


@pytest.mark.parametrize("q", [5, 7])
def test_linear_regime_exponent(q):
    import torch
    n, dX, dT = 64, 0.4, 1e-3
    ens = Ensemble([n, n], q, "fp64").set_physical(dX, dT, 0.0)
    tau = ens.tau
    coef = oracle.coefficients(q, dX, dT, tau)
    # largest |eigenvalue| of the one-step operator about rho = 0 over k = 2 pi m / n
    vel = oracle.velocities(q)
    E = (oracle.feq(q, coef, 1.0) - oracle.feq(q, coef, -1.0)) / 2.0
    w = 1.0 / tau
    M = (1.0 - w) * np.eye(q) + w * np.outer(E, np.ones(q))
    r = max(max(abs(np.linalg.eigvals(M @ np.diag(np.exp(-1j * 2 * np.pi * m / n * vel))))) for m in range(n))
    lam_lin = np.log(r) / dT
    say("case linear exponent q=%d tau=%.4f lambda_lin=%.6f" % (q, tau, lam_lin))
    ens.init_rho(0, np.zeros(n)).init_rho(1, 1e-9 * random_modes_ic(n, n * dX, seed=7, n_modes=8, amplitude=1.0))
    delta, per, intervals, skip = 1e-9, 1000, 120, 60
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    logs = []
    for k in range(intervals):
        ens.advance(per)
        before = float(acc.cpu()[0])
        ens.renormalize([0], [1], delta, acc)
        logs.append(float(acc.cpu()[0]) - before)
    assert np.all(ens.rho(0) == 0.0)                   # the reference stays at the fixed point
    lam = np.mean(logs[skip:]) / (per * dT)
    say("  lambda_gpu=%.6f" % lam)
    assert abs(lam - lam_lin) < 2e-4


@pytest.mark.parametrize("q", [5, 7])
def test_group_orthonormalisation_matches_qr_of_oracle_states(q):
    import torch
    n, dX, dT, tau, steps, delta, k = 200, 0.2, 1e-4, 1.1, 300, 1e-7, 3
    say("case orthonormalise q=%d k=%d" % (q, k))
    base = 1.0 + random_modes_ic(n, n * dX, seed=3, amplitude=0.3)
    rhos = [base] + [base + 1e-6 * random_modes_ic(n, n * dX, seed=10 + m, amplitude=1.0) for m in range(k)]
    ens = Ensemble([n] * (k + 1), q, "fp64").set_physical(dX, dT, tau)
    for i, r in enumerate(rhos):
        ens.init_rho(i, r)
    ens.advance(steps)
    acc = torch.zeros(k, dtype=torch.float64, device="cuda")
    ens.orthonormalize([0], [list(range(1, k + 1))], delta, acc)
    coef = oracle.coefficients(q, dX, dT, tau)
    S = [post_collision(q, coef, tau, r, steps) for r in rhos]
    V = np.stack([(S[m + 1] - S[0]).ravel() for m in range(k)], axis=1)
    Qm, R = np.linalg.qr(V)
    sign = np.sign(np.diag(R))
    want_log = np.log(np.abs(np.diag(R)) / delta)
    got_log = acc.cpu().numpy()
    assert np.max(np.abs(got_log - want_log)) < 1e-6, (got_log, want_log)
    # the perturbed densities now differ from the reference by delta times U
    # (density = sum over populations of each column of U, reshaped Q x n)
    for m in range(k):
        u = (Qm[:, m] * sign[m]).reshape(q, n)
        want = delta * u.sum(axis=0)
        got = ens.rho(m + 1) - ens.rho(0)
        assert np.max(np.abs(got - want)) < 1e-4 * np.max(np.abs(want)), m
    # a second call: the perturbations are orthonormal at scale delta, R = delta I
    before = acc.cpu().numpy().copy()
    ens.orthonormalize([0], [list(range(1, k + 1))], delta, acc)
    assert np.max(np.abs(acc.cpu().numpy() - before)) < 1e-6


def test_single_vector_group_equals_pair_renormalisation():
    import torch
    n, dX, dT, tau, steps, delta = 300, 0.2, 1e-4, 1.1, 200, 1e-7
    say("case orthonormalise k=1 vs pairs")
    rho_a = 1.0 + random_modes_ic(n, n * dX, seed=5, amplitude=0.3)
    rho_b = rho_a + 1e-6 * random_modes_ic(n, n * dX, seed=6, amplitude=1.0)
    outs = []
    for use_group in (False, True):
        ens = Ensemble([n, n], 7, "fp64").set_physical(dX, dT, tau)
        ens.init_rho(0, rho_a).init_rho(1, rho_b).advance(steps)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        if use_group:
            ens.orthonormalize([0], [[1]], delta, acc)
        else:
            ens.renormalize([0], [1], delta, acc)
        outs.append((float(acc.cpu()[0]), ens.rho(1) - ens.rho(0)))
    assert abs(outs[0][0] - outs[1][0]) < 1e-12 * abs(outs[0][0])
    assert np.max(np.abs(outs[0][1] - outs[1][1])) < 1e-6 * np.max(np.abs(outs[0][1]))


def test_group_orthonormalisation_errors():
    import torch
    from paper_1711_03540_amd import KslbError
    acc = torch.zeros(16, dtype=torch.float64, device="cuda")
    ens = Ensemble([64] * 4 + [80], 7, "fp64").set_physical(0.4, 1e-3, 1.0)
    for i, n in enumerate([64] * 4 + [80]):
        ens.init_rho(i, 1.0 + 0.01 * np.arange(n) / n)
    with pytest.raises(KslbError):
        ens.orthonormalize([0], [[1, 4]], 1e-6, acc)            # sizes differ
    with pytest.raises(KslbError):
        ens.orthonormalize([0], [[1, 1]], 1e-6, acc)            # an instance twice
    with pytest.raises(KslbError):
        ens.orthonormalize([0], [[0, 1]], 1e-6, acc)            # the reference perturbed
    with pytest.raises(KslbError):
        ens.orthonormalize([0], [list(range(1, 4)) * 3], 1e-6, acc)   # k > 8 (and repeats)
    # identical states: R is singular -> NaN recorded, states untouched
    ens.orthonormalize([0], [[1, 2]], 1e-6, acc)
    assert np.isnan(acc.cpu().numpy()[:2]).all()
    assert np.array_equal(ens.rho(1), ens.rho(0))


def test_linear_regime_leading_exponents():
    # about the fixed point rho = 0 the k leading exponents are the logs of the
    # k largest |eigenvalues| of the one-step operator over all wavenumbers
    # (m and n - m give equal moduli), divided by dT
    import torch
    q, n, dX, dT, k = 7, 64, 0.4, 1e-3, 3
    ens = Ensemble([n] * (k + 1), q, "fp64").set_physical(dX, dT, 0.0)
    tau = ens.tau
    coef = oracle.coefficients(q, dX, dT, tau)
    vel = oracle.velocities(q)
    E = (oracle.feq(q, coef, 1.0) - oracle.feq(q, coef, -1.0)) / 2.0
    w = 1.0 / tau
    M = (1.0 - w) * np.eye(q) + w * np.outer(E, np.ones(q))
    mods = sorted((abs(ev) for m in range(n) for ev in np.linalg.eigvals(M @ np.diag(np.exp(-1j * 2 * np.pi * m / n * vel)))),
                  reverse=True)
    lam_lin = np.log(np.array(mods[:k])) / dT
    say("case linear leading exponents k=%d lambda_lin=%s" % (k, lam_lin))
    ens.init_rho(0, np.zeros(n))
    for m in range(k):
        ens.init_rho(m + 1, 1e-9 * random_modes_ic(n, n * dX, seed=20 + m, n_modes=8, amplitude=1.0))
    delta, per, intervals, skip = 1e-9, 1000, 120, 60
    acc = torch.zeros(k, dtype=torch.float64, device="cuda")
    logs = []
    for t in range(intervals):
        ens.advance(per)
        before = acc.cpu().numpy().copy()
        ens.orthonormalize([0], [list(range(1, k + 1))], delta, acc)
        logs.append(acc.cpu().numpy() - before)
    assert np.all(ens.rho(0) == 0.0)
    lam = np.mean(np.array(logs[skip:]), axis=0) / (per * dT)
    say("  lambda_gpu=%s" % lam)
    assert np.max(np.abs(lam - lam_lin)) < 2e-3
