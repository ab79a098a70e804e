"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
library routine (matrix inverse, eigenvalues), a closed form, a brute-force
definition, an independent textbook scheme, a conservation law or symmetry, or
a value the paper prints (tests/golden/paper_constants.txt).
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1711_03540_amd.inputs import random_modes_ic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            out[k.strip()] = float(v)
    return out


C5 = np.array([0, 1, -1, 2, -2])
C7 = np.array([0, 1, -1, 2, -2, 3, -3])


# ---------------------------------------------------------------- weights (appendix A)

def test_velocity_order():
    assert list(oracle.velocities(5)) == list(C5)
    assert list(oracle.velocities(7)) == list(C7)


def test_d1q5_weights_are_the_inverse_moment_matrix():
    # Eq. (cond_weight): sum_i c_i^p w(l)_i = delta_pl; the weights are the
    # columns of the inverse of the matrix M_pi = c_i^p (appendix A).
    M = np.array([[float(c) ** p for c in C5] for p in range(5)])
    inv = np.linalg.inv(M)
    w = oracle.weights()
    for l in range(5):
        np.testing.assert_allclose(w[l, :5], inv[:, l], rtol=0, atol=1e-14)
        assert w[l, 5] == 0.0 and w[l, 6] == 0.0


def test_d1q7_high_weights_are_the_inverse_moment_matrix():
    M = np.array([[float(c) ** p for c in C7] for p in range(7)])
    inv = np.linalg.inv(M)
    w = oracle.weights()
    for l in (5, 6):
        np.testing.assert_allclose(w[l], inv[:, l], rtol=0, atol=1e-14)


def test_padded_weights_sixth_moments():
    # The D1Q5 weights padded to D1Q7 carry sixth moments -4 (w2) and 5 (w4);
    # with C6 = -5M the w(6) term then cancels exactly the alpha^2/6 part of
    # Eq. (KS_trunc11), leaving alpha^4/90 as Eq. (remained_truc_error_KS) states.
    w = oracle.weights()
    assert np.dot(C7.astype(float) ** 6, w[2]) == pytest.approx(-4.0, abs=1e-13)
    assert np.dot(C7.astype(float) ** 6, w[4]) == pytest.approx(5.0, abs=1e-13)
    coef = oracle.coefficients(7, 0.1, 1e-5, 1.3)
    assert coef[4] == pytest.approx(-5.0 * coef[2], rel=1e-14)


# ---------------------------------------------------------------- T_i (Eq. (T_form))

def _T_series(i, tau, terms=20000):
    r = 1.0 - 1.0 / tau
    s = 0.0
    p = 1.0
    for n in range(1, terms):
        p *= r
        s += p * ((n + 1) ** i - n ** i)
        if abs(p) * (n + 1) ** i < 1e-30:
            break
    return s


@pytest.mark.parametrize("tau", [0.6, 0.75, 0.95, 1.0, 1.0065829931442369, 1.3, 2.0, 5.0])
@pytest.mark.parametrize("i", [1, 2, 3, 4])
def test_T_closed_form_matches_series_definition(i, tau):
    ref = _T_series(i, tau)
    got = oracle.T(i, tau)
    assert got == pytest.approx(ref, rel=1e-11, abs=1e-12)


# ---------------------------------------------------------------- equilibrium moments (Table 1)

@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("tau", [1.0, 1.4])
def test_equilibrium_moments(q, tau):
    dX, dT = 0.15, 3e-5
    coef = oracle.coefficients(q, dX, dT, tau)
    J, K, M, dM, C6 = coef
    c = (C5 if q == 5 else C7).astype(float)
    for rho in (0.7, -1.3, 2.9):
        f = oracle.feq(q, coef, rho)
        mom = [np.dot(c ** p, f) for p in range(7)]
        scale = abs(rho) + rho * rho
        assert mom[0] == pytest.approx(rho, abs=1e-14 * scale)
        assert mom[1] == pytest.approx(J * rho * rho, abs=1e-15 * scale)
        assert mom[2] == pytest.approx(K * rho, abs=1e-15 * scale)
        assert mom[3] == pytest.approx(0.0, abs=1e-15 * scale)
        assert mom[4] == pytest.approx((M + dM) * rho, rel=1e-13)


# ---------------------------------------------------------------- tau fit (Eqs. (general_tau_formula), (A_B_fit_*))

def test_tau_fit_branch_points_match_printed_values():
    g = golden()
    for q, key in ((5, "dT_crit_d1q5_dx0.1"), (7, "dT_crit_d1q7_dx0.1")):
        printed = g[key]
        # the fit gives tau = 1 below dT_crit and tau > 1 above it
        assert oracle.tau_fit(q, 0.1, printed * 0.99) == 1.0
        assert oracle.tau_fit(q, 0.1, printed * 1.01) > 1.0
        assert oracle.tau_fit(q, 0.1, printed * 1.01) < 1.0 + 1e-4
    assert 0.1 ** 4 / 90.0 == pytest.approx(g["beta_max_cond_stability_dx0.1"], rel=5e-3)


def test_tau_fit_d1q7_needs_larger_tau():
    # section 3: the D1Q7 model needs a larger tau than D1Q5 for stability
    for dX in (0.05, 0.1, 0.2):
        for dT in (1e-5, 1e-4, 1e-3):
            t5, t7 = oracle.tau_fit(5, dX, dT), oracle.tau_fit(7, dX, dT)
            if t5 > 1.0:
                assert t7 > t5


def _table3_bounded(q, dX, dT, tau):
    # the Table 3 run with fixed ends to T = 0.5 stays finite and |rho| < 100
    # (its solution lies in [0.6, 5.4])
    rho = oracle.solve_tanh_fixed(q, dX, dT, tau, int(round(0.5 / dT)))
    return bool(np.all(np.isfinite(rho)) and np.max(np.abs(rho)) < 100.0)


def _fit_with(A, B, dT):
    l = math.log10(dT)
    return A * (l + B) ** 2 + 1.0 if l >= -B else 1.0


TAU_FIT_CASES = [(q, dT) for q in (5, 7) for dT in (5e-4, 1e-3)]


def _band_holds(q, dT, fit):
    return _table3_bounded(q, 0.2, dT, fit + 0.04) and not _table3_bounded(q, 0.2, dT, fit - 0.06)


def test_tau_fit_tracks_the_blow_up_threshold_at_dx02():
    # Figs. 1-3 (left panels): the fit of Eq. (general_tau_formula) with the
    # A, B of Eqs. (A_B_fit_*) is the smallest stable tau of the Table 3
    # problem.  At dX = 0.2, where its A-dependent branch is active for these
    # dT, the oracle's run (pinned elsewhere) stays bounded at fit + 0.04 and
    # blows up at fit - 0.06 (its threshold lies 0.01-0.02 above the fit).
    for q, dT in TAU_FIT_CASES:
        fit = oracle.tau_fit(q, 0.2, dT)
        assert fit > 1.05
        assert _band_holds(q, dT, fit), (q, dT, fit)


def test_tau_fit_band_rejects_plausible_mistakes_in_A():
    # the band above would catch a mistyped A: the dX power dropped, its sign
    # flipped, or the prefactor off by ten each fail at least one case
    dX = 0.2
    coeffs = {5: (0.103, -0.381, -13.2 * dX + 6.56), 7: (0.0886, -0.472, -12.5 * dX + 6.64)}
    for mutate in (lambda a, e: a, lambda a, e: a * dX ** -e, lambda a, e: 10 * a * dX ** e):
        ok = []
        for q, dT in TAU_FIT_CASES:
            a, e, B = coeffs[q]
            assert _fit_with(a * dX ** e, B, dT) == pytest.approx(oracle.tau_fit(q, dX, dT), rel=1e-14)
            ok.append(_band_holds(q, dT, _fit_with(mutate(a, e), B, dT)))
        assert not all(ok)


# ---------------------------------------------------------------- tau = 1: textbook finite differences

def _fd_step(q, rho, dX, dT):
    """Forward Euler with central 4th-order stencils for rho_t = -(rho^2/2)_X - rho_XX - rho_XXXX.

    D1Q7 adds the sixth-difference correction that makes the fourth derivative
    4th-order accurate and the (dT^2/2) d^4 term (the first-order-in-dT part
    of the Taylor series of exp(dT L) for L = -d2 - d4, which is how a scheme
    removes the beta d^4 error of Eq. (KS_trunc2)).
    """
    def sh(a, k):  # a[j - k]
        return np.roll(a, k)
    u = rho
    u2 = u * u
    d1_u2 = (sh(u2, 2) - 8 * sh(u2, 1) + 8 * sh(u2, -1) - sh(u2, -2)) / (12 * dX)
    d2 = (-sh(u, 2) + 16 * sh(u, 1) - 30 * u + 16 * sh(u, -1) - sh(u, -2)) / (12 * dX * dX)
    delta4 = sh(u, 2) - 4 * sh(u, 1) + 6 * u - 4 * sh(u, -1) + sh(u, -2)
    if q == 5:
        d4 = delta4 / dX ** 4
        return u + dT * (-0.5 * d1_u2 - d2 - d4)
    delta6 = (sh(u, 3) - 6 * sh(u, 2) + 15 * sh(u, 1) - 20 * u + 15 * sh(u, -1)
              - 6 * sh(u, -2) + sh(u, -3))
    d4 = (delta4 - delta6 / 6.0) / dX ** 4
    return u + dT * (-0.5 * d1_u2 - d2 - d4) + 0.5 * dT * dT * delta4 / dX ** 4


@pytest.mark.parametrize("q", [5, 7])
def test_tau1_step_is_textbook_finite_differences(q):
    n, dX, dT, steps = 96, 0.3, 2e-4, 60
    rho0 = 1.0 + random_modes_ic(n, n * dX, seed=11, n_modes=8, amplitude=0.3)
    got = oracle.solve_periodic(q, rho0, dX, dT, 1.0, steps)
    ref = rho0.copy()
    for _ in range(steps):
        ref = _fd_step(q, ref, dX, dT)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- linear growth of Fourier modes

def _A_of_k(q, coef, tau, k):
    c = (C5 if q == 5 else C7).astype(float)
    E = (oracle.feq(q, coef, 1.0) - oracle.feq(q, coef, -1.0)) / 2.0   # d feq / d rho at rho = 0
    om = 1.0 / tau
    D = np.diag(np.exp(-1j * k * c))
    return D @ ((1.0 - om) * np.eye(q) + om * np.outer(E, np.ones(q)))


def _lambda_h(q, coef, tau, k):
    ev = np.linalg.eigvals(_A_of_k(q, coef, tau, k))
    return ev[np.argmin(np.abs(ev - 1.0))]


@pytest.mark.parametrize("q,tau", [(5, 1.0), (5, 1.5), (7, 1.0), (7, 1.0066), (7, 1.5)])
def test_mode_growth_matches_linear_operator_eigenvalue(q, tau):
    n, dX, dT = 64, 0.2, 1e-4
    coef = oracle.coefficients(q, dX, dT, tau)
    m = 3
    k = 2 * math.pi * m / n
    rho0 = 1e-10 * np.cos(k * np.arange(n))
    f = oracle.init(q, coef, rho0)
    f = oracle.advance(q, coef, tau, f, 200)
    r0 = np.fft.fft(oracle.density(f))[m]
    f = oracle.advance(q, coef, tau, f, 1)
    r1 = np.fft.fft(oracle.density(f))[m]
    lam = _lambda_h(q, coef, tau, k)
    assert abs(r1 / r0 - lam) < 1e-13


def _U(tau):
    # U_i = T_i + 1 from the series definition of T_i (section 2)
    return {i: _T_series(i, tau) + 1.0 for i in range(1, 7)}


def _basic_alpha_error(dX, tau):
    # beta^0 sixth-derivative coefficient of the basic D1Q5 scheme, Eq. (KS_trunc11)
    U = _U(tau)
    return dX ** 4 * U[6] / (90 * U[2]) - dX ** 2 * U[6] / (6 * U[4])


@pytest.mark.parametrize("tau", [1.0, 1.4])
@pytest.mark.parametrize("dX", [0.05, 0.1])
def test_d1q5_growth_rate_matches_truncation_analysis(tau, dX):
    # Linearised KS, rho_T = -rho_XX - rho_XXXX, grows exp(i kappa X) at
    # kappa^2 - kappa^4.  The LB growth per step ln|lambda|/dT differs from it
    # by the truncation errors of Eqs. (KS_trunc11) and (KS_trunc2); a d^m
    # term contributes (i kappa)^m times its coefficient.
    dT = 1e-6
    U = _U(tau)
    coef = oracle.coefficients(5, dX, dT, tau)
    e6 = _basic_alpha_error(dX, tau) + dT * (U[2] / U[1] - U[3] / U[2] - U[5] / U[4])
    e4 = dT * (U[2] / (2 * U[1]) - U[3] / U[2])
    for kappa in (0.3, 0.7071, 1.0):
        sigma = math.log(abs(_lambda_h(5, coef, tau, kappa * dX))) / dT
        model = kappa ** 2 - kappa ** 4 + e4 * kappa ** 4 - e6 * kappa ** 6
        err = abs(_basic_alpha_error(dX, tau)) * kappa ** 6
        assert abs(sigma - (kappa ** 2 - kappa ** 4)) > 0.5 * err      # the error is there ...
        assert abs(sigma - model) < 0.05 * err + 1e-9, (kappa, sigma, model)   # ... and predicted


@pytest.mark.parametrize("tau", [1.0, 1.4])
def test_d1q7_growth_rate_removes_alpha2_error(tau):
    # The w(6) correction of section 2.2 removes the alpha^2 d^6 error: D1Q7's
    # growth rate is far closer to kappa^2 - kappa^4 than D1Q5's, and its error
    # falls at 4th order in dX (Eq. (remained_truc_error_KS)).
    dT = 1e-6
    devs = []
    for dX in (0.05, 0.1):
        coef = oracle.coefficients(7, dX, dT, tau)
        for kappa in (0.7071, 1.0):
            sigma = math.log(abs(_lambda_h(7, coef, tau, kappa * dX))) / dT
            dev = abs(sigma - (kappa ** 2 - kappa ** 4))
            assert dev < 0.1 * abs(_basic_alpha_error(dX, tau)) * kappa ** 6
            if kappa == 1.0:
                devs.append(dev)
    if tau != 1.0:      # at tau = 1 the remaining error is dominated by dT terms
        assert devs[1] / devs[0] > 10.0


def test_delta_M_reading_cancels_fourth_order_error():
    # delta M (Eq. (delta_M)) is introduced to cancel the beta d^4 term of
    # Eq. (KS_trunc2).  Fit the small-kappa expansion of the D1Q7 growth rate
    # sigma = c2 kappa^2 + c4 kappa^4 + c6 kappa^6 + c8 kappa^8: with the bracket
    # read as (T3+1)/(T2+1) (dm_variant 0) c4 must be -1; the printed
    # (T3+1)/(T4+1) (dm_variant 1) misses it, and D1Q5 keeps the beta error.
    dX, dT, tau = 0.1, 1e-4, 1.5
    kap = np.linspace(0.05, 0.6, 24)

    def c4(q, variant):
        coef = oracle.coefficients(q, dX, dT, tau, variant)
        sig = np.array([math.log(abs(_lambda_h(q, coef, tau, k * dX))) / dT for k in kap])
        V = np.stack([kap ** 2, kap ** 4, kap ** 6, kap ** 8, kap ** 10], axis=1)
        sol = np.linalg.lstsq(V, sig, rcond=None)[0]
        return sol[0], sol[1]

    c2, c4d = c4(7, 0)
    assert c2 == pytest.approx(1.0, abs=1e-6)
    assert c4d == pytest.approx(-1.0, abs=2e-6)
    _, c4l = c4(7, 1)
    assert abs(c4l + 1.0) > 1e-5
    _, c45 = c4(5, 0)
    U1, U2, U3 = tau, tau * (2 * tau - 1), tau * (6 * tau * tau - 6 * tau + 1)
    # D1Q5 keeps beta {(T2+1)/(2(T1+1)) - (T3+1)/(T2+1)} d^4 (Eq. (KS_trunc2))
    assert c45 == pytest.approx(-1.0 + dT * (U2 / (2 * U1) - U3 / U2), abs=2e-6)


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("q,tau", [(5, 1.0), (7, 1.3)])
def test_mass_conservation(q, tau):
    n, dX, dT = 128, 0.2, 1e-4
    rho0 = random_modes_ic(n, n * dX, seed=5, n_modes=8, amplitude=0.5)
    rho = oracle.solve_periodic(q, rho0, dX, dT, tau, 2000)
    assert abs(rho.sum() - rho0.sum()) < 1e-12 * np.abs(rho0).sum()
    assert np.max(np.abs(rho - rho0)) > 1e-3   # it did evolve


@pytest.mark.parametrize("q", [5, 7])
def test_reflection_symmetry(q):
    # (X, rho) -> (-X, -rho) maps the KS equation and the scheme to themselves.
    n, dX, dT, tau = 80, 0.25, 1e-4, 1.2
    rho0 = random_modes_ic(n, n * dX, seed=9, n_modes=6, amplitude=0.6)
    mirror = lambda a: -np.roll(a[::-1], 1)       # site j -> site -j (mod n), sign flip
    a = oracle.solve_periodic(q, rho0, dX, dT, tau, 300)
    b = oracle.solve_periodic(q, mirror(rho0), dX, dT, tau, 300)
    np.testing.assert_allclose(mirror(a), b, rtol=0, atol=1e-13)


def test_periodic_shift_is_bitwise():
    n, dX, dT, tau = 70, 0.25, 1e-4, 1.1
    rho0 = random_modes_ic(n, n * dX, seed=3, n_modes=6, amplitude=0.6)
    a = oracle.solve_periodic(7, rho0, dX, dT, tau, 200)
    b = oracle.solve_periodic(7, np.roll(rho0, 13), dX, dT, tau, 200)
    assert np.array_equal(np.roll(a, 13), b)


@pytest.mark.parametrize("q", [5, 7])
def test_uniform_state_is_fixed_point(q):
    rho0 = np.full(50, 2.25)
    rho, f = oracle.solve_periodic(q, rho0, 0.2, 1e-4, 1.3, 100, want_f=True)
    np.testing.assert_allclose(rho, rho0, rtol=1e-14)
    coef = oracle.coefficients(q, 0.2, 1e-4, 1.3)
    np.testing.assert_allclose(f[:, 7], oracle.feq(q, coef, 2.25), rtol=1e-13, atol=1e-16)


# ---------------------------------------------------------------- Table 3 travelling wave

def test_tanh_constants_and_ends():
    g = golden()
    lo, hi = oracle.tanh_ends()
    assert lo + hi == pytest.approx(2 * g["tanh_b"], abs=1e-15)
    # the end values are the limits of the travelling wave far from its core
    assert oracle.tanh_solution(-1e3, 0.0)[0] == pytest.approx(lo, abs=1e-12)
    assert oracle.tanh_solution(1e3, 0.0)[0] == pytest.approx(hi, abs=1e-12)


def test_tanh_profile_solves_ks():
    # rho_T + rho rho_X + rho_XX + rho_XXXX = 0 for the Table 3 profile, checked
    # with centred differences of the closed form.
    X = np.linspace(10.0, 30.0, 41)
    h, t = 1e-2, 0.3
    r = lambda x, tt=t: oracle.tanh_solution(x, tt)
    rt = (r(X, t + 1e-5) - r(X, t - 1e-5)) / 2e-5
    rx = (r(X + h) - r(X - h)) / (2 * h)
    rxx = (r(X + h) - 2 * r(X) + r(X - h)) / h ** 2
    rxxxx = (r(X + 2 * h) - 4 * r(X + h) + 6 * r(X) - 4 * r(X - h) + r(X - 2 * h)) / h ** 4
    res = rt + r(X) * rx + rxx + rxxxx
    assert np.max(np.abs(res)) < 2e-3


def _G(q, dX, dT, tau, T):
    steps = int(round(T / dT))
    rho = oracle.solve_tanh_fixed(q, dX, dT, tau, steps)
    X = np.arange(rho.size) * dX
    return oracle.global_error(rho, oracle.tanh_solution(X, steps * dT))


def test_tanh_convergence_orders():
    # tau = 1, dT = dX^4/100: G falls at 2nd order for D1Q5 (beta^0 error
    # alpha^2 d^6, Eq. (KS_trunc11)) and at about 4th order for D1Q7, whose
    # alpha^2 term is removed (Eq. (remained_truc_error_KS)).
    T = 0.1
    g5 = [_G(5, dx, dx ** 4 / 100, 1.0, T) for dx in (0.4, 0.2)]
    g7 = [_G(7, dx, dx ** 4 / 100, 1.0, T) for dx in (0.4, 0.2)]
    o5 = math.log2(g5[0] / g5[1])
    o7 = math.log2(g7[0] / g7[1])
    assert 1.8 < o5 < 2.3, g5
    assert o7 > 3.3, g7
    assert g7[1] < g5[1]


@pytest.mark.slow
def test_tanh_convergence_orders_fine():
    T = 0.1
    g5 = [_G(5, dx, dx ** 4 / 100, 1.0, T) for dx in (0.2, 0.1)]
    g7 = [_G(7, dx, dx ** 4 / 100, 1.0, T) for dx in (0.2, 0.1)]
    assert 1.8 < math.log2(g5[0] / g5[1]) < 2.3
    assert math.log2(g7[0] / g7[1]) > 3.3


def test_d1q7_more_accurate_than_d1q5_at_fitted_tau():
    # section 3: at the same dT the improved D1Q7 scheme (larger, fitted tau)
    # is more accurate than the basic D1Q5 scheme.
    dX, dT, T = 0.1, 1e-4, 1.0
    g5 = _G(5, dX, dT, oracle.tau_fit(5, dX, dT), T)
    g7 = _G(7, dX, dT, oracle.tau_fit(7, dX, dT), T)
    assert g7 < 0.5 * g5
    assert g5 < 1e-2


# ---------------------------------------------------------------- G and the collision on their own

def test_global_error_hand_worked():
    # G of section 3: sum_x |rho^N - rho^A| / sum_x |rho^A|.  Worked by hand:
    # |diff| = 0.5, 0, 1, 1, 0.25 -> 2.75; |rho^A| = 1.5, 2, 2, 2, 0.25 -> 7.75.
    num = np.array([1.0, 2.0, 3.0, -1.0, 0.0])
    ana = np.array([1.5, 2.0, 2.0, -2.0, 0.25])
    assert oracle.global_error(num, ana) == 2.75 / 7.75
    # plausible slips give other values: normalising by sum |rho^N| (7),
    # dropping the absolute value of a negative rho^A (3.75), squaring
    assert 2.75 / 7.0 != 2.75 / 7.75 and 2.75 / 3.75 != 2.75 / 7.75
    # swapping the arguments changes only the denominator
    assert oracle.global_error(ana, num) == 2.75 / 7.0
    # exact agreement gives zero; scaling both arrays leaves G unchanged
    assert oracle.global_error(ana, ana) == 0.0
    assert oracle.global_error(4.0 * num, 4.0 * ana) == 2.75 / 7.75


@pytest.mark.parametrize("q", [5, 7])
@pytest.mark.parametrize("tau", [1.0, 1.3])
def test_collide_then_push_equals_one_step(q, tau):
    # Eq. (2) is collision at x followed by a move to x + c_i: the oracle's
    # collision alone, then a periodic shift of population i by c_i (numpy),
    # is bitwise its one-step advance.
    n, dX, dT = 97, 0.2, 1e-4
    c = C5 if q == 5 else C7
    coef = oracle.coefficients(q, dX, dT, tau)
    rng = np.random.default_rng(11)
    f = oracle.init(q, coef, random_modes_ic(n, n * dX, seed=4, amplitude=0.8))
    f = f + 1e-3 * rng.standard_normal(f.shape)          # off equilibrium
    post = oracle.collide(q, coef, tau, f)
    pushed = np.stack([np.roll(post[i], int(c[i])) for i in range(q)])
    assert np.array_equal(pushed, oracle.advance(q, coef, tau, f, 1))
    # the collision conserves the density of every site (section 2, rho = sum_i f_i)
    np.testing.assert_allclose(post.sum(axis=0), f.sum(axis=0), rtol=0, atol=1e-14)
    # it relaxes by 1/tau: post - feq = (1 - 1/tau)(f - feq), feq of the site's density
    eq = np.stack([oracle.feq(q, coef, r) for r in f.sum(axis=0)], axis=1)
    np.testing.assert_allclose(post - eq, (1.0 - 1.0 / tau) * (f - eq), rtol=0, atol=1e-14)
