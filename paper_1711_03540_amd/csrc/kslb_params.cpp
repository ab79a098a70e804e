// kslb_params.cpp -- host-side parameters of the KS lattice Boltzmann scheme:
// weights, coefficients, the fitted tau and the linear stability guard.
//
// Weights: appendix A defines w(l) by the moment conditions of
// Eq. (cond_weight), sum_i c_i^p w(l)_i = delta_pl.  That makes w(l)_i the
// x^l coefficient of the Lagrange basis polynomial of node c_i,
//     L_i(x) = prod_{j != i} (x - c_j) / (c_i - c_j),
// which is how they are computed here (integer polynomial products, one
// division per weight, so every weight is the correctly rounded rational).
// D1Q7 uses the D1Q5 weights w(0..4), zero at c = +-3, plus w(6) of the
// seven-velocity lattice (section 2.3 names both appendix equations).
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>

#include "kslb_internal.h"

namespace kslb {

static const int kVel[7] = {0, +1, -1, +2, -2, +3, -3};

// x^l coefficient of L_i(x) over the first n velocities.
static double lagrange_weight(int n, int i, int l)
{
    int64_t poly[8] = {1, 0, 0, 0, 0, 0, 0, 0};   // ascending powers
    int deg = 0;
    int64_t den = 1;
    for (int j = 0; j < n; j++) {
        if (j == i) continue;
        // poly *= (x - c_j)
        for (int d = deg + 1; d >= 1; d--) poly[d] = poly[d - 1] - kVel[j] * poly[d];
        poly[0] = -kVel[j] * poly[0];
        deg++;
        den *= (kVel[i] - kVel[j]);
    }
    return (double)poly[l] / (double)den;
}

void scheme_weights(int q, double w[7][7])
{
    std::memset(w, 0, sizeof(double) * 49);
    for (int l = 0; l <= 4; l++)
        for (int i = 0; i < 5; i++) w[l][i] = lagrange_weight(5, i, l);
    if (q == 7)
        for (int l = 5; l <= 6; l++)
            for (int i = 0; i < 7; i++) w[l][i] = lagrange_weight(7, i, l);
}

// U_n = T_n + 1 with T_n from Eq. (T_form), in factored form.
static void u_terms(double tau, double& U1, double& U2, double& U3, double& U4)
{
    U1 = tau;
    U2 = tau * (2.0 * tau - 1.0);
    U3 = tau * (6.0 * tau * tau - 6.0 * tau + 1.0);
    U4 = tau * (2.0 * tau - 1.0) * (12.0 * tau * tau - 12.0 * tau + 1.0);
}

int scheme_coefficients(int q, double dX, double dT, double tau, int dm_variant, double jkm[5],
                        double* E, double* G)
{
    if (q != 5 && q != 7) return -1;
    if (!(dX > 0.0) || !(dT > 0.0) || !(tau >= kTauMin) || !std::isfinite(dX) ||
        !std::isfinite(dT) || !std::isfinite(tau))
        return -1;
    if (dm_variant != 0 && dm_variant != 1) return -1;
    double U1, U2, U3, U4;
    u_terms(tau, U1, U2, U3, U4);
    const double a2 = dX * dX, a4 = a2 * a2;
    // Table 2
    const double J = dT / (2.0 * dX);
    const double K = -2.0 * dT * U1 / (a2 * U2);
    const double M = -24.0 * dT * U1 / (a4 * U4);
    double dM = 0.0, C6 = 0.0;
    if (q == 7) {
        // Eq. (delta_M); bracket per dm_variant
        const double r = (dm_variant == 0) ? U3 / U2 : U3 / U4;
        dM = -24.0 * dT * dT * U1 / (a4 * U4) * (U2 / (2.0 * U1) - r);
        // delta f_eq of section 2.2
        C6 = 120.0 * U1 * dT / (U4 * a4);
    }
    jkm[0] = J; jkm[1] = K; jkm[2] = M; jkm[3] = dM; jkm[4] = C6;
    double w[7][7];
    scheme_weights(q, w);
    for (int i = 0; i < q; i++) {
        double e = w[0][i] + K * w[2][i] + (M + dM) * w[4][i] + C6 * w[6][i];
        if (E) E[i] = e;
        if (G) G[i] = J * w[1][i];
    }
    // Eq. (feq): the even-moment weights take equal values at +c and -c and
    // w(1) changes sign; state that symmetry exactly (the kernels share the
    // product E rho within a +-c pair)
    for (int k = 1; 2 * k < q; k++) {
        if (E) E[2 * k] = E[2 * k - 1];
        if (G) G[2 * k] = -G[2 * k - 1];
    }
    return 0;
}

double tau_fit(int q, double dX, double dT)
{
    if (!(dX > 0.0) || !(dT > 0.0)) return NAN;
    double A, B;
    if (q == 5) {            // Eq. (A_B_fit_D1Q5)
        A = 0.103 * std::pow(dX, -0.381);
        B = -13.2 * dX + 6.56;
    } else if (q == 7) {     // Eq. (A_B_fit_D1Q7)
        A = 0.0886 * std::pow(dX, -0.472);
        B = -12.5 * dX + 6.64;
    } else {
        return NAN;
    }
    const double lg = std::log10(dT);   // Eq. (general_tau_formula)
    return (lg + B >= 0.0) ? A * (lg + B) * (lg + B) + 1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// Linear stability.  Linearised about rho_bar, one step maps Fourier
// amplitudes f^ by A(k) = D [(1 - w) I + w v 1^T], D = diag(exp(-i k c)),
// v = E + 2 rho_bar G.  By the matrix determinant lemma its characteristic
// polynomial is
//     p(z) = prod_i (z - a_i) - w sum_i d_i v_i prod_{j != i} (z - a_j),
// a_i = (1 - w) d_i, whose roots are found by Durand-Kerner iteration.
// ---------------------------------------------------------------------------
typedef std::complex<double> cplx;

static void poly_mul_linear(cplx* p, int& deg, cplx root)   // p *= (z - root)
{
    for (int d = deg + 1; d >= 1; d--) p[d] = p[d - 1] - root * p[d];
    p[0] = -root * p[0];
    deg++;
}

double spectral_radius(int q, const double* E, const double* G, double omega, double rho_bar,
                       double k)
{
    cplx d[7], a[7], v[7];
    for (int i = 0; i < q; i++) {
        d[i] = std::exp(cplx(0.0, -k * kVel[i]));
        a[i] = (1.0 - omega) * d[i];
        v[i] = E[i] + 2.0 * rho_bar * G[i];
    }
    cplx p[8] = {};
    int deg = 0;
    p[0] = 1.0;
    for (int i = 0; i < q; i++) poly_mul_linear(p, deg, a[i]);
    for (int i = 0; i < q; i++) {
        cplx t[8] = {};
        int dt = 0;
        t[0] = 1.0;
        for (int j = 0; j < q; j++)
            if (j != i) poly_mul_linear(t, dt, a[j]);
        for (int e = 0; e <= dt; e++) p[e] -= omega * d[i] * v[i] * t[e];
    }
    // monic degree q; Durand-Kerner
    cplx z[7];
    const cplx seed(0.4, 0.9);
    z[0] = 1.0;
    for (int i = 1; i < q; i++) z[i] = z[i - 1] * seed;
    for (int it = 0; it < 2000; it++) {
        double change = 0.0;
        for (int i = 0; i < q; i++) {
            cplx num = p[q];
            for (int e = q - 1; e >= 0; e--) num = num * z[i] + p[e];
            cplx den = 1.0;
            for (int j = 0; j < q; j++)
                if (j != i) den *= (z[i] - z[j]);
            if (std::abs(den) == 0.0) den = 1e-300;
            cplx dz = num / den;
            z[i] -= dz;
            change = std::fmax(change, std::abs(dz));
        }
        // roots are O(1): a step below 1e-15 is within a few ulp (quadratic
        // convergence reaches it from about 1e-8 in one iteration)
        if (change < 1e-15) break;
    }
    double r = 0.0;
    for (int i = 0; i < q; i++) r = std::fmax(r, std::abs(z[i]));
    return r;
}

int stability_check(int q, const double* E, const double* G, double omega, double dX, double dT,
                    double rho_max)
{
    const double rb[3] = {0.0, rho_max, -rho_max};
    const double grow = std::exp(0.3 * dT);
    for (int r = 0; r < (rho_max > 0.0 ? 3 : 1); r++) {
        for (int s = 0; s <= 800; s++) {
            const double k = M_PI * s / 800.0;
            const double rad = spectral_radius(q, E, G, omega, rb[r], k);
            const double lim = (k > 1.5 * dX) ? 1.0 + 1e-13 : grow;
            if (!(rad <= lim)) return 0;
        }
    }
    return 1;
}

}  // namespace kslb
