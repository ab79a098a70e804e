// Host-side parameter code of libkslb under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py with g++):
// coefficients, the tau fit, spectral radii and the stability guard over a
// grid of schemes and parameters.  Prints one checksum line; any sanitizer
// report aborts with a nonzero status.
#include <cmath>
#include <cstdio>
#include <initializer_list>

#include "kslb_internal.h"

int main()
{
    double sum = 0.0;
    int checks = 0;
    const double dXs[3] = {0.05, 0.2, 0.3927};
    const double dTs[3] = {1e-6, 1e-4, 2e-3};
    const double taus[4] = {0.0, 0.95, 1.0, 1.6};
    for (int q : {5, 7}) {
        double w[7][7];
        kslb::scheme_weights(q, w);
        for (int l = 0; l < 7; l++)
            for (int i = 0; i < 7; i++) sum += w[l][i];
        for (double dX : dXs)
            for (double dT : dTs)
                for (double tau0 : taus)
                    for (int dm = 0; dm < 2; dm++) {
                        const double tau = tau0 > 0.0 ? tau0 : kslb::tau_fit(q, dX, dT);
                        double jkm[5], E[7] = {}, G[7] = {};
                        if (kslb::scheme_coefficients(q, dX, dT, tau, dm, jkm, E, G)) continue;
                        for (int i = 0; i < q; i++) sum += E[i] + G[i];
                        for (double k : {0.0, 0.5, 1.5, 3.14159})
                            sum += kslb::spectral_radius(q, E, G, 1.0 / tau, 1.0, k);
                        sum += kslb::stability_check(q, E, G, 1.0 / tau, dX, dT, 3.0);
                        checks++;
                    }
    }
    std::printf("params checks=%d checksum=%.12e\n", checks, sum);
    return std::isfinite(sum) ? 0 : 1;
}
