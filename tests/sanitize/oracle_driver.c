/* The FP64 CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py with gcc): periodic solves of both
 * schemes on small and ragged lattices, the fixed-end Table 3 solve and the
 * global error.  Prints the mass drift of each periodic solve; any sanitizer
 * report aborts with a nonzero status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int ko_solve_periodic(int q, long n, double dX, double dT, double tau, int dm_variant,
                      const double *rho0, long nsteps, double *rho_out, double *f_out);
int ko_solve_tanh_fixed(int q, double dX, double dT, double tau, int dm_variant,
                        long nsteps, double *rho_out, long *n_out);
double ko_tanh_solution(double X, double t);
double ko_global_error(long n, const double *rho_num, const double *rho_ana);

int main(void)
{
    const long sizes[4] = {1, 3, 7, 100};
    double worst = 0.0;
    for (int q = 5; q <= 7; q += 2) {
        for (int s = 0; s < 4; s++) {
            const long n = sizes[s];
            double *rho0 = malloc(sizeof(double) * (size_t)n), *rho = malloc(sizeof(double) * (size_t)n);
            double *f = malloc(sizeof(double) * (size_t)q * (size_t)n);
            double m0 = 0.0, m1 = 0.0;
            for (long j = 0; j < n; j++) {
                rho0[j] = 1.0 + 0.1 * sin(0.37 * (double)j);
                m0 += rho0[j];
            }
            if (ko_solve_periodic(q, n, 0.2, 1e-4, 1.1, 0, rho0, 50, rho, f)) return 2;
            for (long j = 0; j < n; j++) m1 += rho[j];
            worst = fmax(worst, fabs(m1 - m0));
            free(rho0);
            free(rho);
            free(f);
        }
        long n = 0;
        double *rho = malloc(sizeof(double) * 2000), *ana = malloc(sizeof(double) * 2000);
        if (ko_solve_tanh_fixed(q, 0.2, 1e-4, 1.0, 0, 100, rho, &n) || n > 2000) return 3;
        for (long j = 0; j < n; j++) ana[j] = ko_tanh_solution(0.2 * (double)j, 100 * 1e-4);
        printf("q=%d fixed-end G=%.3e\n", q, ko_global_error(n, rho, ana));
        free(rho);
        free(ana);
    }
    printf("oracle mass drift max=%.3e\n", worst);
    return worst < 1e-12 ? 0 : 1;
}
