// Operation counts of the oracle's 1D Euler P2 stage (test infrastructure).
#include "ora_real.hpp"
#include "../oecdg_oracle.c"
#undef double

void ora_count_report(const char *name, const ora_count::Counts &c, double per);

extern "C++" void count_1d() {
    const long n = 256;
    ora1d p;
    std::memset(&p, 0, sizeof(p));
    p.k = 2, p.nc = 3, p.flux = FLUX_EULER, p.bc = BC_OUTFLOW, p.n = n, p.xlo = 0.0, p.xhi = 1.0, p.gamma = 1.4;
    const int K1 = 3, nc = 3;
    const long nd = n + 1;
    ora_real *uC = (ora_real *)calloc((size_t)nc * K1 * n, sizeof(ora_real));
    ora_real *uD = (ora_real *)calloc((size_t)nc * K1 * nd, sizeof(ora_real));
    ora_real *LC = (ora_real *)calloc((size_t)nc * K1 * n, sizeof(ora_real));
    ora_real *LD = (ora_real *)calloc((size_t)nc * K1 * nd, sizeof(ora_real));
    // smooth data: rho = 1 + 0.2 sin(2 pi x), v = 0.5, p = 1, with small slopes
    for (int mesh = 0; mesh < 2; ++mesh) {
        const long m = mesh == 0 ? n : nd;
        ora_real *u = mesh == 0 ? uC : uD;
        for (long i = 0; i < m; ++i) {
            const double x = (i + (mesh == 0 ? 0.5 : 0.0)) / (double)n;
            const double rho = 1.0 + 0.2 * std::sin(6.283185307179586 * x), v = 0.5, pr = 1.0;
            const double w[3] = {rho, rho * v, pr / 0.4 + 0.5 * rho * v * v};
            for (int q = 0; q < nc; ++q) {
                u[(q * K1 + 0) * m + i] = w[q];
                u[(q * K1 + 1) * m + i] = 0.01 * w[q] * std::cos(6.283185307179586 * x);
                u[(q * K1 + 2) * m + i] = 0.001 * w[q];
            }
        }
    }
    const double tau_max = 0.15 / (double)n / 2.0;
    const double cells = (double)(n + nd), dofs = cells * nc * K1;
    ora_count::counts() = ora_count::Counts();
    ora1d_rhs(&p, ora_real(tau_max), uC, uD, LC, LD);
    ora_count_report("1d_euler_p2.operator", ora_count::counts(), dofs);
    ora_count::counts() = ora_count::Counts();
    ora1d_oe(&p, ora_real(tau_max), uC, uD);
    ora_count_report("1d_euler_p2.oe", ora_count::counts(), dofs);
    ora_count::counts() = ora_count::Counts();
    ora1d_step(&p, 3, 1, ora_real(tau_max), ora_real(tau_max), uC, uD);
    ora_count_report("1d_euler_p2.step", ora_count::counts(), dofs);
    free(uC), free(uD), free(LC), free(LD);
}
