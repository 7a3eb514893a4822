// Operation counts of the oracle's 2D Euler Q2 stage (test infrastructure).
#include "ora_real.hpp"
#include "../oecdg_oracle_2d.c"
#undef double

void ora_count_report(const char *name, const ora_count::Counts &c, double per);

extern "C++" void count_2d() {
    const long nx = 32, ny = 32;
    ora2d p;
    std::memset(&p, 0, sizeof(p));
    p.k = 2, p.nc = 4, p.flux = FLUX_EULER, p.nx = nx, p.ny = ny, p.xlo = 0.0, p.xhi = 1.0, p.ylo = 0.0, p.yhi = 1.0;
    p.gamma = 1.4, p.space = 0;
    const int K1 = 3, nc = 4;
    const long ncell = nx * ny, sz = (long)nc * K1 * K1 * ncell;
    ora_real *uC = (ora_real *)calloc(sz, sizeof(ora_real)), *uD = (ora_real *)calloc(sz, sizeof(ora_real));
    ora_real *LC = (ora_real *)calloc(sz, sizeof(ora_real)), *LD = (ora_real *)calloc(sz, sizeof(ora_real));
    for (int mesh = 0; mesh < 2; ++mesh) {
        ora_real *u = mesh == 0 ? uC : uD;
        for (long iy = 0; iy < ny; ++iy)
            for (long ix = 0; ix < nx; ++ix) {
                const double s = mesh == 0 ? 0.5 : 0.0;
                const double x = (ix + s) / (double)nx, y = (iy + s) / (double)ny;
                const double rho = 1.0 + 0.2 * std::sin(6.283185307179586 * (x + y)), vx = 0.3, vy = -0.2, pr = 1.0;
                const double w[4] = {rho, rho * vx, rho * vy, pr / 0.4 + 0.5 * rho * (vx * vx + vy * vy)};
                for (int q = 0; q < nc; ++q)
                    for (int a = 0; a < K1; ++a)
                        for (int b = 0; b < K1; ++b) {
                            const double c = (a == 0 && b == 0) ? w[q] : 0.003 * w[q] / (1.0 + a + b);
                            u[((((long)q * K1 + a) * K1 + b) * ny + iy) * nx + ix] = c;
                        }
            }
    }
    const double tau_max = 0.3 / (double)nx / 4.0;
    const double dofs = 2.0 * ncell * nc * K1 * K1;
    ora_count::counts() = ora_count::Counts();
    ora2d_rhs(&p, ora_real(tau_max), uC, uD, LC, LD);
    ora_count_report("2d_euler_q2.operator", ora_count::counts(), dofs);
    ora_count::counts() = ora_count::Counts();
    ora2d_oe(&p, ora_real(tau_max), uC, uD);
    ora_count_report("2d_euler_q2.oe", ora_count::counts(), dofs);
    ora_count::counts() = ora_count::Counts();
    ora2d_step(&p, 3, 1, ora_real(tau_max), ora_real(tau_max), uC, uD);
    ora_count_report("2d_euler_q2.step", ora_count::counts(), dofs);
    free(uC), free(uD), free(LC), free(LD);
}
