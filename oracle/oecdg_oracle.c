/*
 * oecdg_oracle.c -- plain, serial FP64 CPU oracle of the oscillation-eliminating
 * central DG (OECDG) method of Peng, Wu and Yuan, "Oscillation-eliminating
 * central DG schemes for hyperbolic conservation laws" (arXiv 2503.12473).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the product path never does.  It
 * shares no source, header, table or helper with the HIP implementation.
 *
 * Every routine is a direct, slow transcription of the paper's definitions:
 *   - semi-discrete CDG on the primal and dual meshes: Sec. 2.1, eq. (equcdg)
 *     and its 1D bilinear form eq. (eq:1D_H);
 *   - fully discrete RK-OECDG in c/d form: Sec. 2.2, eq. (eq:RKCDG);
 *   - the OE damping ODE (OEstep2D), the damping coefficients delta_K^m, the
 *     global scale sigma_K and the wave speed beta_{e,K}: Sec. 2.2 and the
 *     remarks after it (1D coefficients; shared coefficients for systems);
 *   - time step tau = C_CFL h / beta: Sec. 2.1 and Sec. 4 (numerical setup).
 * Integrals are evaluated with Gauss-Legendre quadrature with k+1 nodes on
 * each of the two halves of a cell (the halves on which the overlapping
 * solution of the other mesh is smooth); the paper names no rule.
 *
 * Data layout: coefficient m of component q of cell i is u[(q*(k+1)+m)*ncell+i]
 * in the unnormalised Legendre basis P_m(xi), xi = 2(x - x_K)/h.  Primal cell i
 * is [xlo + i h, xlo + (i+1) h].  Dual cell j is centred on the left edge of
 * primal cell j: [xlo + (j-1/2) h, xlo + (j+1/2) h]; there are n of them with
 * periodic boundaries and n+1 with outflow or reflective boundaries.  Outflow
 * ghost primal cells -1 and n are the constant extensions of the cell averages
 * of cells 0 and n-1.  Reflective walls (Euler only; the two-blast-wave example
 * of Sec. 4) make the ghosts the mirror images of cells 0 and n-1 about the
 * wall: the polynomial u(2 x_wall - x) with the momentum negated, i.e. mode m
 * of component q times (-1)^m, and times -1 more for the momentum.  Inflow
 * boundaries (the examples of Sec. 4 that prescribe an incoming state) make
 * the ghosts constant states given by the caller, held for the whole run.
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_ENONFINITE = -4, ORA_ENONPHYSICAL = -5 };
enum { FLUX_ADVECTION = 0, FLUX_BURGERS = 1, FLUX_EULER = 2 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3 };

typedef struct {
    int k;          /* polynomial degree */
    int nc;         /* components: 1 (advection, Burgers) or 3 (Euler) */
    int flux;       /* FLUX_* */
    int bc;         /* BC_* */
    long n;         /* primal cells */
    double xlo, xhi;
    double a;       /* advection speed */
    double gamma;   /* adiabatic index */
    int allow_negative_pressure;   /* Euler: a cell average with p <= 0 is not an error */
    int pad;
    double inflow[2][3];           /* BC_INFLOW: cell averages of the ghost cells left of cell 0
                                    * and right of cell n-1, held fixed */
} ora1d;

/* ------------------------------------------------------------------------ */
/* Legendre polynomials and Gauss-Legendre quadrature                         */
/* ------------------------------------------------------------------------ */

/* P_n(x) by Bonnet's recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}. */
double ora_legendre(int n, double x)
{
    if (n == 0) return 1.0;
    double pm = 1.0, p = x;
    for (int j = 1; j < n; ++j) {
        double pn = ((2.0 * j + 1.0) * x * p - j * pm) / (j + 1.0);
        pm = p;
        p = pn;
    }
    return p;
}

/* m-th derivative of P_n at x, from P_n' = sum_{j = n-1, n-3, ...} (2j+1) P_j. */
double ora_legendre_deriv(int n, int m, double x)
{
    if (m == 0) return ora_legendre(n, x);
    if (n < m) return 0.0;
    double s = 0.0;
    for (int j = n - 1; j >= 0; j -= 2) s += (2.0 * j + 1.0) * ora_legendre_deriv(j, m - 1, x);
    return s;
}

/* Q-point Gauss-Legendre rule on [-1,1]: Newton iteration on P_Q, nodes ascending. */
void ora_gauss_legendre(int Q, double *s, double *w)
{
    for (int i = 0; i < Q; ++i) {
        double x = -cos(M_PI * (i + 0.75) / (Q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p = ora_legendre(Q, x);
            double dp = ora_legendre_deriv(Q, 1, x);
            double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        double dp = ora_legendre_deriv(Q, 1, x);
        s[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

static double factorial(int m)
{
    double f = 1.0;
    for (int j = 2; j <= m; ++j) f *= j;
    return f;
}

/* ------------------------------------------------------------------------ */
/* Mesh bookkeeping                                                           */
/* ------------------------------------------------------------------------ */

static double cell_width(const ora1d *p) { return (p->xhi - p->xlo) / (double)p->n; }

long ora1d_ncell(const ora1d *p, int mesh)
{
    if (mesh == 0) return p->n;
    return p->bc == BC_PERIODIC ? p->n : p->n + 1;
}

/* Coefficient (q, m) of cell idx of mesh (0 primal, 1 dual), with the
 * periodic wrap or the outflow / reflective ghost rule for primal cells -1
 * and n. */
static double coef(const ora1d *p, const double *uC, const double *uD, int mesh, long idx, int q, int m)
{
    const int K1 = p->k + 1;
    if (mesh == 0) {
        if (p->bc == BC_PERIODIC) {
            idx = ((idx % p->n) + p->n) % p->n;
        } else if (p->bc == BC_REFLECTIVE && (idx < 0 || idx >= p->n)) {
            long src = idx < 0 ? -1 - idx : 2 * p->n - 1 - idx;      /* the mirror cell */
            double sign = (m % 2 == 1) ? -1.0 : 1.0;
            if (q == 1) sign = -sign;                                 /* momentum */
            return sign * uC[(long)(q * K1 + m) * p->n + src];
        } else if (p->bc == BC_INFLOW && (idx < 0 || idx >= p->n)) {
            return m == 0 ? p->inflow[idx < 0 ? 0 : 1][q] : 0.0;
        } else if (idx < 0 || idx >= p->n) {
            long src = idx < 0 ? 0 : p->n - 1;
            return m == 0 ? uC[(long)(q * K1) * p->n + src] : 0.0;
        }
        return uC[(long)(q * K1 + m) * p->n + idx];
    }
    long nd = ora1d_ncell(p, 1);
    if (p->bc == BC_PERIODIC) idx = ((idx % nd) + nd) % nd;
    return uD[(long)(q * K1 + m) * nd + idx];
}

/* Values (all components) at local xi of the polynomial on cell idx of mesh,
 * given basis[m] = the order-th derivative of P_m at xi. */
static void eval_cell(const ora1d *p, const double *uC, const double *uD, int mesh, long idx, const double *basis, double *out)
{
    for (int q = 0; q < p->nc; ++q) {
        double v = 0.0;
        for (int m = 0; m <= p->k; ++m) v += coef(p, uC, uD, mesh, idx, q, m) * basis[m];
        out[q] = v;
    }
}

/* basis[m] = d^order/dxi^order P_m(xi), m = 0..k */
static void basis_at(int k, int order, double xi, double *basis)
{
    for (int m = 0; m <= k; ++m) basis[m] = ora_legendre_deriv(m, order, xi);
}

/* Neighbours on the other mesh: the cell overlapping the left half and the
 * cell overlapping the right half of cell idx (the other mesh is smooth on
 * each half and its cell centres sit on this cell's edges). */
static void neighbours(int mesh, long idx, long *left, long *right)
{
    if (mesh == 0) { *left = idx; *right = idx + 1; }      /* dual cells centred at x_{i-1/2}, x_{i+1/2} */
    else           { *left = idx - 1; *right = idx; }      /* primal cells centred at x_{j-1}, x_j      */
}

/* ------------------------------------------------------------------------ */
/* Flux and wave speed                                                        */
/* ------------------------------------------------------------------------ */

static void flux1d(const ora1d *p, const double *w, double *f)
{
    if (p->flux == FLUX_ADVECTION) {
        f[0] = p->a * w[0];
    } else if (p->flux == FLUX_BURGERS) {
        f[0] = 0.5 * w[0] * w[0];
    } else {
        double rho = w[0], mom = w[1], E = w[2];
        double v = mom / rho;
        double pr = (p->gamma - 1.0) * (E - 0.5 * mom * v);
        f[0] = mom;
        f[1] = mom * v + pr;
        f[2] = (E + pr) * v;
    }
}

/* Spectral radius of f'(u) at a state (the local maximum wave speed).  Euler:
 * |v| + sqrt(gamma |p| / rho); the same as |v| + c for every physical state,
 * and finite where a cell average carries a non-positive pressure that the
 * problem tolerates (allow_negative_pressure). */
double ora1d_wavespeed(const ora1d *p, const double *ubar)
{
    if (p->flux == FLUX_ADVECTION) return fabs(p->a);
    if (p->flux == FLUX_BURGERS) return fabs(ubar[0]);
    double rho = ubar[0], mom = ubar[1], E = ubar[2];
    double v = mom / rho;
    double pr = (p->gamma - 1.0) * (E - 0.5 * mom * v);
    return fabs(v) + sqrt(p->gamma * fabs(pr) / rho);
}

/* A cell average is physical with positive density and pressure; with
 * allow_negative_pressure only the density is required to be positive. */
static int physical(const ora1d *p, const double *ubar)
{
    if (p->flux != FLUX_EULER) return 1;
    double rho = ubar[0], mom = ubar[1], E = ubar[2];
    if (!(rho > 0.0)) return 0;
    if (p->allow_negative_pressure) return 1;
    double pr = (p->gamma - 1.0) * (E - 0.5 * mom * mom / rho);
    return pr > 0.0;
}

/* ------------------------------------------------------------------------ */
/* CDG spatial operator (equcdg / eq:1D_H)                                     */
/* ------------------------------------------------------------------------ */

/* Time derivative of the modal coefficients on both meshes:
 *   (h/(2m+1)) da_m/dt = (1/tau_max) int_K (w - u_K) P_m dx
 *                        + int_K f(w) d/dx P_m dx
 *                        - [ f(w) P_m ]_{left edge}^{right edge}
 * where w is the solution of the other mesh (smooth on each half of K and
 * continuous at the edges of K, which are the other mesh's cell centres). */
int ora1d_rhs(const ora1d *p, double tau_max, const double *uC, const double *uD, double *LC, double *LD)
{
    const int k = p->k, K1 = k + 1, Q = k + 1, nc = p->nc;
    const double h = cell_width(p);
    double s[16], wq[16];
    double w[3], uk[3], fw[3], fl[3], fr[3], vl[3], vr[3];
    if (k < 0 || k > 6 || nc < 1 || nc > 3) return ORA_EINVAL;
    if (p->bc == BC_REFLECTIVE && p->flux != FLUX_EULER) return ORA_EINVAL;
    ora_gauss_legendre(Q, s, wq);

    /* basis values at the quadrature nodes of both halves: own cell at xi,
     * overlapping cell at xn = xi + 1 (left half) or xi - 1 (right half) */
    double own[2][16][8], nb[2][16][8], test[2][16][8], dtest[2][16][8], centre[8];
    for (int half = 0; half < 2; ++half)
        for (int g = 0; g < Q; ++g) {
            double xi = half == 0 ? 0.5 * (s[g] - 1.0) : 0.5 * (s[g] + 1.0);
            double xn = half == 0 ? xi + 1.0 : xi - 1.0;
            basis_at(k, 0, xi, own[half][g]);
            basis_at(k, 0, xn, nb[half][g]);
            basis_at(k, 0, xi, test[half][g]);
            basis_at(k, 1, xi, dtest[half][g]);
        }
    basis_at(k, 0, 0.0, centre);

    for (int mesh = 0; mesh < 2; ++mesh) {
        const long nk = ora1d_ncell(p, mesh);
        double *out = mesh == 0 ? LC : LD;
        for (long i = 0; i < nk; ++i) {
            long il, ir;
            neighbours(mesh, i, &il, &ir);
            double coup[3][8], vol[3][8];
            for (int q = 0; q < nc; ++q)
                for (int m = 0; m <= k; ++m) coup[q][m] = vol[q][m] = 0.0;
            for (int half = 0; half < 2; ++half) {
                for (int g = 0; g < Q; ++g) {
                    eval_cell(p, uC, uD, 1 - mesh, half == 0 ? il : ir, nb[half][g], w);
                    eval_cell(p, uC, uD, mesh, i, own[half][g], uk);
                    flux1d(p, w, fw);
                    for (int q = 0; q < nc; ++q)
                        for (int m = 0; m <= k; ++m) {
                            coup[q][m] += 0.5 * wq[g] * (w[q] - uk[q]) * test[half][g][m];
                            vol[q][m] += 0.5 * wq[g] * fw[q] * dtest[half][g][m];
                        }
                }
            }
            /* the other mesh at the edges of K: its cell centres (xi = 0) */
            eval_cell(p, uC, uD, 1 - mesh, il, centre, vl);
            eval_cell(p, uC, uD, 1 - mesh, ir, centre, vr);
            flux1d(p, vl, fl);
            flux1d(p, vr, fr);
            for (int q = 0; q < nc; ++q)
                for (int m = 0; m <= k; ++m) {
                    double sgn = (m % 2 == 0) ? 1.0 : -1.0;       /* P_m(-1); P_m(1) = 1 */
                    double R = (0.5 * h / tau_max) * coup[q][m] + vol[q][m] - (fr[q] * 1.0 - fl[q] * sgn);
                    out[(long)(q * K1 + m) * nk + i] = (2.0 * m + 1.0) / h * R;
                }
        }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* OE step: global statistics, damping coefficients, exact exponential        */
/* ------------------------------------------------------------------------ */

/* Points of the reference cell where ||u - avg(u)||_inf is sampled: the two
 * edges and the quadrature nodes of both halves. Returns the count. */
static int sigma_points(int k, double *xs)
{
    const int Q = k + 1;
    double s[16], wq[16];
    ora_gauss_legendre(Q, s, wq);
    int c = 0;
    xs[c++] = -1.0;
    for (int g = 0; g < Q; ++g) xs[c++] = 0.5 * (s[g] - 1.0);
    for (int g = 0; g < Q; ++g) xs[c++] = 0.5 * (s[g] + 1.0);
    xs[c++] = 1.0;
    return c;
}

#ifdef ORA_PAIRWISE_MEAN
/* Test-only build variant: the sum of the cell averages of cells [lo, hi) in
 * pairwise order instead of left to right.  Both are valid FP64 evaluations of
 * the same mean; the variant measures how far such rounding differences grow
 * over a long run. */
static double pairwise_sum(const ora1d *p, const double *uC, const double *uD, int mesh, int q, long lo, long hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (long i = lo; i < hi; ++i) s += coef(p, uC, uD, mesh, i, q, 0);
        return s;
    }
    long mid = lo + (hi - lo) / 2;
    return pairwise_sum(p, uC, uD, mesh, q, lo, mid) + pairwise_sum(p, uC, uD, mesh, q, mid, hi);
}
#endif

/* avg(u^M_q) = domain mean of the cell averages; sigma = max |u^M_q - avg|
 * over the sample points of every cell of mesh M.  avg/sigma: [mesh][q]. */
void ora1d_stats(const ora1d *p, const double *uC, const double *uD, double *avg, double *sigma)
{
    double xs[40], v[3], bs[40][8];
    int np = sigma_points(p->k, xs);
    for (int j = 0; j < np; ++j) basis_at(p->k, 0, xs[j], bs[j]);
    for (int mesh = 0; mesh < 2; ++mesh) {
        long nk = ora1d_ncell(p, mesh);
        for (int q = 0; q < p->nc; ++q) {
#ifdef ORA_PAIRWISE_MEAN
            double sum = pairwise_sum(p, uC, uD, mesh, q, 0, nk);
#else
            double sum = 0.0;
            for (long i = 0; i < nk; ++i) sum += coef(p, uC, uD, mesh, i, q, 0);
#endif
            avg[mesh * 3 + q] = sum / (double)nk;
        }
        for (int q = 0; q < p->nc; ++q) sigma[mesh * 3 + q] = 0.0;
        for (long i = 0; i < nk; ++i)
            for (int j = 0; j < np; ++j) {
                eval_cell(p, uC, uD, mesh, i, bs[j], v);
                for (int q = 0; q < p->nc; ++q) {
                    double d = fabs(v[q] - avg[mesh * 3 + q]);
                    if (d > sigma[mesh * 3 + q]) sigma[mesh * 3 + q] = d;
                }
            }
    }
}

/* Damping coefficients delta_K^m (m = 0..k) of every cell of both meshes,
 * from the undamped state:
 *   delta_K^m = max_q sum_{e in dK} beta_K (2m+1) h^{m-1} / ((2k-1) m! sigma_q)
 *                       | d^m/dx^m (u_K - v)_q (e) |
 * with u_K's own trace at e, v the other mesh (its centre sits on e), beta_K
 * the spectral radius at K's cell average, and 0 where sigma_q = 0.
 * dC: [m*nC + i], dD: [m*nD + j]. */
int ora1d_delta(const ora1d *p, const double *uC, const double *uD, double *dC, double *dD)
{
    const int k = p->k, nc = p->nc;
    const double h = cell_width(p);
    double avg[6], sigma[6], ubar[3], ownL[3], ownR[3], nbL[3], nbR[3];
    double bm1[8][8], bp1[8][8], b0[8][8];          /* [order][mode] at xi = -1, +1, 0 */
    if (p->bc == BC_REFLECTIVE && p->flux != FLUX_EULER) return ORA_EINVAL;
    ora1d_stats(p, uC, uD, avg, sigma);
    for (int m = 0; m <= k; ++m) {
        basis_at(k, m, -1.0, bm1[m]);
        basis_at(k, m, 1.0, bp1[m]);
        basis_at(k, m, 0.0, b0[m]);
    }
    for (int mesh = 0; mesh < 2; ++mesh) {
        long nk = ora1d_ncell(p, mesh);
        double *d = mesh == 0 ? dC : dD;
        for (long i = 0; i < nk; ++i) {
            long il, ir;
            neighbours(mesh, i, &il, &ir);
            for (int q = 0; q < nc; ++q) ubar[q] = coef(p, uC, uD, mesh, i, q, 0);
            double beta = ora1d_wavespeed(p, ubar);
            for (int m = 0; m <= k; ++m) {
                eval_cell(p, uC, uD, mesh, i, bm1[m], ownL);
                eval_cell(p, uC, uD, mesh, i, bp1[m], ownR);
                eval_cell(p, uC, uD, 1 - mesh, il, b0[m], nbL);
                eval_cell(p, uC, uD, 1 - mesh, ir, b0[m], nbR);
                double scale = pow(2.0 / h, m);                  /* d/dx = (2/h) d/dxi */
                double c = (2.0 * m + 1.0) * pow(h, m - 1) / ((2.0 * k - 1.0) * factorial(m));
                double dm = 0.0;
                for (int q = 0; q < nc; ++q) {
                    if (sigma[mesh * 3 + q] == 0.0) continue;
                    double jr = fabs(scale * (ownR[q] - nbR[q]));
                    double jl = fabs(scale * (ownL[q] - nbL[q]));
                    double val = c * (beta * jr + beta * jl) / sigma[mesh * 3 + q];
                    if (val > dm) dm = val;
                }
                d[(long)m * nk + i] = dm;
            }
        }
    }
    return ORA_OK;
}

/* F_tau: exact solution at time tau of the damping ODE with delta frozen at
 * the undamped state.  In the Legendre basis, u - P^{m-1} u keeps the modes
 * j >= max(m,1) (P^{-1} := P^0), so mode j >= 1 decays with rate
 * sum_{m=0}^{j} delta^m and mode 0 is untouched. In place on both meshes. */
int ora1d_oe(const ora1d *p, double tau, double *uC, double *uD)
{
    const int k = p->k, K1 = k + 1, nc = p->nc;
    if (k < 1) return ORA_OK;                       /* nothing to damp for k = 0 */
    long nC = ora1d_ncell(p, 0), nD = ora1d_ncell(p, 1);
    double *dC = malloc(sizeof(double) * K1 * nC);
    double *dD = malloc(sizeof(double) * K1 * nD);
    if (!dC || !dD) { free(dC); free(dD); return ORA_ENOMEM; }
    int rc = ora1d_delta(p, uC, uD, dC, dD);        /* all deltas before any damping */
    if (rc != ORA_OK) { free(dC); free(dD); return rc; }
    for (int mesh = 0; mesh < 2; ++mesh) {
        long nk = mesh == 0 ? nC : nD;
        double *u = mesh == 0 ? uC : uD;
        double *d = mesh == 0 ? dC : dD;
        for (long i = 0; i < nk; ++i)
            for (int j = 1; j <= k; ++j) {
                double S = 0.0;
                for (int m = 0; m <= j; ++m) S += d[(long)m * nk + i];
#ifdef ORA_EXP_LONG_DOUBLE
                double fac = (double)expl(-(long double)tau * S);   /* test-only variant */
#else
                double fac = exp(-tau * S);
#endif
                for (int q = 0; q < nc; ++q) u[(long)(q * K1 + j) * nk + i] *= fac;
            }
    }
    free(dC);
    free(dD);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Time step and RK-OECDG                                                     */
/* ------------------------------------------------------------------------ */

/* Largest wave speed over the cell averages of both meshes. */
double ora1d_max_wavespeed(const ora1d *p, const double *uC, const double *uD)
{
    double b = 0.0, ubar[3];
    for (int mesh = 0; mesh < 2; ++mesh) {
        long nk = ora1d_ncell(p, mesh);
        for (long i = 0; i < nk; ++i) {
            for (int q = 0; q < p->nc; ++q) ubar[q] = coef(p, uC, uD, mesh, i, q, 0);
            double s = ora1d_wavespeed(p, ubar);
            if (!(s <= b)) b = s;            /* NaN propagates */
        }
    }
    return b;
}

/* RK tables in the c/d form of eq:RKCDG, row l holds c_{l,0..l}, d_{l,0..l}. */
static int rk_table(int rk, double c[4][4], double d[4][4])
{
    memset(c, 0, sizeof(double) * 16);
    memset(d, 0, sizeof(double) * 16);
    switch (rk) {
    case 1: c[0][0] = 1; d[0][0] = 1; return 1;
    case 2: c[0][0] = 1; d[0][0] = 1; c[1][0] = 0.5; c[1][1] = 0.5; d[1][1] = 0.5; return 2;
    case 3:
        c[0][0] = 1; d[0][0] = 1;
        c[1][0] = 0.75; c[1][1] = 0.25; d[1][1] = 0.25;
        c[2][0] = 1.0 / 3.0; c[2][2] = 2.0 / 3.0; d[2][2] = 2.0 / 3.0;
        return 3;
    case 4:
        c[0][0] = 1; d[0][0] = 0.5;
        c[1][0] = 1; d[1][1] = 0.5;
        c[2][0] = 1; d[2][2] = 1;
        c[3][0] = -1.0 / 3.0; c[3][1] = 1.0 / 3.0; c[3][2] = 2.0 / 3.0; c[3][3] = 1.0 / 3.0; d[3][3] = 1.0 / 6.0;
        return 4;
    }
    return 0;
}

/* The same tables for the 2D oracle. */
int ora_rk_table(int rk, double c[4][4], double d[4][4]) { return rk_table(rk, c, d); }

static int check_state(const ora1d *p, const double *uC, const double *uD)
{
    const int K1 = p->k + 1;
    double ubar[3];
    for (int mesh = 0; mesh < 2; ++mesh) {
        long nk = ora1d_ncell(p, mesh);
        const double *u = mesh == 0 ? uC : uD;
        for (long e = 0; e < (long)p->nc * K1 * nk; ++e)
            if (!isfinite(u[e])) return ORA_ENONFINITE;
        for (long i = 0; i < nk; ++i) {
            for (int q = 0; q < p->nc; ++q) ubar[q] = u[(long)(q * K1) * nk + i];
            if (!physical(p, ubar)) return ORA_ENONPHYSICAL;
        }
    }
    return ORA_OK;
}

/* One fully discrete RK-OECDG step (eq:RKCDG) of size tau with the coupling
 * parameter tau_max; (uC, uD) holds u_sigma^n on entry, u_sigma^{n+1} on exit. */
int ora1d_step(const ora1d *p, int rk, int oe, double tau, double tau_max, double *uC, double *uD)
{
    double c[4][4], d[4][4];
    int s = rk_table(rk, c, d);
    if (s == 0) return ORA_EINVAL;
    const long sz_C = (long)p->nc * (p->k + 1) * ora1d_ncell(p, 0);
    const long sz_D = (long)p->nc * (p->k + 1) * ora1d_ncell(p, 1);
    const long sz = sz_C + sz_D;
    double *us = malloc(sizeof(double) * sz * (s + 1));   /* u_sigma^{n,m}, m = 0..s */
    double *Ls = malloc(sizeof(double) * sz * s);         /* L(u_sigma^{n,m}), m = 0..s-1 */
    if (!us || !Ls) { free(us); free(Ls); return ORA_ENOMEM; }
    memcpy(us, uC, sizeof(double) * sz_C);
    memcpy(us + sz_C, uD, sizeof(double) * sz_D);
    int rc = ORA_OK;
    for (int l = 0; l < s && rc == ORA_OK; ++l) {
        double *ul = us + sz * l;
        rc = ora1d_rhs(p, tau_max, ul, ul + sz_C, Ls + sz * l, Ls + sz * l + sz_C);
        double *un = us + sz * (l + 1);
        for (long e = 0; e < sz; ++e) {
            double v = 0.0;
            for (int m = 0; m <= l; ++m) v += c[l][m] * us[sz * m + e] + tau * d[l][m] * Ls[sz * m + e];
            un[e] = v;
        }
        if (oe) ora1d_oe(p, tau, un, un + sz_C);
        if (rc == ORA_OK) rc = check_state(p, un, un + sz_C);
    }
    if (rc == ORA_OK) {
        memcpy(uC, us + sz * s, sizeof(double) * sz_C);
        memcpy(uD, us + sz * s + sz_C, sizeof(double) * sz_D);
    }
    free(us);
    free(Ls);
    return rc;
}

/* March from t = 0 until t_end (last step clipped so that it lands on t_end)
 * or until nsteps steps (nsteps < 0: no limit).  tau_max = C_CFL h / beta with
 * beta from the cell averages of u^n on both meshes; dt_fixed > 0 replaces it.
 * A clipped last step keeps tau_max and uses the shorter tau. */
int ora1d_run(const ora1d *p, double cfl, int rk, int oe, double t_end, long nsteps, double dt_fixed,
              double *uC, double *uD, double *t_out, long *steps_out)
{
    const double h = cell_width(p);
    double t = 0.0;
    long step = 0;
    int rc = check_state(p, uC, uD);
    while (rc == ORA_OK && t < t_end && (nsteps < 0 || step < nsteps)) {
        double tau_max;
        if (dt_fixed > 0.0) {
            tau_max = dt_fixed;
        } else {
            double beta = ora1d_max_wavespeed(p, uC, uD);
            if (!(beta > 0.0) || !isfinite(beta)) { rc = ORA_EINVAL; break; }
            tau_max = cfl * h / beta;
        }
        double tau = tau_max;
        int last = 0;
        if (t + tau >= t_end) { tau = t_end - t; last = 1; }
        rc = ora1d_step(p, rk, oe, tau, tau_max, uC, uD);
        t = last ? t_end : t + tau;
        ++step;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = step;
    return rc;
}

/* One stage l of the RK table rk in the c/d form of eq:RKCDG given u_sigma^n
 * and u_sigma^{n,l}, followed by F_tau:
 *   out = F_tau( c_{l0} u^n + c_{ll} u^l + tau d_{ll} L(u^l) ),
 * for the stages whose other c_{lm}, d_{lm} vanish (every stage of forward
 * Euler, SSP-RK2 and SSP-RK3, the first three of classical RK4); EINVAL for
 * the others. */
int ora1d_rk_stage(const ora1d *p, int rk, int l, int oe, double tau, double tau_max,
                   const double *unC, const double *unD, const double *ulC, const double *ulD,
                   double *outC, double *outD)
{
    double c[4][4], d[4][4];
    const int s = rk_table(rk, c, d);
    if (s == 0 || l < 0 || l >= s) return ORA_EINVAL;
    for (int m = 0; m < l; ++m)             /* only u^n, u^{n,l} and L(u^{n,l}) may enter */
        if ((m > 0 && c[l][m] != 0.0) || d[l][m] != 0.0) return ORA_EINVAL;
    const long sz_C = (long)p->nc * (p->k + 1) * ora1d_ncell(p, 0);
    const long sz_D = (long)p->nc * (p->k + 1) * ora1d_ncell(p, 1);
    double *LC = malloc(sizeof(double) * sz_C), *LD = malloc(sizeof(double) * sz_D);
    if (!LC || !LD) { free(LC); free(LD); return ORA_ENOMEM; }
    int rc = ora1d_rhs(p, tau_max, ulC, ulD, LC, LD);
    for (long e = 0; e < sz_C; ++e) outC[e] = c[l][0] * unC[e] + (c[l][l] * ulC[e] + tau * d[l][l] * LC[e]);
    for (long e = 0; e < sz_D; ++e) outD[e] = c[l][0] * unD[e] + (c[l][l] * ulD[e] + tau * d[l][l] * LD[e]);
    if (l == 0) {   /* c_{00} multiplies u^n = u^{n,0} itself */
        for (long e = 0; e < sz_C; ++e) outC[e] = c[0][0] * ulC[e] + tau * d[0][0] * LC[e];
        for (long e = 0; e < sz_D; ++e) outD[e] = c[0][0] * ulD[e] + tau * d[0][0] * LD[e];
    }
    if (oe && rc == ORA_OK) rc = ora1d_oe(p, tau, outC, outD);
    if (rc == ORA_OK) rc = check_state(p, outC, outD);
    free(LC);
    free(LD);
    return rc;
}

int ora1d_ssprk3_stage(const ora1d *p, int l, int oe, double tau, double tau_max,
                       const double *unC, const double *unD, const double *ulC, const double *ulD,
                       double *outC, double *outD)
{
    return ora1d_rk_stage(p, 3, l, oe, tau, tau_max, unC, unD, ulC, ulD, outC, outD);
}
