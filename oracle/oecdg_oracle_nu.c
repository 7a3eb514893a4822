/*
 * oecdg_oracle_nu.c -- plain, serial FP64 CPU oracle of the 1D OECDG method on
 * a non-uniform periodic mesh.
 *
 * TEST INFRASTRUCTURE, like the rest of this library: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never does, and it shares nothing with the HIP implementation.
 *
 * What it follows:
 *   - the meshes of the 1D setting of Sec. 2.1: primal cells
 *     [x_{i-1/2}, x_{i+1/2}] of width h_i with centres x_i, dual cells
 *     [x_i, x_{i+1}] between neighbouring primal centres, h = max_i h_i;
 *   - the bilinear form eq. (eq:1D_H), the RK-OECDG stages eq. (eq:RKCDG), the
 *     damping ODE and delta_K^m, sigma_K, beta_{e,K} of Sec. 2.2 with h_{e,K}
 *     = the width of K (the largest distance from a point of K to an end point)
 *     and avg = the domain integral over |Omega| (width-weighted cell averages);
 *   - tau_max = C_CFL h / beta with h the largest primal width (Sec. 2.1).
 * The analysis of Sec. 3 assumes quasi-uniform meshes and periodic boundaries;
 * only periodic boundaries are accepted here.
 *
 * Geometry: edges[i] = x_{i-1/2} for i = 0..n, edges[0] = xlo, edges[n] = xhi,
 * strictly increasing.  Dual cell j is [x_{j-1}, x_j] (index j-1 taken
 * periodically, shifted by the period), so it holds the primal edge edges[j]
 * at its own local coordinate (h_{j-1} - h_j)/(h_{j-1} + h_j), not at its centre.
 * Each cell is integrated piecewise, split where the other mesh has its edge
 * (a primal cell at its centre, a dual cell at the primal edge it holds), with
 * k+1 Gauss-Legendre nodes per piece, as in the uniform oracle.  Modal layout
 * and basis as in the uniform oracle: u[(q*(k+1)+m)*n + i], P_m(xi) with xi =
 * 2(x - centre)/width of the cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_ENONFINITE = -4, ORA_ENONPHYSICAL = -5 };
enum { FLUX_ADVECTION = 0, FLUX_BURGERS = 1, FLUX_EULER = 2 };
enum { BC_PERIODIC = 0 };

/* the same parameter block as the uniform oracle's */
typedef struct {
    int k, nc, flux, bc;
    long n;
    double xlo, xhi, a, gamma;
    int allow_negative_pressure, pad;
    double inflow[2][3];
} ora1d;

double ora_legendre_deriv(int n, int m, double x);
void ora_gauss_legendre(int Q, double *s, double *w);
int ora_rk_table(int rk, double c[4][4], double d[4][4]);
double ora1d_wavespeed(const ora1d *p, const double *ubar);

static int check_mesh(const ora1d *p, const double *edges)
{
    if (p->k < 0 || p->k > 6 || p->nc < 1 || p->nc > 3 || p->n < 2 || p->bc != BC_PERIODIC) return ORA_EINVAL;
    if (p->flux == FLUX_EULER ? p->nc != 3 : p->nc != 1) return ORA_EINVAL;
    if (edges[0] != p->xlo || edges[p->n] != p->xhi) return ORA_EINVAL;
    for (long i = 0; i < p->n; ++i)
        if (!(edges[i + 1] > edges[i])) return ORA_EINVAL;
    return ORA_OK;
}

static long wrap(long i, long n) { return ((i % n) + n) % n; }

/* Centre and width of cell idx of mesh (0 primal, 1 dual); idx outside 0..n-1
 * names a periodic image, shifted by whole periods. */
static void geom(const ora1d *p, const double *edges, int mesh, long idx, double *centre, double *width)
{
    const long n = p->n;
    const double L = p->xhi - p->xlo;
    if (mesh == 0) {
        const long i = wrap(idx, n);
        const double shift = (double)((idx - i) / n) * L;
        *centre = 0.5 * (edges[i] + edges[i + 1]) + shift;
        *width = edges[i + 1] - edges[i];
    } else {
        double cl, wl, cr, wr;
        geom(p, edges, 0, idx - 1, &cl, &wl);
        geom(p, edges, 0, idx, &cr, &wr);
        *centre = 0.5 * (cl + cr);
        *width = 0.5 * (wl + wr);
    }
}

static double coef(const ora1d *p, const double *u, long idx, int q, int m)
{
    return u[(long)(q * (p->k + 1) + m) * p->n + wrap(idx, p->n)];
}

/* d^order/dx^order of cell idx's polynomial (all components) at the point x. */
static void eval_at(const ora1d *p, const double *edges, const double *u, int mesh, long idx, int order, double x,
                    double *out)
{
    double c, w;
    geom(p, edges, mesh, idx, &c, &w);
    const double xi = 2.0 * (x - c) / w, scale = pow(2.0 / w, order);
    for (int q = 0; q < p->nc; ++q) {
        double v = 0.0;
        for (int m = 0; m <= p->k; ++m) v += coef(p, u, idx, q, m) * ora_legendre_deriv(m, order, xi);
        out[q] = scale * v;
    }
}

static void flux1d(const ora1d *p, const double *w, double *f)
{
    if (p->flux == FLUX_ADVECTION) {
        f[0] = p->a * w[0];
    } else if (p->flux == FLUX_BURGERS) {
        f[0] = 0.5 * w[0] * w[0];
    } else {
        const double v = w[1] / w[0], pr = (p->gamma - 1.0) * (w[2] - 0.5 * w[1] * v);
        f[0] = w[1];
        f[1] = w[1] * v + pr;
        f[2] = (w[2] + pr) * v;
    }
}

/* The two pieces of cell i (0 <= i < n) of mesh: [lo, split] overlaps cell
 * *nl of the other mesh, [split, hi] overlaps cell *nr. */
static void pieces(const ora1d *p, const double *edges, int mesh, long i, double *lo, double *split, double *hi,
                   long *nl, long *nr)
{
    double c, w;
    if (mesh == 0) {                   /* dual cells i and i+1 meet at the primal centre */
        geom(p, edges, 0, i, &c, &w);
        *lo = edges[i];
        *hi = edges[i + 1];
        *split = c;
        *nl = i;
        *nr = i + 1;
    } else {                           /* primal cells i-1 and i meet at the edge x_{i-1/2} */
        double wl;
        geom(p, edges, 0, i - 1, lo, &wl);
        geom(p, edges, 0, i, hi, &w);
        *split = edges[i];
        *nl = i - 1;
        *nr = i;
    }
}

/* Time derivative of the modal coefficients on both meshes from eq:1D_H:
 *   (w_K/(2m+1)) da_m/dt = (1/tau_max) int_K (v - u_K) P_m dx + int_K f(v) dP_m/dx dx
 *                          - [ f(v) P_m ]_{left end}^{right end},
 * v the other mesh's solution. */
int ora1n_rhs(const ora1d *p, const double *edges, double tau_max, const double *uC, const double *uD, double *LC,
              double *LD)
{
    int rc = check_mesh(p, edges);
    if (rc != ORA_OK) return rc;
    const int k = p->k, K1 = k + 1, Q = k + 1, nc = p->nc;
    const long n = p->n;
    double s[16], wq[16], v[3], uk[3], fv[3], fl[3], fr[3];
    ora_gauss_legendre(Q, s, wq);
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *own = mesh == 0 ? uC : uD, *oth = mesh == 0 ? uD : uC;
        double *out = mesh == 0 ? LC : LD;
        for (long i = 0; i < n; ++i) {
            double c, w, lo, split, hi;
            long nl, nr;
            geom(p, edges, mesh, i, &c, &w);
            pieces(p, edges, mesh, i, &lo, &split, &hi, &nl, &nr);
            double R[3][8];
            for (int q = 0; q < nc; ++q)
                for (int m = 0; m <= k; ++m) R[q][m] = 0.0;
            for (int piece = 0; piece < 2; ++piece) {
                const double a = piece == 0 ? lo : split, b = piece == 0 ? split : hi;
                const long nb = piece == 0 ? nl : nr;
                for (int g = 0; g < Q; ++g) {
                    const double x = 0.5 * (a + b) + 0.5 * (b - a) * s[g], jac = 0.5 * (b - a) * wq[g];
                    const double xi = 2.0 * (x - c) / w;
                    eval_at(p, edges, oth, 1 - mesh, nb, 0, x, v);
                    eval_at(p, edges, own, mesh, i, 0, x, uk);
                    flux1d(p, v, fv);
                    for (int q = 0; q < nc; ++q)
                        for (int m = 0; m <= k; ++m)
                            R[q][m] += jac * ((v[q] - uk[q]) / tau_max * ora_legendre_deriv(m, 0, xi)
                                              + fv[q] * (2.0 / w) * ora_legendre_deriv(m, 1, xi));
                }
            }
            eval_at(p, edges, oth, 1 - mesh, nl, 0, lo, v);
            flux1d(p, v, fl);
            eval_at(p, edges, oth, 1 - mesh, nr, 0, hi, v);
            flux1d(p, v, fr);
            for (int q = 0; q < nc; ++q)
                for (int m = 0; m <= k; ++m) {
                    const double sgn = (m % 2 == 0) ? 1.0 : -1.0;       /* P_m(-1); P_m(1) = 1 */
                    out[(long)(q * K1 + m) * n + i] = (2.0 * m + 1.0) / w * (R[q][m] - (fr[q] - fl[q] * sgn));
                }
        }
    }
    return ORA_OK;
}

/* avg(u^M_q) = (1/|Omega|) int u^M_q = sum_K w_K (cell average) / sum_K w_K;
 * sigma = max |u^M_q - avg| over the end points and the quadrature nodes of
 * both pieces of every cell.  avg/sigma: [mesh][q] with 3 slots per mesh. */
int ora1n_stats(const ora1d *p, const double *edges, const double *uC, const double *uD, double *avg, double *sigma)
{
    int rc = check_mesh(p, edges);
    if (rc != ORA_OK) return rc;
    const int Q = p->k + 1;
    double s[16], wq[16], v[3];
    ora_gauss_legendre(Q, s, wq);
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *u = mesh == 0 ? uC : uD;
        for (int q = 0; q < p->nc; ++q) {
            double sum = 0.0, tot = 0.0;
            for (long i = 0; i < p->n; ++i) {
                double c, w;
                geom(p, edges, mesh, i, &c, &w);
                sum += w * coef(p, u, i, q, 0);
                tot += w;
            }
            avg[mesh * 3 + q] = sum / tot;
            sigma[mesh * 3 + q] = 0.0;
        }
        for (long i = 0; i < p->n; ++i) {
            double lo, split, hi, xs[40];
            long nl, nr;
            pieces(p, edges, mesh, i, &lo, &split, &hi, &nl, &nr);
            int np = 0;
            xs[np++] = lo;
            for (int g = 0; g < Q; ++g) xs[np++] = 0.5 * (lo + split) + 0.5 * (split - lo) * s[g];
            for (int g = 0; g < Q; ++g) xs[np++] = 0.5 * (split + hi) + 0.5 * (hi - split) * s[g];
            xs[np++] = hi;
            for (int j = 0; j < np; ++j) {
                eval_at(p, edges, u, mesh, i, 0, xs[j], v);
                for (int q = 0; q < p->nc; ++q) {
                    const double d = fabs(v[q] - avg[mesh * 3 + q]);
                    if (d > sigma[mesh * 3 + q]) sigma[mesh * 3 + q] = d;
                }
            }
        }
    }
    return ORA_OK;
}

/* delta_K^m = max_q sum_{e = ends of K} beta_K (2m+1) w_K^{m-1} / ((2k-1) m! sigma_q)
 *             | d^m/dx^m (u_K - v)_q (e) |,
 * v the other mesh's cell holding e (each side with its own width in the
 * chain rule), beta_K the spectral radius at K's cell average, 0 where
 * sigma_q = 0.  dC, dD: [m*n + i]. */
int ora1n_delta(const ora1d *p, const double *edges, const double *uC, const double *uD, double *dC, double *dD)
{
    double avg[6], sigma[6], ubar[3], oL[3], oR[3], vL[3], vR[3];
    int rc = ora1n_stats(p, edges, uC, uD, avg, sigma);
    if (rc != ORA_OK) return rc;
    const int k = p->k;
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *own = mesh == 0 ? uC : uD, *oth = mesh == 0 ? uD : uC;
        double *d = mesh == 0 ? dC : dD;
        for (long i = 0; i < p->n; ++i) {
            double c, w, lo, split, hi, fact = 1.0;
            long nl, nr;
            geom(p, edges, mesh, i, &c, &w);
            pieces(p, edges, mesh, i, &lo, &split, &hi, &nl, &nr);
            for (int q = 0; q < p->nc; ++q) ubar[q] = coef(p, own, i, q, 0);
            const double beta = ora1d_wavespeed(p, ubar);
            for (int m = 0; m <= k; ++m) {
                if (m > 1) fact *= m;
                eval_at(p, edges, own, mesh, i, m, lo, oL);
                eval_at(p, edges, own, mesh, i, m, hi, oR);
                eval_at(p, edges, oth, 1 - mesh, nl, m, lo, vL);
                eval_at(p, edges, oth, 1 - mesh, nr, m, hi, vR);
                const double cm = (2.0 * m + 1.0) * pow(w, m - 1) / ((2.0 * k - 1.0) * fact);
                double dm = 0.0;
                for (int q = 0; q < p->nc; ++q) {
                    if (sigma[mesh * 3 + q] == 0.0) continue;
                    const double val = cm * beta * (fabs(oL[q] - vL[q]) + fabs(oR[q] - vR[q])) / sigma[mesh * 3 + q];
                    if (val > dm) dm = val;
                }
                d[(long)m * p->n + i] = dm;
            }
        }
    }
    return ORA_OK;
}

/* F_tau: mode j >= 1 of every cell decays by exp(-tau sum_{m<=j} delta^m);
 * the cell averages are untouched.  In place on both meshes. */
int ora1n_oe(const ora1d *p, const double *edges, double tau, double *uC, double *uD)
{
    const int k = p->k, K1 = k + 1;
    const long n = p->n;
    if (k < 1) return check_mesh(p, edges);
    double *dC = malloc(sizeof(double) * K1 * n), *dD = malloc(sizeof(double) * K1 * n);
    if (!dC || !dD) { free(dC); free(dD); return ORA_ENOMEM; }
    int rc = ora1n_delta(p, edges, uC, uD, dC, dD);
    for (int mesh = 0; mesh < 2 && rc == ORA_OK; ++mesh) {
        double *u = mesh == 0 ? uC : uD, *d = mesh == 0 ? dC : dD;
        for (long i = 0; i < n; ++i)
            for (int j = 1; j <= k; ++j) {
                double S = 0.0;
                for (int m = 0; m <= j; ++m) S += d[(long)m * n + i];
                const double fac = exp(-tau * S);
                for (int q = 0; q < p->nc; ++q) u[(long)(q * K1 + j) * n + i] *= fac;
            }
    }
    free(dC);
    free(dD);
    return rc;
}

static int check_state(const ora1d *p, const double *u)
{
    const long sz = (long)p->nc * (p->k + 1) * p->n;
    for (long e = 0; e < sz; ++e)
        if (!isfinite(u[e])) return ORA_ENONFINITE;
    if (p->flux == FLUX_EULER)
        for (long i = 0; i < p->n; ++i) {
            const double rho = u[i], mom = u[(long)(p->k + 1) * p->n + i], E = u[(long)2 * (p->k + 1) * p->n + i];
            if (!(rho > 0.0) || !((p->gamma - 1.0) * (E - 0.5 * mom * mom / rho) > 0.0)) return ORA_ENONPHYSICAL;
        }
    return ORA_OK;
}

/* One RK-OECDG step (eq:RKCDG) of size tau; (uC, uD) holds u_sigma^n on entry
 * and u_sigma^{n+1} on exit. */
int ora1n_step(const ora1d *p, const double *edges, int rk, int oe, double tau, double tau_max, double *uC,
               double *uD)
{
    double c[4][4], d[4][4];
    const int s = ora_rk_table(rk, c, d);
    if (s == 0) return ORA_EINVAL;
    int rc = check_mesh(p, edges);
    if (rc != ORA_OK) return rc;
    const long sz1 = (long)p->nc * (p->k + 1) * p->n, sz = 2 * sz1;
    double *us = malloc(sizeof(double) * sz * (s + 1)), *Ls = malloc(sizeof(double) * sz * s);
    if (!us || !Ls) { free(us); free(Ls); return ORA_ENOMEM; }
    memcpy(us, uC, sizeof(double) * sz1);
    memcpy(us + sz1, uD, sizeof(double) * sz1);
    for (int l = 0; l < s && rc == ORA_OK; ++l) {
        double *ul = us + sz * l, *un = us + sz * (l + 1);
        rc = ora1n_rhs(p, edges, tau_max, ul, ul + sz1, Ls + sz * l, Ls + sz * l + sz1);
        for (long e = 0; e < sz; ++e) {
            double v = 0.0;
            for (int m = 0; m <= l; ++m) v += c[l][m] * us[sz * m + e] + tau * d[l][m] * Ls[sz * m + e];
            un[e] = v;
        }
        if (oe && rc == ORA_OK) rc = ora1n_oe(p, edges, tau, un, un + sz1);
        if (rc == ORA_OK) rc = check_state(p, un);
        if (rc == ORA_OK) rc = check_state(p, un + sz1);
    }
    if (rc == ORA_OK) {
        memcpy(uC, us + sz * s, sizeof(double) * sz1);
        memcpy(uD, us + sz * s + sz1, sizeof(double) * sz1);
    }
    free(us);
    free(Ls);
    return rc;
}

/* March to t_end (last step clipped) or nsteps steps (< 0: no limit) with
 * tau = tau_max = C_CFL h / beta, h the largest primal width and beta the
 * largest wave speed at a cell average of either mesh; dt_fixed > 0 replaces
 * it.  A clipped last step keeps tau_max. */
int ora1n_run(const ora1d *p, const double *edges, double cfl, int rk, int oe, double t_end, long nsteps,
              double dt_fixed, double *uC, double *uD, double *t_out, long *steps_out)
{
    int rc = check_mesh(p, edges);
    double hmax = 0.0, t = 0.0, ubar[3];
    long step = 0;
    if (rc == ORA_OK) {
        for (long i = 0; i < p->n; ++i) hmax = fmax(hmax, edges[i + 1] - edges[i]);
        rc = check_state(p, uC);
        if (rc == ORA_OK) rc = check_state(p, uD);
    }
    while (rc == ORA_OK && t < t_end && (nsteps < 0 || step < nsteps)) {
        double tau_max = dt_fixed;
        if (!(dt_fixed > 0.0)) {
            double beta = 0.0;
            for (int mesh = 0; mesh < 2; ++mesh)
                for (long i = 0; i < p->n; ++i) {
                    for (int q = 0; q < p->nc; ++q) ubar[q] = coef(p, mesh == 0 ? uC : uD, i, q, 0);
                    const double b = ora1d_wavespeed(p, ubar);
                    if (!(b <= beta)) beta = b;
                }
            if (!(beta > 0.0) || !isfinite(beta)) { rc = ORA_EINVAL; break; }
            tau_max = cfl * hmax / beta;
        }
        double tau = tau_max;
        int last = 0;
        if (t + tau >= t_end) { tau = t_end - t; last = 1; }
        rc = ora1n_step(p, edges, rk, oe, tau, tau_max, uC, uD);
        t = last ? t_end : t + tau;
        ++step;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = step;
    return rc;
}
