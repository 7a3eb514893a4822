/*
 * oecdg_oracle_2d.c -- plain, serial FP64 CPU oracle of the 2D OECDG method on
 * uniform periodic Cartesian primal and dual meshes (arXiv 2503.12473, Sec. 2).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the product path never does.  It
 * shares no source, header, table or helper with the HIP implementation.
 *
 * Transcribed from the paper's definitions:
 *   - the 2D bilinear form eq. (eq:2D_H): the 1/tau_max coupling over the whole
 *     cell, the volume integral of f(w) . grad(phi), and the edge terms in which
 *     f_1 (f_2) of the other mesh is taken on its vertical (horizontal) centre
 *     lines, which are the edges of this cell;
 *   - tau_max = C_CFL / (max|f_1'|/h_x + max|f_2'|/h_y) (Sec. 2.1);
 *   - RK-OECDG in c/d form (eq:RKCDG) with the OE step after every stage;
 *   - the damping ODE (OEstep2D) with delta_K^m summed over the four edges of
 *     K, the m-th order derivative norm of the primal/dual difference
 *     integrated along each edge, h_{e,K} = distance across K normal to e,
 *     beta_{e,K} = spectral radius of the normal flux Jacobian at K's cell
 *     average, sigma_K = the L-infinity distance from the domain average, and
 *     the maximum over components for systems (Sec. 2.2 and its remarks).
 * Readings where the paper leaves a choice:
 *   - the space is the tensor product Q^k (modes P_a(xi) P_b(eta), a, b <= k)
 *     or, with space = 1, the paper's own P^k (total degree a + b <= k, Sec.
 *     2.1): the products of Legendre polynomials are L2-orthogonal on a cell,
 *     so the P^k Galerkin equations are the Q^k ones for the modes a + b <= k
 *     and every stage's combination is truncated to those modes (the layout
 *     keeps all (k+1)^2 slots, the others zero);
 *     P^{m-1} u keeps the modes of total degree a + b <= m - 1, so mode (a,b)
 *     decays with rate sum_{m=0}^{min(a+b,k)} delta^m, mode (0,0) not at all;
 *   - integrals: Gauss-Legendre with k+1 nodes per direction on each quadrant
 *     of a cell (volume) and on each half of an edge (edge terms and the edge
 *     integrals in delta): the other mesh is smooth on each piece;
 *   - sigma is sampled at the tensor product of {-1, the half-cell nodes, +1};
 *   - tau_max uses the largest |f_1'| and |f_2'| over the cell averages of
 *     both meshes.
 *
 * Data layout: coefficient (a, b) of component q of cell (ix, iy) is
 * u[(((q*(k+1) + a)*(k+1) + b)*ny + iy)*nx + ix], a the x mode, b the y mode,
 * unnormalised Legendre P_a(xi) P_b(eta).  Primal cell (ix, iy) is
 * [xlo + ix hx, xlo + (ix+1) hx] x [ylo + iy hy, ylo + (iy+1) hy]; dual cell
 * (ix, iy) is centred on its lower-left vertex (xlo + ix hx, ylo + iy hy).
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_ENONFINITE = -4, ORA_ENONPHYSICAL = -5 };
enum { FLUX_ADVECTION = 0, FLUX_EULER = 2 };

double ora_legendre(int n, double x);
double ora_legendre_deriv(int n, int m, double x);
void ora_gauss_legendre(int Q, double *s, double *w);
int ora_rk_table(int rk, double c[4][4], double d[4][4]);

typedef struct {
    int k;          /* degree in each direction */
    int nc;         /* components: 1 (advection) or 4 (Euler) */
    int flux;       /* FLUX_ADVECTION or FLUX_EULER */
    long nx, ny;    /* cells per direction (both meshes) */
    double xlo, xhi, ylo, yhi;
    double ax, ay;  /* advection velocity */
    double gamma;
    int space;      /* 0: tensor Q^k, 1: total degree P^k */
} ora2d;

#define KMAX 3
#define QMAX (KMAX + 1)
#define NCMAX 4

static double hx_of(const ora2d *p) { return (p->xhi - p->xlo) / (double)p->nx; }
static double hy_of(const ora2d *p) { return (p->yhi - p->ylo) / (double)p->ny; }
static long wrap(long i, long n) { return ((i % n) + n) % n; }

static double coef2(const ora2d *p, const double *u, long ix, long iy, int q, int a, int b)
{
    const int K1 = p->k + 1;
    ix = wrap(ix, p->nx);
    iy = wrap(iy, p->ny);
    return u[((((long)q * K1 + a) * K1 + b) * p->ny + iy) * p->nx + ix];
}

/* P_n^(d)(x) for the few distinct arguments the oracle uses (quadrature
 * nodes, their shifts, 0, +-1, sample points), memoised by the exact value of
 * x: the same numbers as calling ora_legendre_deriv each time. */
static double leg_cached(int n, int d, double x)
{
    enum { NX = 128 };
    static double xs[NX], val[NX][KMAX + 1][KMAX + 1];
    static int count = 0;
    static int last = 0;
    int i = (last < count && xs[last] == x) ? last : 0;
    while (i < count && xs[i] != x) ++i;
    last = i;
    if (i == count) {
        if (count == NX) return ora_legendre_deriv(n, d, x);
        xs[i] = x;
        for (int nn = 0; nn <= KMAX; ++nn)
            for (int dd = 0; dd <= KMAX; ++dd) val[i][nn][dd] = ora_legendre_deriv(nn, dd, x);
        ++count;
    }
    return val[i][n][d];
}

/* Value of component q of cell (ix, iy) of u, derivative order (da, db) in
 * the reference coordinates, at (xi, eta). */
static double eval2(const ora2d *p, const double *u, long ix, long iy, int q, int da, int db, double xi, double eta)
{
    const int K1 = p->k + 1;
    const long plane = p->nx * p->ny;
    const long c = wrap(iy, p->ny) * p->nx + wrap(ix, p->nx);
    double bx[KMAX + 1], by[KMAX + 1];
    for (int a = 0; a <= p->k; ++a) bx[a] = leg_cached(a, da, xi);
    for (int b = 0; b <= p->k; ++b) by[b] = leg_cached(b, db, eta);
    double v = 0.0;
    for (int a = 0; a <= p->k; ++a)
        for (int b = 0; b <= p->k; ++b)
            v += u[(((long)q * K1 + a) * K1 + b) * plane + c] * bx[a] * by[b];
    return v;
}

/* The other-mesh cell overlapping half s (0 = low side, 1 = high side) of
 * cell i of mesh M along one direction, and the shift from this cell's
 * reference coordinate to that cell's. */
static long other_index(int mesh, long i, int s) { return mesh == 0 ? i + s : i - 1 + s; }
static double other_shift(int s) { return s == 0 ? 1.0 : -1.0; }

static double factorial(int m)
{
    double f = 1.0;
    for (int j = 2; j <= m; ++j) f *= j;
    return f;
}

/* ------------------------------------------------------------------------ */
/* Flux and wave speeds                                                       */
/* ------------------------------------------------------------------------ */

/* f_dir(w), dir 0 = x, 1 = y. */
static void flux2d(const ora2d *p, int dir, const double *w, double *f)
{
    if (p->flux == FLUX_ADVECTION) {
        f[0] = (dir == 0 ? p->ax : p->ay) * w[0];
        return;
    }
    double rho = w[0], mx = w[1], my = w[2], E = w[3];
    double u = mx / rho, v = my / rho;
    double pr = (p->gamma - 1.0) * (E - 0.5 * (mx * u + my * v));
    if (dir == 0) {
        f[0] = mx;
        f[1] = mx * u + pr;
        f[2] = my * u;
        f[3] = (E + pr) * u;
    } else {
        f[0] = my;
        f[1] = mx * v;
        f[2] = my * v + pr;
        f[3] = (E + pr) * v;
    }
}

/* Spectral radius of the Jacobian of f_dir at a state. */
double ora2d_wavespeed(const ora2d *p, int dir, const double *ubar)
{
    if (p->flux == FLUX_ADVECTION) return fabs(dir == 0 ? p->ax : p->ay);
    double rho = ubar[0], mx = ubar[1], my = ubar[2], E = ubar[3];
    double u = mx / rho, v = my / rho;
    double pr = (p->gamma - 1.0) * (E - 0.5 * (mx * u + my * v));
    return fabs(dir == 0 ? u : v) + sqrt(p->gamma * pr / rho);
}

static int physical(const ora2d *p, const double *ubar)
{
    if (p->flux != FLUX_EULER) return 1;
    double rho = ubar[0], mx = ubar[1], my = ubar[2], E = ubar[3];
    if (!(rho > 0.0)) return 0;
    double pr = (p->gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho);
    return pr > 0.0;
}

/* ------------------------------------------------------------------------ */
/* CDG spatial operator (eq:2D_H)                                             */
/* ------------------------------------------------------------------------ */

/* Time derivative of the modal coefficients of every cell of both meshes:
 *   (hx hy / ((2a+1)(2b+1))) dc_ab/dt
 *     = (1/tau_max) int_K (w - u_K) phi_ab
 *       + int_K f_1(w) d/dx phi_ab + f_2(w) d/dy phi_ab
 *       - int_{east} f_1(w) phi_ab dy + int_{west} f_1(w) phi_ab dy
 *       - int_{north} f_2(w) phi_ab dx + int_{south} f_2(w) phi_ab dx
 * with w the other mesh's solution: smooth on each quadrant of K, and
 * continuous across K's edges, which are the other mesh's centre lines. */
int ora2d_rhs(const ora2d *p, double tau_max, const double *uC, const double *uD, double *LC, double *LD)
{
    const int k = p->k, K1 = k + 1, Q = k + 1, nc = p->nc;
    const double hx = hx_of(p), hy = hy_of(p);
    const long nx = p->nx, ny = p->ny;
    double s[QMAX], wq[QMAX];
    if (k < 0 || k > KMAX || (nc != 1 && nc != 4)) return ORA_EINVAL;
    ora_gauss_legendre(Q, s, wq);
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *own = mesh == 0 ? uC : uD, *oth = mesh == 0 ? uD : uC;
        double *out = mesh == 0 ? LC : LD;
        for (long iy = 0; iy < ny; ++iy)
            for (long ix = 0; ix < nx; ++ix) {
                double R[NCMAX][QMAX][QMAX];
                memset(R, 0, sizeof(R));
                double w[NCMAX], uk[NCMAX], f1[NCMAX], f2[NCMAX];
                /* coupling and volume over the four quadrants */
                for (int sx = 0; sx < 2; ++sx)
                    for (int sy = 0; sy < 2; ++sy) {
                        long ox = other_index(mesh, ix, sx), oy = other_index(mesh, iy, sy);
                        for (int gp = 0; gp < Q; ++gp)
                            for (int gq = 0; gq < Q; ++gq) {
                                double xi = sx == 0 ? 0.5 * (s[gp] - 1.0) : 0.5 * (s[gp] + 1.0);
                                double eta = sy == 0 ? 0.5 * (s[gq] - 1.0) : 0.5 * (s[gq] + 1.0);
                                double xo = xi + other_shift(sx), yo = eta + other_shift(sy);
                                double wt = hx * hy / 16.0 * wq[gp] * wq[gq];
                                for (int q = 0; q < nc; ++q) {
                                    w[q] = eval2(p, oth, ox, oy, q, 0, 0, xo, yo);
                                    uk[q] = eval2(p, own, ix, iy, q, 0, 0, xi, eta);
                                }
                                flux2d(p, 0, w, f1);
                                flux2d(p, 1, w, f2);
                                double Pa[KMAX + 1], dPa[KMAX + 1], Pb[KMAX + 1], dPb[KMAX + 1];
                                for (int j = 0; j <= k; ++j) {
                                    Pa[j] = leg_cached(j, 0, xi);
                                    dPa[j] = leg_cached(j, 1, xi);
                                    Pb[j] = leg_cached(j, 0, eta);
                                    dPb[j] = leg_cached(j, 1, eta);
                                }
                                for (int q = 0; q < nc; ++q)
                                    for (int a = 0; a <= k; ++a)
                                        for (int b = 0; b <= k; ++b) {
                                            double phi = Pa[a] * Pb[b];
                                            double phx = (2.0 / hx) * dPa[a] * Pb[b];
                                            double phy = (2.0 / hy) * Pa[a] * dPb[b];
                                            R[q][a][b] += wt * ((w[q] - uk[q]) * phi / tau_max + f1[q] * phx + f2[q] * phy);
                                        }
                            }
                    }
                /* east / west edges (xi = +1 / -1): f_1 of the other mesh on its
                 * vertical centre line, two half-edges */
                for (int side = 0; side < 2; ++side)
                    for (int sy = 0; sy < 2; ++sy) {
                        long ox = other_index(mesh, ix, side), oy = other_index(mesh, iy, sy);
                        double sgn_out = side == 1 ? 1.0 : -1.0;          /* outward normal x-component */
                        double xi_e = side == 1 ? 1.0 : -1.0;
                        for (int g = 0; g < Q; ++g) {
                            double eta = sy == 0 ? 0.5 * (s[g] - 1.0) : 0.5 * (s[g] + 1.0);
                            for (int q = 0; q < nc; ++q) w[q] = eval2(p, oth, ox, oy, q, 0, 0, 0.0, eta + other_shift(sy));
                            flux2d(p, 0, w, f1);
                            double wt = hy / 4.0 * wq[g];
                            for (int q = 0; q < nc; ++q)
                                for (int a = 0; a <= k; ++a)
                                    for (int b = 0; b <= k; ++b)
                                        R[q][a][b] -= wt * sgn_out * f1[q] * leg_cached(a, 0, xi_e) * leg_cached(b, 0, eta);
                        }
                    }
                /* north / south edges (eta = +1 / -1): f_2 on horizontal centre lines */
                for (int side = 0; side < 2; ++side)
                    for (int sx = 0; sx < 2; ++sx) {
                        long ox = other_index(mesh, ix, sx), oy = other_index(mesh, iy, side);
                        double sgn_out = side == 1 ? 1.0 : -1.0;
                        double eta_e = side == 1 ? 1.0 : -1.0;
                        for (int g = 0; g < Q; ++g) {
                            double xi = sx == 0 ? 0.5 * (s[g] - 1.0) : 0.5 * (s[g] + 1.0);
                            for (int q = 0; q < nc; ++q) w[q] = eval2(p, oth, ox, oy, q, 0, 0, xi + other_shift(sx), 0.0);
                            flux2d(p, 1, w, f2);
                            double wt = hx / 4.0 * wq[g];
                            for (int q = 0; q < nc; ++q)
                                for (int a = 0; a <= k; ++a)
                                    for (int b = 0; b <= k; ++b)
                                        R[q][a][b] -= wt * sgn_out * f2[q] * leg_cached(a, 0, xi) * leg_cached(b, 0, eta_e);
                        }
                    }
                for (int q = 0; q < nc; ++q)
                    for (int a = 0; a <= k; ++a)
                        for (int b = 0; b <= k; ++b)
                            out[((((long)q * K1 + a) * K1 + b) * ny + iy) * nx + ix] =
                                (2.0 * a + 1.0) * (2.0 * b + 1.0) / (hx * hy) * R[q][a][b];
            }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* OE step                                                                    */
/* ------------------------------------------------------------------------ */

/* Reference points of one direction where sigma is sampled: -1, the k+1
 * Gauss nodes of each half, +1.  Returns the count. */
static int sample_points(int k, double *xs)
{
    const int Q = k + 1;
    double s[QMAX], wq[QMAX];
    ora_gauss_legendre(Q, s, wq);
    int c = 0;
    xs[c++] = -1.0;
    for (int g = 0; g < Q; ++g) xs[c++] = 0.5 * (s[g] - 1.0);
    for (int g = 0; g < Q; ++g) xs[c++] = 0.5 * (s[g] + 1.0);
    xs[c++] = 1.0;
    return c;
}

/* avg[mesh*4+q] = mean of the cell averages of mesh; sigma[mesh*4+q] = max
 * |u_q - avg| over the sample points of every cell of that mesh. */
void ora2d_stats(const ora2d *p, const double *uC, const double *uD, double *avg, double *sigma)
{
    double xs[2 * QMAX + 2];
    int np = sample_points(p->k, xs);
    const long ncell = p->nx * p->ny;
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *u = mesh == 0 ? uC : uD;
        for (int q = 0; q < p->nc; ++q) {
            double sum = 0.0;
            for (long iy = 0; iy < p->ny; ++iy)
                for (long ix = 0; ix < p->nx; ++ix) sum += coef2(p, u, ix, iy, q, 0, 0);
            avg[mesh * 4 + q] = sum / (double)ncell;
            double sg = 0.0;
            for (long iy = 0; iy < p->ny; ++iy)
                for (long ix = 0; ix < p->nx; ++ix)
                    for (int i = 0; i < np; ++i)
                        for (int j = 0; j < np; ++j) {
                            double d = fabs(eval2(p, u, ix, iy, q, 0, 0, xs[i], xs[j]) - avg[mesh * 4 + q]);
                            if (d > sg) sg = d;
                        }
            sigma[mesh * 4 + q] = sg;
        }
    }
}

/* Damping coefficients delta_K^m (m = 0..k) of every cell of both meshes,
 * from the undamped state:
 *   delta_K^m = max_q sum_{e in {W,E,S,N}} beta_{e,K} (2m+1) h_e^{m-1}
 *                 / ((2k-1) m! sigma_q) * (1/|e|) int_e
 *                 ( sum_{alpha1+alpha2=m} (d^alpha (u_K - w)_q)^2 )^{1/2} ds
 * with u_K's own trace on e, w the other mesh (smooth along each half of e,
 * e being its centre line), physical derivatives d^alpha =
 * (2/hx)^alpha1 (2/hy)^alpha2 d_xi^alpha1 d_eta^alpha2, h_e = hx for W/E and
 * hy for S/N, beta_{e,K} the spectral radius of f_1' (W/E) or f_2' (S/N) at
 * K's cell average, and the edge mean (1/|e|) int_e evaluated with k+1 Gauss
 * nodes on each half.  Components with sigma_q = 0 contribute 0.
 * dC, dD: [(m*ny + iy)*nx + ix]. */
int ora2d_delta(const ora2d *p, const double *uC, const double *uD, double *dC, double *dD)
{
    const int k = p->k, Q = k + 1, nc = p->nc;
    const double hx = hx_of(p), hy = hy_of(p);
    const long nx = p->nx, ny = p->ny;
    double avg[8], sigma[8], s[QMAX], wq[QMAX], ubar[NCMAX];
    if (k < 1) return ORA_EINVAL;
    ora2d_stats(p, uC, uD, avg, sigma);
    ora_gauss_legendre(Q, s, wq);
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *own = mesh == 0 ? uC : uD, *oth = mesh == 0 ? uD : uC;
        double *d = mesh == 0 ? dC : dD;
        for (long iy = 0; iy < ny; ++iy)
            for (long ix = 0; ix < nx; ++ix) {
                for (int q = 0; q < nc; ++q) ubar[q] = coef2(p, own, ix, iy, q, 0, 0);
                const double bx = ora2d_wavespeed(p, 0, ubar), by = ora2d_wavespeed(p, 1, ubar);
                for (int m = 0; m <= k; ++m) {
                    double best = 0.0;
                    for (int q = 0; q < nc; ++q) {
                        if (sigma[mesh * 4 + q] == 0.0) continue;
                        double total = 0.0;
                        /* edges: dir 0 = W/E (xi = -+1), dir 1 = S/N (eta = -+1) */
                        for (int dir = 0; dir < 2; ++dir)
                            for (int side = 0; side < 2; ++side) {
                                double mean = 0.0;           /* (1/|e|) int_e g ds */
                                for (int half = 0; half < 2; ++half)
                                    for (int g = 0; g < Q; ++g) {
                                        double t = half == 0 ? 0.5 * (s[g] - 1.0) : 0.5 * (s[g] + 1.0);
                                        double e = side == 1 ? 1.0 : -1.0;
                                        double xi = dir == 0 ? e : t, eta = dir == 0 ? t : e;
                                        long ox, oy;
                                        double xo, yo;
                                        if (dir == 0) {        /* the other cell centred on this vertical edge */
                                            ox = other_index(mesh, ix, side); oy = other_index(mesh, iy, half);
                                            xo = 0.0; yo = t + other_shift(half);
                                        } else {
                                            ox = other_index(mesh, ix, half); oy = other_index(mesh, iy, side);
                                            xo = t + other_shift(half); yo = 0.0;
                                        }
                                        double ss = 0.0;
                                        for (int a1 = 0; a1 <= m; ++a1) {
                                            int a2 = m - a1;
                                            double sc = pow(2.0 / hx, a1) * pow(2.0 / hy, a2);
                                            double diff = eval2(p, own, ix, iy, q, a1, a2, xi, eta) -
                                                          eval2(p, oth, ox, oy, q, a1, a2, xo, yo);
                                            ss += (sc * diff) * (sc * diff);
                                        }
                                        mean += 0.25 * wq[g] * sqrt(ss);
                                    }
                                double he = dir == 0 ? hx : hy, beta = dir == 0 ? bx : by;
                                total += beta * (2.0 * m + 1.0) * pow(he, m - 1) / ((2.0 * k - 1.0) * factorial(m)) * mean;
                            }
                        double val = total / sigma[mesh * 4 + q];
                        if (val > best) best = val;
                    }
                    d[((long)m * ny + iy) * nx + ix] = best;
                }
            }
    }
    return ORA_OK;
}

/* F_tau in place on both meshes: mode (a,b) != (0,0) is multiplied by
 * exp(-tau sum_{m=0}^{min(a+b,k)} delta^m); the deltas of both meshes are
 * computed from the undamped state first. */
int ora2d_oe(const ora2d *p, double tau, double *uC, double *uD)
{
    const int k = p->k, K1 = k + 1, nc = p->nc;
    if (k < 1) return ORA_OK;
    const long ncell = p->nx * p->ny;
    double *dC = malloc(sizeof(double) * K1 * ncell), *dD = malloc(sizeof(double) * K1 * ncell);
    if (!dC || !dD) { free(dC); free(dD); return ORA_ENOMEM; }
    ora2d_delta(p, uC, uD, dC, dD);
    for (int mesh = 0; mesh < 2; ++mesh) {
        double *u = mesh == 0 ? uC : uD, *d = mesh == 0 ? dC : dD;
        for (long c = 0; c < ncell; ++c)
            for (int a = 0; a <= k; ++a)
                for (int b = 0; b <= k; ++b) {
                    if (a + b == 0) continue;
                    int top = a + b < k ? a + b : k;
                    double S = 0.0;
                    for (int m = 0; m <= top; ++m) S += d[(long)m * ncell + c];
                    double fac = exp(-tau * S);
                    for (int q = 0; q < nc; ++q) u[(((long)q * K1 + a) * K1 + b) * ncell + c] *= fac;
                }
    }
    free(dC);
    free(dD);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Time step and RK-OECDG                                                     */
/* ------------------------------------------------------------------------ */

/* Largest |f_1'| and |f_2'| spectral radii over the cell averages of both meshes. */
void ora2d_max_wavespeeds(const ora2d *p, const double *uC, const double *uD, double *bx, double *by)
{
    double ubar[NCMAX];
    *bx = *by = 0.0;
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *u = mesh == 0 ? uC : uD;
        for (long iy = 0; iy < p->ny; ++iy)
            for (long ix = 0; ix < p->nx; ++ix) {
                for (int q = 0; q < p->nc; ++q) ubar[q] = coef2(p, u, ix, iy, q, 0, 0);
                double sx = ora2d_wavespeed(p, 0, ubar), sy = ora2d_wavespeed(p, 1, ubar);
                if (!(sx <= *bx)) *bx = sx;
                if (!(sy <= *by)) *by = sy;
            }
    }
}

static int check_state(const ora2d *p, const double *uC, const double *uD)
{
    const int K1 = p->k + 1;
    const long ncell = p->nx * p->ny;
    double ubar[NCMAX];
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double *u = mesh == 0 ? uC : uD;
        for (long e = 0; e < (long)p->nc * K1 * K1 * ncell; ++e)
            if (!isfinite(u[e])) return ORA_ENONFINITE;
        for (long c = 0; c < ncell; ++c) {
            for (int q = 0; q < p->nc; ++q) ubar[q] = u[(long)q * K1 * K1 * ncell + c];
            if (!physical(p, ubar)) return ORA_ENONPHYSICAL;
        }
    }
    return ORA_OK;
}

/* P^k space: zero the modes of total degree above k (the L2 projection onto
 * P^k in an orthogonal basis). */
static void truncate_pk(const ora2d *p, double *u)
{
    const int K1 = p->k + 1;
    const long plane = p->nx * p->ny;
    for (int q = 0; q < p->nc; ++q)
        for (int a = 0; a <= p->k; ++a)
            for (int b = 0; b <= p->k; ++b)
                if (a + b > p->k)
                    for (long e = 0; e < plane; ++e) u[(((long)q * K1 + a) * K1 + b) * plane + e] = 0.0;
}

/* One RK-OECDG step (eq:RKCDG) of size tau with coupling parameter tau_max. */
int ora2d_step(const ora2d *p, int rk, int oe, double tau, double tau_max, double *uC, double *uD)
{
    double c[4][4], d[4][4];
    int s = ora_rk_table(rk, c, d);
    if (s == 0) return ORA_EINVAL;
    const long sz1 = (long)p->nc * (p->k + 1) * (p->k + 1) * p->nx * p->ny, sz = 2 * sz1;
    double *us = malloc(sizeof(double) * sz * (s + 1)), *Ls = malloc(sizeof(double) * sz * s);
    if (!us || !Ls) { free(us); free(Ls); return ORA_ENOMEM; }
    memcpy(us, uC, sizeof(double) * sz1);
    memcpy(us + sz1, uD, sizeof(double) * sz1);
    int rc = ORA_OK;
    for (int l = 0; l < s && rc == ORA_OK; ++l) {
        double *ul = us + sz * l;
        rc = ora2d_rhs(p, tau_max, ul, ul + sz1, Ls + sz * l, Ls + sz * l + sz1);
        double *un = us + sz * (l + 1);
        for (long e = 0; e < sz; ++e) {
            double v = 0.0;
            for (int m = 0; m <= l; ++m) v += c[l][m] * us[sz * m + e] + tau * d[l][m] * Ls[sz * m + e];
            un[e] = v;
        }
        if (p->space == 1) {
            truncate_pk(p, un);
            truncate_pk(p, un + sz1);
        }
        if (oe && rc == ORA_OK) rc = ora2d_oe(p, tau, un, un + sz1);
        if (rc == ORA_OK) rc = check_state(p, un, un + sz1);
    }
    if (rc == ORA_OK) {
        memcpy(uC, us + sz * s, sizeof(double) * sz1);
        memcpy(uD, us + sz * s + sz1, sizeof(double) * sz1);
    }
    free(us);
    free(Ls);
    return rc;
}

/* One stage l of the RK table rk in the c/d form of eq:RKCDG from u_sigma^n and
 * u_sigma^{n,l}, then F_tau: out = F_tau(c_{l0} u^n + c_{ll} u^l + tau d_{ll} L(u^l)),
 * for the stages whose other c_{lm}, d_{lm} vanish (as the 1D single stage);
 * EINVAL for the others.  Under P^k the combination is truncated first, as in
 * a step. */
int ora2d_rk_stage(const ora2d *p, int rk, int l, int oe, double tau, double tau_max,
                   const double *unC, const double *unD, const double *ulC, const double *ulD,
                   double *outC, double *outD)
{
    double c[4][4], d[4][4];
    const int s = ora_rk_table(rk, c, d);
    if (s == 0 || l < 0 || l >= s) return ORA_EINVAL;
    for (int m = 0; m < l; ++m)
        if ((m > 0 && c[l][m] != 0.0) || d[l][m] != 0.0) return ORA_EINVAL;
    const long sz1 = (long)p->nc * (p->k + 1) * (p->k + 1) * p->nx * p->ny;
    double *LC = malloc(sizeof(double) * sz1), *LD = malloc(sizeof(double) * sz1);
    if (!LC || !LD) { free(LC); free(LD); return ORA_ENOMEM; }
    int rc = ora2d_rhs(p, tau_max, ulC, ulD, LC, LD);
    for (long e = 0; e < sz1; ++e) {
        if (l == 0) {   /* c_{00} multiplies u^n = u^{n,0} itself */
            outC[e] = c[0][0] * ulC[e] + tau * d[0][0] * LC[e];
            outD[e] = c[0][0] * ulD[e] + tau * d[0][0] * LD[e];
        } else {
            outC[e] = c[l][0] * unC[e] + (c[l][l] * ulC[e] + tau * d[l][l] * LC[e]);
            outD[e] = c[l][0] * unD[e] + (c[l][l] * ulD[e] + tau * d[l][l] * LD[e]);
        }
    }
    if (p->space == 1) {
        truncate_pk(p, outC);
        truncate_pk(p, outD);
    }
    if (oe && rc == ORA_OK) rc = ora2d_oe(p, tau, outC, outD);
    if (rc == ORA_OK) rc = check_state(p, outC, outD);
    free(LC);
    free(LD);
    return rc;
}

/* March until t_end (last step clipped) or nsteps steps (< 0: no limit);
 * tau_max = cfl / (bx/hx + by/hy) from u^n, or dt_fixed when positive. */
int ora2d_run(const ora2d *p, double cfl, int rk, int oe, double t_end, long nsteps, double dt_fixed,
              double *uC, double *uD, double *t_out, long *steps_out)
{
    const double hx = hx_of(p), hy = hy_of(p);
    double t = 0.0;
    long step = 0;
    int rc = check_state(p, uC, uD);
    while (rc == ORA_OK && t < t_end && (nsteps < 0 || step < nsteps)) {
        double tau_max;
        if (dt_fixed > 0.0) {
            tau_max = dt_fixed;
        } else {
            double bx, by;
            ora2d_max_wavespeeds(p, uC, uD, &bx, &by);
            double rate = bx / hx + by / hy;
            if (!(rate > 0.0) || !isfinite(rate)) { rc = ORA_EINVAL; break; }
            tau_max = cfl / rate;
        }
        double tau = tau_max;
        int last = 0;
        if (t + tau >= t_end) { tau = t_end - t; last = 1; }
        rc = ora2d_step(p, rk, oe, tau, tau_max, uC, uD);
        t = last ? t_end : t + tau;
        ++step;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = step;
    return rc;
}
