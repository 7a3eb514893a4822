/*
 * oecdg_ref.c -- the CPU oracle behind the library's C interface: every entry
 * point of the HIP library's boundary, with the prefix oecdg_ref_ and host
 * pointers, so a test can run one sequence of calls against either
 * implementation and compare.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It holds no
 * arithmetic of the method: each call checks its arguments, lays out the
 * instances of a batch and hands each instance to the oracle's own routines
 * (oecdg_oracle.c, oecdg_oracle_2d.c, oecdg_oracle_nu.c).
 *
 * The descriptor is declared here field for field like the library's (an
 * interface both sides implement; no header is shared between them).  State
 * layouts are the oracle's and the library's alike: coefficient m of component
 * q of cell i at [(q (k+1) + m) ncell + i] in 1D, [((q (k+1) + a) (k+1) + b)
 * ny nx + iy nx + ix] in 2D.  Error codes are the library's (the oracle's codes
 * coincide with them).  The execution options of the library (mode, tile,
 * graph length, grid, fold) have no meaning here and are accepted and ignored;
 * the adjoint's oracle is a separate program (oracle/adjoint_torch.py), so
 * oecdg_ref_adjoint returns EUNSUPPORTED.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum {
    REF_OK = 0, REF_EINVAL = -1, REF_ENOMEM = -2, REF_EHIP = -3, REF_ENONFINITE = -4, REF_ENONPHYSICAL = -5,
    REF_EUNSUPPORTED = -6, REF_ETIMEOUT = -7, REF_ETOOBIG = -8
};

typedef struct {
    int32_t dim, k, flux, bc;
    int64_t nx, ny;
    double xlo, xhi, ylo, yhi;
    double flux_param[2];
    double cfl;
    int32_t oe, rk, space, flags;
} oecdg_ref_desc;

/* the oracle's problem descriptions (as declared in its sources) */
typedef struct {
    int k, nc, flux, bc;
    long n;
    double xlo, xhi, a, gamma;
    int allow_negative_pressure, pad;
    double inflow[2][3];
} ora1d;

typedef struct {
    int k, nc, flux;
    long nx, ny;
    double xlo, xhi, ylo, yhi;
    double ax, ay, gamma;
    int space;
} ora2d;

long ora1d_ncell(const ora1d *p, int mesh);
double ora1d_max_wavespeed(const ora1d *p, const double *uC, const double *uD);
int ora1d_rk_stage(const ora1d *p, int rk, int l, int oe, double tau, double tau_max, const double *unC,
                   const double *unD, const double *ulC, const double *ulD, double *outC, double *outD);
int ora1d_run(const ora1d *p, double cfl, int rk, int oe, double t_end, long nsteps, double dt_fixed, double *uC,
              double *uD, double *t_out, long *steps_out);
int ora1n_run(const ora1d *p, const double *edges, double cfl, int rk, int oe, double t_end, long nsteps,
              double dt_fixed, double *uC, double *uD, double *t_out, long *steps_out);
void ora2d_max_wavespeeds(const ora2d *p, const double *uC, const double *uD, double *bx, double *by);
int ora2d_rk_stage(const ora2d *p, int rk, int l, int oe, double tau, double tau_max, const double *unC,
                   const double *unD, const double *ulC, const double *ulD, double *outC, double *outD);
int ora2d_run(const ora2d *p, double cfl, int rk, int oe, double t_end, long nsteps, double dt_fixed, double *uC,
              double *uD, double *t_out, long *steps_out);
int ora_rk_table(int rk, double c[4][4], double d[4][4]);

typedef struct oecdg_ref_handle {
    int n;                      /* instances */
    oecdg_ref_desc *d;
    int64_t *offP, *offD;       /* n + 1 offsets each */
    double (*inflow)[2][3];
    int *inflow_set;
    char msg[256];
} oecdg_ref_handle;

static int fail(oecdg_ref_handle *h, int code, const char *what)
{
    if (h) snprintf(h->msg, sizeof h->msg, "%s", what);
    return code;
}

static int ncomp(const oecdg_ref_desc *d)
{
    if (d->flux != 2) return 1;
    return d->dim == 1 ? 3 : 4;
}

static int rk_of(const oecdg_ref_desc *d) { return d->rk == 0 ? 3 : d->rk; }

/* The descriptors the library accepts, with its error codes, checked in its
 * order (include/oecdg.h: the descriptor fields and oecdg_init). */
static int check_desc(const oecdg_ref_desc *d)
{
    if (!d) return REF_EINVAL;
    if (d->dim != 1 && d->dim != 2) return REF_EINVAL;
    if (d->rk < 0 || d->rk > 4) return REF_EINVAL;
    if (d->space != 0 && d->space != 1) return REF_EINVAL;
    if (d->flags & ~1) return REF_EINVAL;
    if (d->flux < 0 || d->flux > 2) return REF_EINVAL;
    if (d->bc < 0 || d->bc > 3) return REF_EINVAL;
    if ((d->bc == 2 || d->bc == 3) && d->flux != 2) return REF_EUNSUPPORTED;   /* walls, inflow: Euler only */
    if (!(d->xhi > d->xlo) || !(d->cfl > 0.0)) return REF_EINVAL;
    if (d->flux == 2 && !(d->flux_param[0] > 1.0)) return REF_EINVAL;
    if (d->dim == 1) {
        if (d->k < 0 || d->k > 3) return REF_EINVAL;
        if (d->nx < 2 || d->nx > (1LL << 30)) return REF_EINVAL;
        if (d->ny != 1 && d->ny != 0) return REF_EINVAL;
        return REF_OK;
    }
    if (d->k < 1 || d->k > 3) return REF_EUNSUPPORTED;
    if (d->flux == 1 || d->bc != 0 || d->flags != 0) return REF_EUNSUPPORTED;
    if (d->nx < 2 || d->ny < 2 || d->nx > 65536 || d->ny > 65536) return REF_EINVAL;
    if (!(d->yhi > d->ylo)) return REF_EINVAL;
    return REF_OK;
}

int oecdg_ref_state_size(const oecdg_ref_desc *d, int64_t *n_primal, int64_t *n_dual)
{
    int rc = check_desc(d);
    if (rc != REF_OK || !n_primal || !n_dual) return rc != REF_OK ? rc : REF_EINVAL;
    const int64_t per = (int64_t)ncomp(d) * (d->k + 1);
    if (d->dim == 1) {
        *n_primal = per * d->nx;
        *n_dual = per * (d->bc == 0 ? d->nx : d->nx + 1);
    } else {
        *n_primal = *n_dual = per * (d->k + 1) * d->nx * d->ny;
    }
    return REF_OK;
}

static ora1d prob1(const oecdg_ref_handle *h, int i)
{
    const oecdg_ref_desc *d = &h->d[i];
    ora1d p;
    memset(&p, 0, sizeof p);
    p.k = d->k;
    p.nc = ncomp(d);
    p.flux = d->flux;
    p.bc = d->bc;
    p.n = (long)d->nx;
    p.xlo = d->xlo;
    p.xhi = d->xhi;
    p.a = d->flux_param[0];
    p.gamma = d->flux == 2 ? d->flux_param[0] : 1.4;
    p.allow_negative_pressure = d->flags & 1;
    memcpy(p.inflow, h->inflow[i], sizeof p.inflow);
    return p;
}

static ora2d prob2(const oecdg_ref_desc *d)
{
    ora2d p;
    memset(&p, 0, sizeof p);
    p.k = d->k;
    p.nc = ncomp(d);
    p.flux = d->flux;
    p.nx = (long)d->nx;
    p.ny = (long)d->ny;
    p.xlo = d->xlo;
    p.xhi = d->xhi;
    p.ylo = d->ylo;
    p.yhi = d->yhi;
    p.ax = d->flux_param[0];
    p.ay = d->flux_param[1];
    p.gamma = d->flux == 2 ? d->flux_param[0] : 1.4;
    p.space = d->space;
    return p;
}

void oecdg_ref_destroy(oecdg_ref_handle *h)
{
    if (!h) return;
    free(h->d);
    free(h->offP);
    free(h->offD);
    free(h->inflow);
    free(h->inflow_set);
    free(h);
}

int oecdg_ref_init(const oecdg_ref_desc *d, int32_t nbatch, void *stream, oecdg_ref_handle **out)
{
    (void)stream;                               /* host calls: nothing is enqueued */
    if (!d || !out || nbatch < 1) return REF_EINVAL;
    *out = NULL;
    for (int i = 0; i < nbatch; ++i) {           /* batches: 1D, one flux and one RK method */
        int rc = check_desc(&d[i]);
        if (rc != REF_OK) return rc;
        if (d[i].dim != d[0].dim) return REF_EINVAL;
        if (nbatch > 1 && d[i].dim != 1) return REF_EUNSUPPORTED;
        if (d[i].flux != d[0].flux || rk_of(&d[i]) != rk_of(&d[0])) return REF_EUNSUPPORTED;
    }
    oecdg_ref_handle *h = calloc(1, sizeof *h);
    if (!h) return REF_ENOMEM;
    h->n = nbatch;
    h->d = malloc(sizeof *h->d * nbatch);
    h->offP = malloc(sizeof(int64_t) * (nbatch + 1));
    h->offD = malloc(sizeof(int64_t) * (nbatch + 1));
    h->inflow = calloc(nbatch, sizeof *h->inflow);
    h->inflow_set = calloc(nbatch, sizeof(int));
    if (!h->d || !h->offP || !h->offD || !h->inflow || !h->inflow_set) {
        oecdg_ref_destroy(h);
        return REF_ENOMEM;
    }
    memcpy(h->d, d, sizeof *h->d * nbatch);
    h->offP[0] = h->offD[0] = 0;
    for (int i = 0; i < nbatch; ++i) {
        int64_t np, nd;
        oecdg_ref_state_size(&d[i], &np, &nd);
        h->offP[i + 1] = h->offP[i] + np;
        h->offD[i + 1] = h->offD[i] + nd;
    }
    *out = h;
    return REF_OK;
}

int oecdg_ref_batch_offsets(oecdg_ref_handle *h, int64_t *off_primal, int64_t *off_dual)
{
    if (!h || !off_primal || !off_dual) return REF_EINVAL;
    memcpy(off_primal, h->offP, sizeof(int64_t) * (h->n + 1));
    memcpy(off_dual, h->offD, sizeof(int64_t) * (h->n + 1));
    return REF_OK;
}

int oecdg_ref_set_option(oecdg_ref_handle *h, int32_t key, int64_t value)
{
    if (!h) return REF_EINVAL;
    if (key < 1 || key > 5) return fail(h, REF_EINVAL, "unknown option key");
    (void)value;
    return REF_OK;
}

int oecdg_ref_set_inflow(oecdg_ref_handle *h, int32_t instance, const double *left, const double *right)
{
    if (!h || !left || !right) return REF_EINVAL;
    if (instance < 0 || instance >= h->n || h->d[instance].bc != 3)
        return fail(h, REF_EINVAL, "not an inflow instance");
    for (int q = 0; q < 3; ++q) {
        h->inflow[instance][0][q] = left[q];
        h->inflow[instance][1][q] = right[q];
    }
    h->inflow_set[instance] = 1;
    return REF_OK;
}

int oecdg_ref_dt(oecdg_ref_handle *h, const double *uC, const double *uD, double *dt_out)
{
    if (!h || !uC || !uD || !dt_out) return REF_EINVAL;
    const oecdg_ref_desc *d = &h->d[0];
    if (d->dim == 1) {
        ora1d p = prob1(h, 0);
        const double beta = ora1d_max_wavespeed(&p, uC, uD);
        if (!(beta > 0.0) || !isfinite(beta)) return fail(h, REF_ENONFINITE, "wave speed is zero or not finite");
        *dt_out = d->cfl * ((d->xhi - d->xlo) / (double)d->nx) / beta;
        return REF_OK;
    }
    ora2d p = prob2(d);
    double bx, by;
    ora2d_max_wavespeeds(&p, uC, uD, &bx, &by);
    const double rate = bx / ((d->xhi - d->xlo) / (double)d->nx) + by / ((d->yhi - d->ylo) / (double)d->ny);
    if (!(rate > 0.0) || !isfinite(rate)) return fail(h, REF_ENONFINITE, "wave speed is zero or not finite");
    *dt_out = d->cfl / rate;
    return REF_OK;
}

int oecdg_ref_stage(oecdg_ref_handle *h, int32_t stage, double dt, double tau_max, const double *uC_n,
                    const double *uD_n, const double *uC_l, const double *uD_l, double *uC_out, double *uD_out)
{
    if (!h || !uC_n || !uD_n || !uC_out || !uD_out) return REF_EINVAL;
    double c[4][4], dd[4][4];
    const int rk = rk_of(&h->d[0]), ns = ora_rk_table(rk, c, dd);
    if (stage < 0 || stage >= ns) return fail(h, REF_EINVAL, "stage out of range for the RK method");
    if (rk == 4 && stage == 3) return fail(h, REF_EUNSUPPORTED, "the last stage of classical RK4 reads the earlier stages");
    if (!(dt > 0.0) || !(tau_max > 0.0)) return fail(h, REF_EINVAL, "dt and tau_max must be positive");
    if (stage > 0 && (!uC_l || !uD_l)) return fail(h, REF_EINVAL, "stages after the first need u_l");
    if (h->n != 1) return fail(h, REF_EUNSUPPORTED, "single-instance handles only");
    const double *lC = stage == 0 ? uC_n : uC_l, *lD = stage == 0 ? uD_n : uD_l;
    int rc;
    if (h->d[0].dim == 1) {
        ora1d p = prob1(h, 0);
        rc = ora1d_rk_stage(&p, rk, stage, h->d[0].oe, dt, tau_max, uC_n, uD_n, lC, lD, uC_out, uD_out);
    } else {
        ora2d p = prob2(&h->d[0]);
        rc = ora2d_rk_stage(&p, rk, stage, h->d[0].oe, dt, tau_max, uC_n, uD_n, lC, lD, uC_out, uD_out);
    }
    return rc == REF_OK ? rc : fail(h, rc, "oracle stage failed");
}

int oecdg_ref_run(oecdg_ref_handle *h, double *uC, double *uD, double t_end, int64_t nsteps, double dt_fixed,
                  double *t_out, int64_t *steps_out)
{
    if (!h || !uC || !uD) return REF_EINVAL;
    if (nsteps < 0 && !(t_end < INFINITY)) return fail(h, REF_EINVAL, "run needs a finite t_end or nsteps >= 0");
    if (!(t_end > 0.0)) return fail(h, REF_EINVAL, "t_end must be positive");
    for (int i = 0; i < h->n; ++i)
        if (h->d[i].bc == 3 && !h->inflow_set[i]) return fail(h, REF_EINVAL, "inflow states not set");
    for (int i = 0; i < h->n; ++i) {
        const oecdg_ref_desc *d = &h->d[i];
        double t = 0.0;
        long s = 0;
        int rc;
        if (d->dim == 1) {
            ora1d p = prob1(h, i);
            rc = ora1d_run(&p, d->cfl, rk_of(d), d->oe, t_end, (long)nsteps, dt_fixed, uC + h->offP[i],
                           uD + h->offD[i], &t, &s);
        } else {
            ora2d p = prob2(d);
            rc = ora2d_run(&p, d->cfl, rk_of(d), d->oe, t_end, (long)nsteps, dt_fixed, uC, uD, &t, &s);
        }
        if (i == 0) {
            if (t_out) *t_out = t;
            if (steps_out) *steps_out = s;
        }
        if (rc != REF_OK) return fail(h, rc, "oracle run failed");
    }
    return REF_OK;
}

int oecdg_ref_run_noalloc(const oecdg_ref_desc *d, void *stream, double *uC, double *uD, double t_end,
                          int64_t nsteps, double dt_fixed, double *t_out, int64_t *steps_out)
{
    if (!d) return REF_EINVAL;
    if (d->dim != 1) return check_desc(d) == REF_OK ? REF_EUNSUPPORTED : check_desc(d);
    oecdg_ref_handle *h = NULL;
    int rc = oecdg_ref_init(d, 1, stream, &h);
    if (rc == REF_OK) rc = oecdg_ref_run(h, uC, uD, t_end, nsteps, dt_fixed, t_out, steps_out);
    oecdg_ref_destroy(h);
    return rc;
}

int oecdg_ref_run_nonuniform(oecdg_ref_handle *h, const double *edges, double *uC, double *uD, double t_end,
                             int64_t nsteps, double dt_fixed, double *t_out, int64_t *steps_out)
{
    if (!h || !edges || !uC || !uD) return REF_EINVAL;
    const oecdg_ref_desc *d = &h->d[0];
    if (h->n != 1 || d->dim != 1 || d->bc != 0 || rk_of(d) == 4)
        return fail(h, REF_EUNSUPPORTED, "one periodic 1D instance with rk 0..3");
    if (nsteps < 0 && !(t_end < INFINITY)) return fail(h, REF_EINVAL, "run needs a finite t_end or nsteps >= 0");
    if (!(t_end > 0.0)) return fail(h, REF_EINVAL, "t_end must be positive");
    ora1d p = prob1(h, 0);
    double t = 0.0;
    long s = 0;
    int rc = ora1n_run(&p, edges, d->cfl, rk_of(d), d->oe, t_end, (long)nsteps, dt_fixed, uC, uD, &t, &s);
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = s;
    return rc == REF_OK ? rc : fail(h, rc, "oracle run failed");
}

int oecdg_ref_adjoint(oecdg_ref_handle *h, const double *uC0, const double *uD0, int64_t nsteps, double dt,
                      const double *gC_T, const double *gD_T, double *gC0, double *gD0, int32_t checkpoint_every)
{
    (void)uC0; (void)uD0; (void)nsteps; (void)dt; (void)gC_T; (void)gD_T; (void)gC0; (void)gD0;
    (void)checkpoint_every;
    return fail(h, REF_EUNSUPPORTED, "the adjoint's oracle is the autograd program oracle/adjoint_torch.py");
}

const char *oecdg_ref_strerror(int code)
{
    switch (code) {
    case REF_OK: return "ok";
    case REF_EINVAL: return "invalid argument";
    case REF_ENOMEM: return "out of memory";
    case REF_EHIP: return "HIP runtime error";
    case REF_ENONFINITE: return "non-finite value";
    case REF_ENONPHYSICAL: return "non-physical state";
    case REF_EUNSUPPORTED: return "unsupported";
    case REF_ETIMEOUT: return "timeout";
    case REF_ETOOBIG: return "too big";
    default: return "unknown error";
    }
}

const char *oecdg_ref_last_error(oecdg_ref_handle *h) { return h ? h->msg : "no handle"; }
