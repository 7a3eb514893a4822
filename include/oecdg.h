/*
 * oecdg.h -- C ABI of the MI355X (gfx950) implementation of the
 * oscillation-eliminating central DG (OECDG) method of Peng, Wu and Yuan,
 * "Oscillation-eliminating central DG schemes for hyperbolic conservation
 * laws" (arXiv 2503.12473).
 *
 * The library advances the pair (u^C, u^D) of piecewise polynomials on the
 * primal mesh and the dual mesh (Sec. 2.1, the semi-discrete CDG system
 * equcdg) with the fully discrete RK-OECDG scheme (Sec. 2.2, eq. RKCDG):
 * an RK stage update (SSP-RK3 unless the descriptor asks for another method)
 * followed, after every stage, by the OE step F_tau (damping ODE OEstep2D,
 * solved exactly).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All numbers are IEEE FP64.  All state pointers are DEVICE pointers to
 *    caller-owned memory (e.g. torch tensors on the GPU); the library never
 *    frees them.  The library owns its scratch from oecdg_init to
 *    oecdg_destroy.
 *  - Modal coefficients are in the unnormalised Legendre basis P_m(xi),
 *    xi = 2 (x - x_K)/h, so coefficient 0 is the cell average.
 *  - 1D layout: u[(q*(k+1) + m)*ncell + i], component q, mode m, cell i
 *    (structure of arrays, cells fastest).  Primal cell i is
 *    [xlo + i h, xlo + (i+1) h], h = (xhi - xlo)/nx.  Dual cell j is centred
 *    on the left edge of primal cell j: [xlo + (j-1/2) h, xlo + (j+1/2) h];
 *    there are nx dual cells with periodic boundaries and nx+1 with outflow
 *    or reflective boundaries (the last one centred on xhi).  Outflow ghost
 *    primal cells (-1 and nx) are the constant extensions of the averages of
 *    cells 0 and nx-1.  Reflective walls (1D Euler only; the two-blast-wave
 *    example of Sec. 4) make them the mirror images of cells 0 and nx-1 about
 *    the wall: mode m times (-1)^m, the momentum negated once more.  The dual
 *    cells on the walls then reach half a cell outside the domain; their
 *    initial data are the mirror extension of the data inside.  Inflow
 *    boundaries (1D Euler; the examples of Sec. 4 that prescribe an incoming
 *    state) make the ghosts constant states set with oecdg_set_inflow and
 *    held for the whole run; the dual mesh has nx+1 cells as with outflow.
 *  - 2D layout (tensor-product modes; a P^k state keeps the same slots with
 *    the modes a + b > k zero): u[(((q*(k+1) + a)*(k+1) + b)*ny
 *    + iy)*nx + ix], mode a in x, b in y.  Primal cell (ix, iy) is
 *    [xlo + ix hx, xlo + (ix+1) hx] x [ylo + iy hy, ylo + (iy+1) hy]; dual
 *    cell (ix, iy) is centred on the primal vertex (xlo + ix hx, ylo + iy hy).
 *    2D meshes are periodic.
 *  - Every call is enqueued on the HIP stream given to oecdg_init.  Calls
 *    that return host scalars synchronise that stream before returning.
 *  - Entry points return OECDG_OK (0) or a negative error code; no C++
 *    exception crosses the ABI.  oecdg_last_error() gives a message.
 *  - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef OECDG_H
#define OECDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handle: library-owned scratch, tables and launch state. */
typedef struct oecdg_handle oecdg_handle;

enum {
    OECDG_OK = 0,
    OECDG_EINVAL = -1,          /* bad descriptor, size, pointer or argument */
    OECDG_ENOMEM = -2,          /* device or host allocation failed */
    OECDG_EHIP = -3,            /* HIP runtime error (message in oecdg_last_error) */
    OECDG_ENONFINITE = -4,      /* a NaN/Inf coefficient was produced */
    OECDG_ENONPHYSICAL = -5,    /* Euler: density or pressure <= 0 at a cell average */
    OECDG_EUNSUPPORTED = -6,    /* valid but not implemented combination */
    OECDG_ETIMEOUT = -7,        /* a device-side grid barrier exceeded its spin limit */
    OECDG_ETOOBIG = -8          /* oecdg_run_noalloc: the problem exceeds its fixed device scratch */
};

enum { OECDG_FLUX_ADVECTION = 0, OECDG_FLUX_BURGERS = 1, OECDG_FLUX_EULER = 2 };
enum { OECDG_BC_PERIODIC = 0, OECDG_BC_OUTFLOW = 1, OECDG_BC_REFLECTIVE = 2, OECDG_BC_INFLOW = 3 };

/* Descriptor flags. */
enum {
    OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE = 1   /* 1D Euler: a cell average with non-positive pressure is not
                                              * an error (ENONPHYSICAL then means density <= 0 only); the
                                              * wave speeds use |v| + sqrt(gamma |p| / rho) throughout,
                                              * which is |v| + c for every physical state */
};

/* Execution modes of oecdg_run (oecdg_set_option(OECDG_OPT_MODE, ...)). */
enum {
    OECDG_MODE_AUTO = 0,        /* library choice */
    OECDG_MODE_EAGER = 1,       /* one kernel launch per RK stage */
    OECDG_MODE_GRAPH = 2,       /* the three stage kernels of several steps captured in a hipGraph */
    OECDG_MODE_PERSISTENT = 3   /* one cooperative launch, grid barrier between stages */
};

/* Option keys for oecdg_set_option. */
enum {
    OECDG_OPT_MODE = 1,         /* OECDG_MODE_* */
    OECDG_OPT_TILE = 2,         /* primal cells per workgroup tile: 32, 64 or 128 (1D; 128 spills
                                 * registers and is never the library's choice) */
    OECDG_OPT_GRAPH_STEPS = 3,  /* steps per captured graph (>= 1) */
    OECDG_OPT_GRID = 4,         /* workgroups of the persistent launch (0: library choice) */
    OECDG_OPT_FOLD = 5          /* where the global statistics of Sec. 2.2 (avg, sigma) and the wave
                                 * speed are reduced before each 1D stage: 0 library choice (a
                                 * per-instance fold kernel for batches and for meshes of more
                                 * than 1024 tiles, inside every stage workgroup otherwise),
                                 * 1 inside the stage kernel, 2 the fold kernel (not when the
                                 * last tile carries the dual cell np, which then reduces
                                 * inside).  The same bits either way. */
};

/* Problem descriptor (one instance).  Sec. 2.1 defines the meshes and the
 * operator; tau_max = cfl h / max|f'(u)| in 1D and
 * cfl / (max|f_1'|/hx + max|f_2'|/hy) in 2D (Sec. 2.1 and Sec. 4), with the
 * maxima over the cell averages of both meshes. */
typedef struct {
    int32_t dim;                /* 1 or 2 */
    int32_t k;                  /* polynomial degree: 0..3 in 1D; 1..3 in 2D */
    int32_t flux;               /* OECDG_FLUX_*: 1D any; 2D advection or Euler */
    int32_t bc;                 /* OECDG_BC_*; 2D: periodic only */
    int64_t nx, ny;             /* primal cells per direction (ny = 1 in 1D) */
    double xlo, xhi, ylo, yhi;  /* domain (ylo, yhi ignored in 1D) */
    double flux_param[2];       /* advection: speeds (a, b); Euler: {gamma, 0}; Burgers: unused */
    double cfl;                 /* C_CFL */
    int32_t oe;                 /* 1: OECDG (OE step after every stage); 0: plain CDG */
    int32_t rk;                 /* time integrator, as the c/d table of eq. RKCDG (Sec. 4 runs accuracy
                                 * tests with an RK method of order k+1):
                                 * 0 or 3: SSP-RK3 (Shu-Osher), 1: forward Euler, 2: SSP-RK2 (Heun),
                                 * 4: classical fourth-order RK, whose last stage
                                 * -u^n/3 + u^1/3 + 2u^2/3 + u^3/3 + tau/6 L(u^3) uses the damped stage
                                 * values (library-owned buffer of one state).  All instances of a
                                 * batch use one method. */
    int32_t space;              /* 2D space: 0 = tensor Q^k, 1 = the paper's total-degree P^k (Sec. 2.1):
                                 * same layout; the modes with a + b > k are ignored on input and zero on
                                 * output (oecdg_run, oecdg_stage).  1D: either value (the spaces coincide). */
    int32_t flags;              /* OECDG_FLAG_* bits (0: none) */
} oecdg_desc;

/* Number of doubles of the primal and dual state arrays of one instance. */
int oecdg_state_size(const oecdg_desc *d, int64_t *n_primal, int64_t *n_dual);

/* Create a handle for nbatch >= 1 instances described by d[0..nbatch-1]
 * (nbatch > 1: 1D instances only, each with its own nx, k, bc and cfl;
 * one flux and one RK method per batch, EUNSUPPORTED otherwise).  With nbatch > 1 the state arrays passed to the other entry points
 * are the concatenation of the instances' arrays in order (offsets from
 * oecdg_batch_offsets).  stream: a hipStream_t (NULL = default stream). */
int oecdg_init(const oecdg_desc *d, int32_t nbatch, void *stream, oecdg_handle **out);

/* Element offsets of each instance's arrays inside the concatenated batch
 * arrays; off_primal and off_dual each hold nbatch+1 entries (the last is the
 * total).  Host pointers. */
int oecdg_batch_offsets(oecdg_handle *h, int64_t *off_primal, int64_t *off_dual);

/* Set an OECDG_OPT_* tuning option (execution mode, tile size, graph length,
 * persistent grid, statistics fold).  The execution mode, graph length,
 * persistent grid and fold change speed only (the same bits); the tile also
 * sets the order in which the
 * per-tile statistics are summed, so results for different tiles agree to
 * rounding.  EINVAL for an unknown key or a value out of range; setting the
 * tile rebuilds the tile list (and may return ENOMEM). */
int oecdg_set_option(oecdg_handle *h, int32_t key, int64_t value);

/* Ghost states of an inflow instance (bc = OECDG_BC_INFLOW): left and right
 * each hold nc = 3 conserved variables (rho, m, E), the cell averages of the
 * constant ghost cells left of primal cell 0 and right of cell nx-1.  Host
 * arrays, copied.  Must be called for every inflow instance before
 * oecdg_run (EINVAL from oecdg_run otherwise); EINVAL for an instance index
 * out of range or an instance without inflow boundaries. */
int oecdg_set_inflow(oecdg_handle *h, int32_t instance, const double *left, const double *right);

/* tau_max of instance 0 for the state (uC, uD) (Sec. 2.1; cell averages of
 * both meshes).  Device inputs, host output; synchronises the stream. */
int oecdg_dt(oecdg_handle *h, const double *uC, const double *uD, double *dt_out);

/* One stage l of the handle's RK method (eq. RKCDG) followed by the OE step
 * (OEstep1):
 *   u_sigma^{n,l+1} = F_tau( c_{l0} u^n + c_{ll} u_sigma^{n,l} + tau d_{ll} L(u_sigma^{n,l}) )
 * e.g. SSP-RK3: (c_{00}, d_{00}) = (1, 1), (c_{10}, c_{11}, d_{11}) = (3/4, 1/4, 1/4),
 * (c_{20}, c_{22}, d_{22}) = (1/3, 2/3, 2/3); at stage 0, u^n is u_sigma^{n,0}
 * and c_{00} multiplies it once.  stage in 0 .. s-1 (EINVAL otherwise); the last
 * stage of classical RK4, which reads the earlier stages, is EUNSUPPORTED.  dt = tau,
 * tau_max = the coupling parameter of the operator.  uC_n/uD_n = u_sigma^n,
 * uC_l/uD_l = u_sigma^{n,l} (ignored/aliasable for stage 0); outputs must not
 * alias inputs.  Single instance handles only.  Device pointers. */
int oecdg_stage(oecdg_handle *h, int32_t stage, double dt, double tau_max,
                const double *uC_n, const double *uD_n,
                const double *uC_l, const double *uD_l,
                double *uC_out, double *uD_out);

/* Advance in place from t = 0: on entry (uC, uD) = u_sigma^0 (no OE is
 * applied to it), on exit u_sigma^N.  Stops at t_end (the last step is
 * shortened to land on t_end; tau_max keeps the CFL value) or after nsteps
 * steps (nsteps < 0: no limit); t_end may be +inf when nsteps >= 0.
 * dt_fixed > 0 replaces the CFL step (tau = tau_max = dt_fixed).  For
 * batches every instance takes the same nsteps/t_end/dt_fixed, each with its
 * own CFL step.  Each step runs the stages of the descriptor's RK method, each
 * followed by F_tau.  t_out/steps_out (host, may be NULL) receive instance 0's
 * final time and step count.  Synchronises the stream. */
int oecdg_run(oecdg_handle *h, double *uC, double *uD, double t_end, int64_t nsteps,
              double dt_fixed, double *t_out, int64_t *steps_out);

/* Bytes of the fixed device scratch of oecdg_run_noalloc (per GPU, held from
 * its first call on that GPU until the process ends). */
#define OECDG_NOALLOC_SCRATCH_BYTES (32u << 20)

/* oecdg_run for one 1D instance without allocating anything, for callers that
 * cannot allocate (code under stream capture by a caller of its own, serving
 * loops, harnesses that forbid hipMalloc): no handle; the stage buffers,
 * damped u^n, partial statistics, step records and error flags live in a
 * fixed file-scope device array of OECDG_NOALLOC_SCRATCH_BYTES per GPU
 * (state arrays, both meshes, three of them, four with classical RK4, plus
 * the statistics: about 1.3 M doubles of state, e.g. 1D Euler P2 up to
 * nx ~ 77000).  d: one 1D descriptor as for oecdg_init; stream: a hipStream_t
 * (NULL = default stream) on the current device; the other arguments as
 * oecdg_run (uC, uD are caller-owned device arrays, advanced in place).
 * Eager launches only (no graph is built) with the tile and launch shape
 * oecdg_init would choose, so results are bitwise those of oecdg_run on a
 * handle of the same descriptor.  Returns ETOOBIG when the problem does not
 * fit the scratch, EINVAL / EUNSUPPORTED for descriptors oecdg_init rejects
 * or dim != 1, the run's own error codes otherwise; there is no handle, so
 * no message.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (two host threads, or streams that run concurrently)
 * race and must be serialised by the caller.  Synchronises the stream. */
int oecdg_run_noalloc(const oecdg_desc *d, void *stream, double *uC, double *uD, double t_end, int64_t nsteps,
                      double dt_fixed, double *t_out, int64_t *steps_out);

/* oecdg_run on a non-uniform periodic 1D mesh (Sec. 2.1: primal cells
 * [x_{i-1/2}, x_{i+1/2}] of width h_i, dual cells [x_{i-1}, x_i] between
 * neighbouring primal centres; h = max_i h_i in tau_max = cfl h / beta).  The
 * damping of Sec. 2.2 takes h_{e,K} = the width of K and avg = the domain
 * mean (width-weighted cell averages).  edges: host array of the nx+1 primal
 * edges, edges[0] = xlo, edges[nx] = xhi, strictly increasing (EINVAL
 * otherwise); copied at each call.  (uC, uD): device arrays [nc][k+1][nx]
 * each, primal cell i and dual cell j = [x_{j-1}, x_j] (dual cell 0 starts
 * at x_{nx-1} minus the period).  The handle must hold one periodic 1D
 * instance with rk 0..3 (EUNSUPPORTED otherwise); the library allocates the
 * mesh's buffers at the first call and keeps them with the handle (the
 * handle's nx, k and flux fix their sizes).  Other arguments and errors as
 * oecdg_run; the execution-mode and tile options do not apply.  Synchronises
 * the stream. */
int oecdg_run_nonuniform(oecdg_handle *h, const double *edges, double *uC, double *uD, double t_end,
                         int64_t nsteps, double dt_fixed, double *t_out, int64_t *steps_out);

/* Discrete adjoint of oecdg_run with a fixed step: the transpose of the
 * derivative of the fully discrete scheme of Sec. 2.2 (SSP-RK3 stages of
 * eq. RKCDG, each followed by F_tau).  Given u_sigma^0 = (uC0, uD0), nsteps
 * steps of size dt = tau = tau_max and the gradient (gC_T, gD_T) of a loss J
 * with respect to u_sigma^N (in modal coefficients), writes dJ/du_sigma^0 into
 * (gC0, gD0).  1D single-instance handles with a scalar flux (advection or
 * Burgers) on a periodic mesh and SSP-RK3; EUNSUPPORTED otherwise; EINVAL for nsteps < 0,
 * dt <= 0 or checkpoint_every < 1.  The forward states are recomputed from
 * checkpoints stored every checkpoint_every steps; the library-owned workspace
 * (checkpoints plus two segments of stage states) grows on demand (ENOMEM if it
 * cannot).  The recomputation of a segment runs on a second library-owned
 * stream, overlapped with the reverse stages of the next one; all of it has
 * finished when the call returns (the call synchronises the handle's stream).
 * Non-smooth points follow fixed conventions: d|x|/dx = 0 at x = 0, the
 * maximum in sigma is attributed to the first maximiser in storage order, a
 * vanishing sigma contributes no derivative.  Device pointers; every input
 * is copied into the workspace before an output is written, so the outputs
 * may alias the inputs. */
int oecdg_adjoint(oecdg_handle *h, const double *uC0, const double *uD0, int64_t nsteps, double dt,
                  const double *gC_T, const double *gD_T, double *gC0, double *gD0,
                  int32_t checkpoint_every);

/* Release the handle and everything it owns (NULL is allowed).  Waits for the
 * library's own streams; work the caller enqueued on its stream is not waited for. */
void oecdg_destroy(oecdg_handle *h);

/* Static description of an error code. */
const char *oecdg_strerror(int code);

/* Message of the last failing call on h (library-owned, valid until the next call). */
const char *oecdg_last_error(oecdg_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* OECDG_H */
