// oecdg_internal.h -- device data structures and host launch interfaces of the
// HIP implementation (library-private; the public ABI is include/oecdg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oecdg {

constexpr int MAXK = 3;

// Per-tile partial statistics written by every stage kernel (and by the
// statistics kernel) for the state it produced, stored [tile][row] (one
// record of NSTAT doubles per tile).  Row (mesh*3 + q)*3 + kind,
// kind 0 = sum of cell averages, 1 = max, 2 = min of the point values at the
// sigma sample points; ST_BETA = largest wave speed at a cell average.
constexpr int NSTAT = 20;
constexpr int ST_BETA = 18;

__host__ __device__ constexpr int stat_index(int mesh, int q, int kind) { return (mesh * 3 + q) * 3 + kind; }

// One 1D problem instance of a (possibly single-element) batch.
struct Inst1D {
    int k, nc, flux, bc;
    int np, nd;              // primal / dual cell counts
    int tile0, ntiles;       // tiles [tile0, tile0 + ntiles) of the global tile list
    long long offC, offD;    // element offsets in the concatenated state arrays
    double h, cfl, p0;       // cell width, C_CFL, flux parameter (speed or gamma)
    int oe;
    int tail;                // the last tile also updates dual cell np (outflow/walls, np a multiple of T)
    int npart;               // partial-statistics columns [tile0, tile0 + npart): ntiles, plus one with a tail
    int flags;               // OECDG_FLAG_* of the descriptor
    double gin[2][3];        // inflow boundaries: cell averages of the ghost cells left of 0 and right of np-1
};

// A tile: primal cells [i0, i0 + T) and dual cells [i0, i0 + T) of instance inst.
struct Tile1D {
    int inst, i0;
};

// Per instance and step parity: the step's start time and its tau/tau_max.
struct Slot {
    double t, tau, tau_max;
    int done, last;
};

// Per instance: time reached, tau of the last executed step, executed steps.
struct Final {
    double t, tau;
    long long nexec;
};

// Tiles of up to 64 cells can take an instance's dual cell np in its last
// tile (a lane of the wave that holds the tile's neighbour cells) instead of
// in a tile of its own.
__host__ __device__ constexpr bool tail_mode(int T) { return T <= 64; }

// One stage of an RK method in the c/d form of eq:RKCDG,
//   u_h^{n,l+1} = sum_{m<=l} c_{lm} u_sigma^{n,m} + tau d_{lm} L(u_sigma^{n,m}).
// Every supported table has d_{lm} = 0 for m < l and, apart from u^n, earlier
// stages enter only the last stage of classical RK4; that stage reads their
// weighted sum, accumulated by the stages that produce them.
struct RKStage {
    double cn;        // c_{l0}, l > 0 (at l = 0 the input is u^n and c_{00} is cw)
    double cw;        // c_{ll}
    double d;         // d_{ll}
    double ca;        // weight of this stage's input in the accumulated sum (0: not part of it)
    int acc_first;    // this stage starts the sum (otherwise it adds to it)
    int acc_read;     // this stage adds the accumulated sum
};

// rk: 1 forward Euler, 2 SSP-RK2 (Heun), 3 SSP-RK3 (Shu-Osher), 4 classical
// fourth-order RK.  Stages per step:
__host__ __device__ inline int rk_stages(int rk) { return rk == 1 ? 1 : (rk == 2 ? 2 : (rk == 4 ? 4 : 3)); }

__host__ __device__ inline RKStage rk_stage(int rk, int l) {
    RKStage s{0.0, 1.0, 1.0, 0.0, 0, 0};
    if (rk == 2) {
        if (l == 1) s.cn = 0.5, s.cw = 0.5, s.d = 0.5;
    } else if (rk == 4) {
        // u^1 = u^n + tau/2 L(u^n), u^2 = u^n + tau/2 L(u^1), u^3 = u^n + tau L(u^2),
        // u^4 = -u^n/3 + u^1/3 + 2u^2/3 + u^3/3 + tau/6 L(u^3)
        if (l == 0) s.d = 0.5;
        if (l == 1) s.cn = 1.0, s.cw = 0.0, s.d = 0.5, s.ca = 1.0 / 3.0, s.acc_first = 1;
        if (l == 2) s.cn = 1.0, s.cw = 0.0, s.d = 1.0, s.ca = 2.0 / 3.0;
        if (l == 3) s.cn = -1.0 / 3.0, s.cw = 1.0 / 3.0, s.d = 1.0 / 6.0, s.acc_read = 1;
    } else if (rk != 1) {
        if (l == 1) s.cn = 0.75, s.cw = 0.25, s.d = 0.25;
        if (l == 2) s.cn = 1.0 / 3.0, s.cw = 2.0 / 3.0, s.d = 2.0 / 3.0;
    }
    return s;
}

struct StageArgs {
    const Inst1D *inst;
    const Tile1D *tiles;
    int ntiles;              // partial-statistics columns of the whole batch (row length of the partials)
    int tbeg, tend;          // tiles [tbeg, tend) handled by this launch (one degree group)
    Slot *slots;             // [ninst][2]
    Final *fin;              // [ninst]
    double *part[2];         // [ntiles][NSTAT] each (one record per tile)
    double *BC[2], *BD[2];   // rotating pre-damping stage states
    double *UC, *UD;         // damped u^n of the current step
    double *DC, *DD;         // optional: damped input of stages 1 and 2 (adjoint recomputation)
    double *AC, *AD;         // classical RK4: weighted sum of the damped inputs of stages 1 and 2
    double *red;             // batched launches: [ninst][NSTAT] statistics reduced by k_fold (else null)
    int *err;                // [0] non-finite, [1] non-physical, [2] barrier timeout, [3] step+1 of an error
    int rk, ns;              // RK method (rk_stage) and its stages per step
    RKStage rs;              // rk_stage(rk, l), set by the stage launcher (the persistent launch forms its own)
    int tailwave;            // launches carry one more wave, for the dual cell np of tail tiles
    int l;                   // stage of the step (0 .. ns-1)
    int par;                 // parity of the step index n
    int first;               // 1 for step 0 (its input is the initial data: no OE)
    int coherent;            // 1 in the persistent launch (cross-workgroup reads after a barrier)
    Inst1D inst0;            // the instance when ninst == 1
    double t_end;
    double dt_fixed;         // > 0: tau = tau_max = dt_fixed
    double tau_override, taumax_override;   // > 0: single-stage call with given tau/tau_max
    int damp_input;          // 0: the stage input is used as is (single-stage call)
    int ninst;               // instances in the batch
    // final / statistics kernels
    const double *srcC, *srcD;
    double *dstC, *dstD;
    int init_records;        // statistics kernel: also clear the step records and error flags (a run's start)
    Final *fin_host;         // final kernel, when set: the step records and error flags copied to these
    int *err_host;           //   host-mapped arrays (device addresses of pinned host memory)
    // persistent launch
    unsigned *bar;           // [0] arrival count, [1] generation
    long long spin_limit;
};

// Arguments of the adjoint kernels (oecdg_adjoint.hip): scalar periodic 1D,
// n cells per mesh, modal arrays [m][cell].
struct AdjArgs {
    int k, flux, n, nb;            // degree, flux id, cells per mesh, workgroups per mesh
    int nbp, pad0;                 // per-wave partial entries per mesh (nb x waves per workgroup)
    long long S;                   // (k+1) n: offset of the dual mesh in every field below
    double hinv, p0, tau, inv_tm;  // 1/h, flux parameter, tau, 1/tau_max
    double inv_n;                  // 1/n (derivative of the mesh average)
    const double *fpart;           // forward per-tile partial statistics of h (the stage prepared here)
    int ftile0, fntiles;
    const double *h;               // undamped output h_l of the stage prepared here
    const double *s;               // damped input s_l of the stage reversed here
    const double *lam;             // adjoint of s_{l+1} (OE off) or of F(h) (prepare-only launch)
    const double *lp_in, *cr_in, *cl_in, *bp_in;   // preparation of the stage above
    double *lp, *cr, *cl, *bp;                      // preparation of this stage
    double *out, *acc;             // adjoint of s_l; adjoint of s_0 accumulated over the stages
    double al, bl;                 // h_{l+1} = al s_0 + bl (s_l + tau L(s_l))
    int stage0, acc_init, oe, do_rk, do_prep, pad;
};
hipError_t launch_adj(const AdjArgs &a, hipStream_t s);
int adj_block_size();
int adj_block_partials();
int adj_waves();

// Host-side launchers (oecdg_1d.hip).
hipError_t launch_init_1d(const StageArgs &a, int ninst, hipStream_t s);
hipError_t launch_stats_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s);
hipError_t launch_stage_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s);   // one workgroup per tile
hipError_t launch_fold_1d(const StageArgs &a, int flux, int tile, hipStream_t s);
hipError_t launch_final_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s);
hipError_t launch_persistent_1d(const StageArgs &a, int kmax, int flux, int tile, int grid,
                                long long nsteps, hipStream_t s);
int persistent_max_grid_1d(int kmax, int flux, int tile, bool tailwave);

}  // namespace oecdg

#include "oecdg.h"

namespace oecdg {

// Descriptor helpers shared by the entry points (oecdg_api.cpp).
int nc_of(int flux, int dim);
int validate(const oecdg_desc &d, const char *&why);                  // why: a static string
void sizes(const oecdg_desc &d, int64_t &np, int64_t &nd);             // state array lengths
Inst1D make_inst(const oecdg_desc &e);                                 // offsets and tiles left zero
int default_tile(int64_t maxn, int nbatch);                            // primal cells per workgroup
bool tail_candidate(const Inst1D &I, int T);                           // dual cell np beyond np / T full tiles

// Handle accessors for the 2D path (defined in oecdg_api.cpp).
hipStream_t handle_stream(oecdg_handle *h);
const oecdg_desc &handle_desc(oecdg_handle *h);
void *&handle_ext2d(oecdg_handle *h);
int handle_fail(oecdg_handle *h, int code, const char *msg);

// 2D path (oecdg_2d.hip) and the 1D adjoint (oecdg_adjoint.hip).
int create_2d(oecdg_handle *h, const oecdg_desc *d);
int dt_2d(oecdg_handle *h, const double *uC, const double *uD, double *dt_out);
int stage_2d(oecdg_handle *h, int stage, double dt, double tau_max, const double *uCn, const double *uDn,
             const double *uCl, const double *uDl, double *uCo, double *uDo);
int run_2d(oecdg_handle *h, double *uC, double *uD, double t_end, int64_t nsteps, double dt_fixed, double *t_out,
           int64_t *steps_out);
void destroy_2d(oecdg_handle *h);
int handle_nbatch(oecdg_handle *h);
void *&handle_extnu(oecdg_handle *h);

// Non-uniform periodic 1D meshes (oecdg_nu.hip).
int run_nonuniform(oecdg_handle *h, const double *edges, double *uC, double *uD, double t_end, int64_t nsteps,
                   double dt_fixed, double *t_out, int64_t *steps_out);
void destroy_nu(oecdg_handle *h);
int adjoint_1d(oecdg_handle *h, const double *uC0, const double *uD0, int64_t nsteps, double dt, const double *gCT,
               const double *gDT, double *gC0, double *gD0, int ckpt);

}  // namespace oecdg
