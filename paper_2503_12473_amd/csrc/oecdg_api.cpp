// oecdg_api.cpp -- host implementation of the C ABI declared in include/oecdg.h.
#include "oecdg.h"
#include "oecdg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace oecdg;

static_assert(sizeof(oecdg_desc) == 104, "oecdg_desc layout is part of the ABI");

struct oecdg_handle {
    std::vector<oecdg_desc> desc;
    int nbatch = 0;
    hipStream_t stream = nullptr;
    int dim = 1;

    // 1D batch bookkeeping
    std::vector<Inst1D> inst_h;
    std::vector<char> inflow_set;   // oecdg_set_inflow was called for the instance
    std::vector<Tile1D> tiles_h;
    struct Group {
        int k, tbeg, tend;
    };
    std::vector<Group> groups;   // tiles ordered by degree: one launch per degree
    std::vector<int64_t> offC, offD;
    int64_t totC = 0, totD = 0;
    int kmax = 0, flux = 0;  // flux: kernel flux id (OECDG_FLUX_*, or 3 = Euler with reflective walls)
    int rk = 3;              // RK method of every instance (rk_stage)
    bool tailwave = false;   // some instance's last tile updates the extra dual cell (launches carry one more wave)
    int ncol = 0;            // partial-statistics columns (the tiles, plus one per tail)
    int tile = 64;
    int mode = OECDG_MODE_AUTO;
    int graph_steps = 64;
    int grid = 0;
    int fold = 0;            // OECDG_OPT_FOLD: 0 auto (batches), 1 in-kernel, 2 fold kernel

    // device memory (library-owned)
    Inst1D *inst_d = nullptr;
    Tile1D *tiles_d = nullptr;
    Slot *slots = nullptr;
    Final *fin = nullptr;
    double *part = nullptr;
    double *B = nullptr;     // BC0 | BC1 | BD0 | BD1
    double *U = nullptr;     // UC | UD
    double *A = nullptr;     // AC | AD: classical RK4 only (sum of earlier stages for the last one)
    int *err = nullptr;
    unsigned *bar = nullptr;
    double *red = nullptr;   // [nbatch][NSTAT] statistics folded by k_fold
    // pinned host mirrors (one block: records, then flags), host-coherent and
    // mapped: the final kernel of a short run writes them directly
    Final *fin_h = nullptr;
    int *err_h = nullptr;
    Final *fin_hd = nullptr;     // device addresses of the same memory
    int *err_hd = nullptr;

    // captured graphs, all for one key (t_end, dt_fixed, tile, graph_steps, fold):
    // graph_steps steps, and 2^j steps (the remainder of a run), both from an
    // odd step index; a whole short run (copies in, steps, final OE, the
    // host copies of the step record and the error flags) for given state
    // pointers and step count
    hipGraphExec_t gexec = nullptr;
    hipGraphExec_t ladder[13] = {};
    hipGraphExec_t whole = nullptr;
    double *w_uC = nullptr, *w_uD = nullptr;
    long long w_limit = -1;
    hipStream_t cap = nullptr;   // capture stream (the caller's stream may be the null stream)
    double g_tend = 0, g_dt = 0;
    int g_tile = 0, g_steps = 0, g_fold = -1;

    double *adj_ws = nullptr;    // adjoint workspace (checkpoints, segment states, adjoint buffers)
    size_t adj_bytes = 0;
    hipStream_t aux = nullptr;   // adjoint: segment recomputation, overlapped with the reverse stages
    hipEvent_t adj_ev[5] = {};   // adjoint: segment buffer ready (2), buffer free (2), checkpoint written

    void *ext2d = nullptr;   // 2D state (oecdg_2d.hip)
    void *extnu = nullptr;   // non-uniform 1D mesh state (oecdg_nu.hip)
    std::string last;
};

namespace {

int fail(oecdg_handle *h, int code, const std::string &msg) {
    if (h) h->last = msg;
    return code;
}

#define HIPCHK(h, expr)                                                                               \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail((h), OECDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Bytes of the step records of nbatch instances followed by the four error flags.
size_t rec_bytes(int nbatch) { return sizeof(Final) * (size_t)nbatch + 4 * sizeof(int); }

void drop_graphs(oecdg_handle *h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec), h->gexec = nullptr;
    for (hipGraphExec_t &g : h->ladder)
        if (g) (void)hipGraphExecDestroy(g), g = nullptr;
    if (h->whole) (void)hipGraphExecDestroy(h->whole), h->whole = nullptr;
    h->w_uC = h->w_uD = nullptr;
    h->w_limit = -1;
}

}  // namespace

int oecdg::nc_of(int flux, int dim) { return flux == OECDG_FLUX_EULER ? (dim == 1 ? 3 : 4) : 1; }

int oecdg::validate(const oecdg_desc &d, const char *&why) {   // why: a static string
    if (d.dim != 1 && d.dim != 2) return why = "dim must be 1 or 2", OECDG_EINVAL;
    if (d.rk < 0 || d.rk > 4) return why = "rk must be 0 (SSP-RK3), 1, 2, 3 or 4", OECDG_EINVAL;
    if (d.space != 0 && d.space != 1) return why = "space must be 0 (Q^k) or 1 (P^k)", OECDG_EINVAL;
    if (d.flags & ~OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE) return why = "unknown flag", OECDG_EINVAL;
    if (d.flux < 0 || d.flux > 2) return why = "unknown flux", OECDG_EINVAL;
    if (d.bc < 0 || d.bc > 3) return why = "unknown boundary condition", OECDG_EINVAL;
    if (d.bc == OECDG_BC_REFLECTIVE && d.flux != OECDG_FLUX_EULER)
        return why = "reflective walls need the Euler flux", OECDG_EUNSUPPORTED;
    if (d.bc == OECDG_BC_INFLOW && d.flux != OECDG_FLUX_EULER)
        return why = "inflow boundaries need the Euler flux", OECDG_EUNSUPPORTED;
    if (!(d.xhi > d.xlo)) return why = "xhi must exceed xlo", OECDG_EINVAL;
    if (!(d.cfl > 0.0)) return why = "cfl must be positive", OECDG_EINVAL;
    if (d.flux == OECDG_FLUX_EULER && !(d.flux_param[0] > 1.0)) return why = "Euler needs gamma > 1", OECDG_EINVAL;
    if (d.dim == 1) {
        if (d.k < 0 || d.k > MAXK) return why = "1D degree must be 0..3", OECDG_EINVAL;
        if (d.nx < 2 || d.nx > (1LL << 30)) return why = "1D nx out of range", OECDG_EINVAL;
        if (d.ny != 1 && d.ny != 0) return why = "1D ny must be 1", OECDG_EINVAL;
    } else {
        if (d.k < 1 || d.k > MAXK) return why = "2D degree must be 1..3", OECDG_EUNSUPPORTED;
        if (d.flux == OECDG_FLUX_BURGERS) return why = "2D Burgers is not implemented", OECDG_EUNSUPPORTED;
        if (d.bc != OECDG_BC_PERIODIC) return why = "2D supports periodic boundaries only", OECDG_EUNSUPPORTED;
        if (d.flags != 0) return why = "descriptor flags are 1D only", OECDG_EUNSUPPORTED;
        if (d.nx < 2 || d.ny < 2 || d.nx > 65536 || d.ny > 65536) return why = "2D nx, ny out of range", OECDG_EINVAL;
        if (!(d.yhi > d.ylo)) return why = "yhi must exceed ylo", OECDG_EINVAL;
    }
    return OECDG_OK;
}

void oecdg::sizes(const oecdg_desc &d, int64_t &np, int64_t &nd) {
    const int64_t nc = nc_of(d.flux, d.dim);
    if (d.dim == 1) {
        np = nc * (d.k + 1) * d.nx;
        nd = nc * (d.k + 1) * (d.bc == OECDG_BC_PERIODIC ? d.nx : d.nx + 1);
    } else {
        np = nd = nc * (d.k + 1) * (d.k + 1) * d.nx * d.ny;
    }
}

// One instance of the descriptor (offsets and tiles are set by the caller).
Inst1D oecdg::make_inst(const oecdg_desc &e) {
    Inst1D I;
    memset(&I, 0, sizeof(I));
    I.k = e.k;
    I.nc = nc_of(e.flux, 1);
    I.flux = e.flux;
    I.bc = e.bc;
    I.np = (int)e.nx;
    I.nd = (int)(e.bc == OECDG_BC_PERIODIC ? e.nx : e.nx + 1);
    I.h = (e.xhi - e.xlo) / (double)e.nx;
    I.cfl = e.cfl;
    I.p0 = e.flux_param[0];
    I.oe = e.oe;
    I.flags = e.flags;
    return I;
}

// Default tile: 64 primal + 64 dual cells per workgroup unless the mesh is
// small (32: more workgroups).  (Tiles of 128 run five waves per workgroup,
// which caps the registers at 256 and spills; large meshes fold their
// statistics instead, fold_on.)
int oecdg::default_tile(int64_t maxn, int nbatch) { return maxn <= 4096 && nbatch == 1 ? 32 : 64; }

// An outflow/walled mesh whose primal count is a multiple of T has its dual
// cell np beyond np / T full tiles.
bool oecdg::tail_candidate(const Inst1D &I, int T) { return I.nd == I.np + 1 && I.np % T == 0 && tail_mode(T); }

namespace {

int build_tiles(oecdg_handle *h) {
    h->tiles_h.clear();
    h->groups.clear();
    h->tailwave = false;
    const int T = h->tile;
    // nd = np + 1 with np a multiple of T leaves dual cell np beyond np / T full
    // tiles.  When that extra tile would take the workgroup count past the
    // number of CUs, the last tile takes the cell instead, with one more wave
    // in every workgroup of the launch (a workgroup of five waves cannot share
    // a CU with another, so this is used only when all tiles then fit one per
    // CU, and for single instances).  The cell's statistics keep a partial
    // column of their own, so the results are those of the separate tile.
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 0;
    long long plain = 0, merged = 0;
    for (const Inst1D &I : h->inst_h) {
        plain += (I.nd + T - 1) / T;
        merged += tail_candidate(I, T) ? I.np / T : (I.nd + T - 1) / T;
    }
    const bool use_tail = h->nbatch == 1 && plain > ncu && merged <= ncu && merged < plain;
    int ncol = 0;
    for (int k = 0; k <= MAXK; ++k) {
        const int tbeg = (int)h->tiles_h.size();
        for (int b = 0; b < h->nbatch; ++b) {
            Inst1D &I = h->inst_h[b];
            if (I.k != k) continue;
            I.tile0 = (int)h->tiles_h.size();
            I.tail = use_tail && tail_candidate(I, T);
            if (I.tail) h->tailwave = true;
            I.ntiles = I.tail ? I.np / T : (I.nd + T - 1) / T;
            I.npart = I.ntiles + (I.tail ? 1 : 0);
            ncol += I.npart;
            for (int t = 0; t < I.ntiles; ++t) h->tiles_h.push_back(Tile1D{b, t * T});
        }
        if ((int)h->tiles_h.size() > tbeg) h->groups.push_back({k, tbeg, (int)h->tiles_h.size()});
    }
    if (h->tiles_d) (void)hipFree(h->tiles_d), h->tiles_d = nullptr;
    if (h->part) (void)hipFree(h->part), h->part = nullptr;
    HIPCHK(h, hipMalloc(&h->tiles_d, sizeof(Tile1D) * h->tiles_h.size()));
    HIPCHK(h, hipMemcpy(h->tiles_d, h->tiles_h.data(), sizeof(Tile1D) * h->tiles_h.size(), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->inst_d, h->inst_h.data(), sizeof(Inst1D) * h->nbatch, hipMemcpyHostToDevice));
    h->ncol = ncol;
    HIPCHK(h, hipMalloc(&h->part, sizeof(double) * 2 * NSTAT * ncol));
    HIPCHK(h, hipMemset(h->part, 0, sizeof(double) * 2 * NSTAT * ncol));
    drop_graphs(h);
    return OECDG_OK;
}

// Statistics folded by a separate per-instance kernel (k_fold) before each
// stage launch, instead of every workgroup reducing its instance's partials:
// the default for batches and for meshes of more than 1024 tiles (whose
// in-kernel reduction would read every tile's record in every workgroup);
// other single instances reduce in-kernel unless asked.
bool fold_on(const oecdg_handle *h) {
    return !h->tailwave && (h->fold == 2 || (h->fold == 0 && (h->nbatch > 1 || h->ncol > 1024)));
}

StageArgs base_args(oecdg_handle *h) {
    StageArgs a;
    memset(&a, 0, sizeof(a));
    a.inst = h->inst_d;
    a.tiles = h->tiles_d;
    a.ntiles = h->ncol;
    a.tbeg = 0;
    a.tend = (int)h->tiles_h.size();
    a.slots = h->slots;
    a.fin = h->fin;
    const size_t ps = (size_t)NSTAT * h->ncol;
    a.part[0] = h->part;
    a.part[1] = h->part + ps;
    a.BC[0] = h->B;
    a.BC[1] = h->B + h->totC;
    a.BD[0] = h->B + 2 * h->totC;
    a.BD[1] = h->B + 2 * h->totC + h->totD;
    a.UC = h->U;
    a.UD = h->U + h->totC;
    if (h->A) {
        a.AC = h->A;
        a.AD = h->A + h->totC;
    }
    a.rk = h->rk;
    a.ns = rk_stages(h->rk);
    a.tailwave = h->tailwave;
    a.err = h->err;
    a.bar = h->bar;
    a.spin_limit = 1LL << 25;
    a.damp_input = 1;
    a.ninst = h->nbatch;
    if (h->nbatch == 1) a.inst0 = h->inst_h[0];
    a.red = fold_on(h) ? h->red : nullptr;
    a.t_end = INFINITY;
    return a;
}

int errors_from_host(oecdg_handle *h) {
    if (h->err_h[2]) return fail(h, OECDG_ETIMEOUT, "grid barrier spin limit exceeded");
    if (h->err_h[0])
        return fail(h, OECDG_ENONFINITE, "non-finite coefficient produced at step " + std::to_string(h->err_h[3] - 1));
    if (h->err_h[1])
        return fail(h, OECDG_ENONPHYSICAL,
                    "non-positive density or pressure at a cell average at step " + std::to_string(h->err_h[3] - 1));
    return OECDG_OK;
}

int check_errors(oecdg_handle *h) {
    HIPCHK(h, hipMemcpyAsync(h->err_h, h->err, 4 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return errors_from_host(h);
}

// One launch per degree group (tiles [tbeg, tend) of equal k), after the
// per-instance fold of the statistics when the stage kernels read it; one
// workgroup per tile.
int stage_all(oecdg_handle *h, const StageArgs &a) {
    if (a.red) HIPCHK(h, launch_fold_1d(a, h->flux, h->tile, h->stream));
    for (auto &g : h->groups) {
        StageArgs b = a;
        b.tbeg = g.tbeg;
        b.tend = g.tend;
        HIPCHK(h, launch_stage_1d(b, g.k, h->flux, h->tile, h->stream));
    }
    return OECDG_OK;
}

// (a.init_records: the first launch also clears the step records)
int stats_all(oecdg_handle *h, const StageArgs &a) {
    bool first = true;
    for (const auto &g : h->groups) {
        StageArgs b = a;
        b.tbeg = g.tbeg;
        b.tend = g.tend;
        b.init_records = first ? a.init_records : 0;
        first = false;
        HIPCHK(h, launch_stats_1d(b, g.k, h->flux, h->tile, h->stream));
    }
    return OECDG_OK;
}

// (a.fin_host: the first launch also copies the records to the host)
int final_all(oecdg_handle *h, const StageArgs &a) {
    bool first = true;
    for (const auto &g : h->groups) {
        StageArgs b = a;
        b.tbeg = g.tbeg;
        b.tend = g.tend;
        if (!first) b.fin_host = nullptr, b.err_host = nullptr;
        first = false;
        HIPCHK(h, launch_final_1d(b, g.k, h->flux, h->tile, h->stream));
    }
    return OECDG_OK;
}

// Launch the stage kernels of steps n0 .. n0 + count - 1.  inC/inD (optional):
// the arrays that the first stage of step 0 reads instead of the stage buffer
// of index 0 (the caller's initial data, read in place).
int launch_steps(oecdg_handle *h, const StageArgs &base, long long n0, long long count,
                 const double *inC = nullptr, const double *inD = nullptr) {
    for (long long n = n0; n < n0 + count; ++n)
        for (int l = 0; l < base.ns; ++l) {
            StageArgs a = base;
            a.l = l;
            a.par = (int)(n & 1);
            a.first = n == 0;
            if (n == 0 && l == 0 && inC) {   // stage (0, 0) reads the buffer of parity 0
                a.BC[0] = const_cast<double *>(inC);
                a.BD[0] = const_cast<double *>(inD);
            }
            int rc = stage_all(h, a);
            if (rc != OECDG_OK) return rc;
        }
    return OECDG_OK;
}

// Capture what body() enqueues on the handle's stream into an executable graph.
template <class F>
int capture(oecdg_handle *h, F &&body, hipGraphExec_t *out) {
    if (!h->cap) HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipStream_t user = h->stream;
    h->stream = h->cap;
    HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    int rc = body();
    hipError_t e = hipStreamEndCapture(h->cap, &g);
    h->stream = user;
    if (rc != OECDG_OK) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(h, OECDG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(h, OECDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return OECDG_OK;
}

// Graphs depend on (t_end, dt_fixed, tile, graph_steps, fold): drop them when these change.
void key_graphs(oecdg_handle *h, const StageArgs &base) {
    const int fold = base.red ? 1 : 0;
    if (h->g_tend == base.t_end && h->g_dt == base.dt_fixed && h->g_tile == h->tile &&
        h->g_steps == h->graph_steps && h->g_fold == fold)
        return;
    drop_graphs(h);
    h->g_tend = base.t_end;
    h->g_dt = base.dt_fixed;
    h->g_tile = h->tile;
    h->g_steps = h->graph_steps;
    h->g_fold = fold;
}

// A graph of graph_steps (even) steps that starts at an odd step index: the
// parities baked into its nodes hold for every replay after step 0.
int ensure_graph(oecdg_handle *h, const StageArgs &base) {
    key_graphs(h, base);
    if (h->gexec) return OECDG_OK;
    return capture(h, [&] { return launch_steps(h, base, 1, h->graph_steps); }, &h->gexec);
}

// 2^j steps from an odd step index (any power of two: starting at an odd index
// with pieces of even length, or ending with the single step, keeps the parity).
int ensure_ladder(oecdg_handle *h, const StageArgs &base, int j) {
    key_graphs(h, base);
    if (h->ladder[j]) return OECDG_OK;
    return capture(h, [&] { return launch_steps(h, base, 1, 1LL << j); }, &h->ladder[j]);
}

// The remainder of a run, count < 2^13 steps from an odd step index, as
// power-of-two graphs, largest first (the single step, if any, comes last).
int launch_remainder(oecdg_handle *h, const StageArgs &base, long long count) {
    for (int j = 12; j >= 0; --j)
        if (count & (1LL << j)) {
            int rc = ensure_ladder(h, base, j);
            if (rc != OECDG_OK) return rc;
            HIPCHK(h, hipGraphLaunch(h->ladder[j], h->stream));
        }
    return OECDG_OK;
}

// Has every instance reached t_end (or an error been flagged)?
int all_done(oecdg_handle *h, const StageArgs &a, bool &done, long long &exec0) {
    HIPCHK(h, hipMemcpyAsync(h->fin_h, h->fin, rec_bytes(h->nbatch), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    exec0 = h->fin_h[0].nexec;
    done = true;
    if (h->err_h[0] || h->err_h[1] || h->err_h[2]) return OECDG_OK;
    for (int b = 0; b < h->nbatch; ++b)
        if (h->fin_h[b].t < a.t_end) done = false;
    return OECDG_OK;
}

// Copy the initial data into the stage buffer (unless the first stage reads it
// in place), clear the step records and take the statistics that the first
// stage reads.
int run_prologue(oecdg_handle *h, const StageArgs &a, const double *uC, const double *uD, bool copy = true) {
    if (copy) {
        HIPCHK(h, hipMemcpyAsync(a.BC[0], uC, sizeof(double) * h->totC, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(a.BD[0], uD, sizeof(double) * h->totD, hipMemcpyDeviceToDevice, h->stream));
    }
    StageArgs st = a;
    st.srcC = copy ? a.BC[0] : const_cast<double *>(uC);
    st.srcD = copy ? a.BD[0] : const_cast<double *>(uD);
    st.init_records = 1;                     // the step records cleared by the statistics kernel
    return stats_all(h, st);
}

// Runs of at most this many steps are replayed as one captured graph.
constexpr long long kWholeRunSteps = 256;

// A whole short run as one graph: the statistics of u^0 (whose kernel also
// clears the step records), every step, and the final OE into (uC, uD), whose
// kernel also writes the step records and the error flags into the host's
// mapped copy of them.  The first stage reads (uC, uD) in place (step 0 always
// runs: t_end > 0), so the initial data are not copied; a run of no steps
// copies them, for the final OE to read.
int run_whole(oecdg_handle *h, const StageArgs &a, double *uC, double *uD, long long limit) {
    key_graphs(h, a);
    if (!h->whole || h->w_uC != uC || h->w_uD != uD || h->w_limit != limit) {
        if (h->whole) (void)hipGraphExecDestroy(h->whole), h->whole = nullptr;
        int rc = capture(h, [&] {
            const bool inplace = limit > 0;
            int r = run_prologue(h, a, uC, uD, !inplace);
            if (r == OECDG_OK) r = launch_steps(h, a, 0, limit, inplace ? uC : nullptr, inplace ? uD : nullptr);
            StageArgs f = a;
            f.dstC = uC;
            f.dstD = uD;
            f.fin_host = h->fin_hd;          // the final kernel writes the records to the host
            f.err_host = h->err_hd;
            if (r == OECDG_OK) r = final_all(h, f);
            return r;
        }, &h->whole);
        if (rc != OECDG_OK) return rc;
        h->w_uC = uC;
        h->w_uD = uD;
        h->w_limit = limit;
    }
    HIPCHK(h, hipGraphLaunch(h->whole, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return OECDG_OK;
}

int run_1d(oecdg_handle *h, double *uC, double *uD, double t_end, int64_t nsteps, double dt_fixed, double *t_out,
           int64_t *steps_out) {
    if (nsteps < 0 && !(t_end < INFINITY)) return fail(h, OECDG_EINVAL, "run needs a finite t_end or nsteps >= 0");
    if (!(t_end > 0.0)) return fail(h, OECDG_EINVAL, "t_end must be positive");
    for (int b = 0; b < h->nbatch; ++b)
        if (h->inst_h[b].bc == OECDG_BC_INFLOW && !h->inflow_set[b])
            return fail(h, OECDG_EINVAL, "inflow instance " + std::to_string(b) + " has no ghost states (oecdg_set_inflow)");
    StageArgs a = base_args(h);
    a.t_end = t_end;
    a.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
    const long long limit = nsteps >= 0 ? nsteps : LLONG_MAX;

    int mode = h->mode;
    if (mode == OECDG_MODE_AUTO) mode = OECDG_MODE_GRAPH;
    if (mode == OECDG_MODE_PERSISTENT && ((h->nbatch > 1 && nsteps < 0) || h->groups.size() != 1))
        mode = OECDG_MODE_GRAPH;   // one cooperative launch serves one degree
    if (mode == OECDG_MODE_GRAPH && limit <= kWholeRunSteps) {
        int rc = run_whole(h, a, uC, uD, limit);
        if (rc != OECDG_OK) return rc;
        rc = errors_from_host(h);
        if (t_out) *t_out = h->fin_h[0].t;
        if (steps_out) *steps_out = h->fin_h[0].nexec;
        return rc;
    }
    int rc0 = run_prologue(h, a, uC, uD);
    if (rc0 != OECDG_OK) return rc0;
    if (mode == OECDG_MODE_PERSISTENT) {
        int maxg = persistent_max_grid_1d(h->kmax, h->flux, h->tile, h->tailwave);
        int grid = h->grid > 0 ? h->grid : (int)h->tiles_h.size();
        if (grid > maxg) grid = maxg;
        if (grid <= 0) return fail(h, OECDG_EHIP, "persistent kernel cannot be made co-resident");
        StageArgs p = a;
        p.coherent = 1;
        p.red = nullptr;                   // the persistent kernel reduces in-kernel
        HIPCHK(h, launch_persistent_1d(p, h->kmax, h->flux, h->tile, grid, limit, h->stream));
    } else if (limit > 0) {
        int rc;
        if ((rc = launch_steps(h, a, 0, 1)) != OECDG_OK) return rc;   // step 0: no OE on the initial data
        long long n = 1, prev = -1;
        const long long G = h->graph_steps;
        if (mode == OECDG_MODE_GRAPH && (rc = ensure_graph(h, a)) != OECDG_OK) return rc;
        while (n < limit) {
            const long long chunk = std::min(G, limit - n);
            if (mode == OECDG_MODE_GRAPH && chunk == G) {
                HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
            } else if (mode == OECDG_MODE_GRAPH) {
                if ((rc = launch_remainder(h, a, chunk)) != OECDG_OK) return rc;
            } else if ((rc = launch_steps(h, a, n, chunk)) != OECDG_OK) {
                return rc;
            }
            n += chunk;
            bool done = false;
            long long exec0 = 0;
            if ((rc = all_done(h, a, done, exec0)) != OECDG_OK) return rc;
            if (done) break;
            if (exec0 == prev && h->nbatch == 1) return fail(h, OECDG_EINVAL, "time stepping made no progress");
            prev = exec0;
        }
    }
    StageArgs f = a;
    f.dstC = uC;
    f.dstD = uD;
    int rcf = final_all(h, f);
    if (rcf != OECDG_OK) return rcf;
    HIPCHK(h, hipMemcpyAsync(h->fin_h, h->fin, rec_bytes(h->nbatch), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    int rc = errors_from_host(h);
    if (t_out) *t_out = h->fin_h[0].t;
    if (steps_out) *steps_out = h->fin_h[0].nexec;
    return rc;
}

}  // namespace

// Discrete adjoint of a fixed-step run (scalar periodic 1D).  Pass 1 runs the
// forward steps and keeps the damped state every `ckpt` steps.  Then, segment
// by segment from the end, the forward kernels recompute the segment keeping
// every stage's undamped output h and its per-tile partial statistics, and the
// adjoint kernels walk the stages backwards.  The segment states live in two
// buffers (segment sg in buffer sg & 1): the recomputation of segment sg - 1
// runs on a second stream while the reverse stages of segment sg run on the
// caller's stream, and events order the buffer hand-overs.
int oecdg::adjoint_1d(oecdg_handle *h, const double *uC0, const double *uD0, int64_t nsteps, double dt,
                      const double *gCT, const double *gDT, double *gC0, double *gD0, int ckpt) {
    const Inst1D I = h->inst_h[0];
    if (I.nc != 1 || I.bc != OECDG_BC_PERIODIC || I.flux == OECDG_FLUX_EULER)
        return fail(h, OECDG_EUNSUPPORTED, "adjoint: scalar flux on a periodic mesh only");
    const int n = I.np, K1 = I.k + 1;
    const size_t S = (size_t)K1 * n, S2 = 2 * S;           // one mesh, both meshes
    const long long nseg = nsteps > 0 ? (nsteps + ckpt - 1) / ckpt : 0;
    const long long n0L = nseg > 0 ? (nseg - 1) * ckpt : 0;  // first step of the last segment
    const size_t ntile = h->ncol, psz = (size_t)NSTAT * ntile;   // partial columns (periodic: one per tile)
    const int NB = adj_block_size(), nb = (n + NB - 1) / NB;
    const size_t bpsz = (size_t)2 * nb * adj_block_partials();
    const size_t segsz = (size_t)ckpt * 6 * S2 + (size_t)ckpt * 3 * psz;
    const size_t slotsz = (2 * sizeof(Slot) + sizeof(Final) + sizeof(double) - 1) / sizeof(double);
    // workspace: checkpoints | 2 x segment (states, 6 per step | partials, 3 per step) |
    //            2 adjoints | acc | 2 x (lp, cR, cL) | 2 x block partials | step slots of the second stream
    const size_t need = (size_t)std::max<long long>(nseg, 1) * S2 + 2 * segsz + 9 * S2 + 2 * bpsz + slotsz;
    if (!h->aux) HIPCHK(h, hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    for (hipEvent_t &e : h->adj_ev)
        if (!e) HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (need * sizeof(double) > h->adj_bytes) {
        HIPCHK(h, hipStreamSynchronize(h->aux));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipFree(h->adj_ws);
        h->adj_ws = nullptr;
        h->adj_bytes = 0;
        if (hipMalloc(&h->adj_ws, need * sizeof(double)) != hipSuccess) return fail(h, OECDG_ENOMEM, "adjoint workspace");
        h->adj_bytes = need * sizeof(double);
    }
    double *ck = h->adj_ws;
    double *segb[2] = {ck + (size_t)std::max<long long>(nseg, 1) * S2, nullptr};
    segb[1] = segb[0] + segsz;
    double *buf = segb[1] + segsz;
    double *lamA = buf, *lamB = buf + S2, *acc = buf + 2 * S2;
    double *prepv[2][3] = {{buf + 3 * S2, buf + 4 * S2, buf + 5 * S2}, {buf + 6 * S2, buf + 7 * S2, buf + 8 * S2}};
    double *bpv[2] = {buf + 9 * S2, buf + 9 * S2 + bpsz};
    double *slotmem = bpv[1] + bpsz;
    // stage states and partials of step j of the segment in buffer b
    auto st = [&](int b, long long j, int which) {           // 0 s0 (damped u^n), 1 h1, 3 h2, 5 h3 (2, 4 unused)
        return segb[b] + ((size_t)j * 6 + which) * S2;
    };
    auto pp = [&](int b, long long j, int l) { return segb[b] + (size_t)ckpt * 6 * S2 + ((size_t)j * 3 + l) * psz; };
    hipEvent_t *ready = h->adj_ev, *freed = h->adj_ev + 2, ckdone = h->adj_ev[4];

    StageArgs base = base_args(h);
    base.dt_fixed = dt;
    base.t_end = INFINITY;
    base.red = nullptr;                                      // the recomputation reduces in-kernel
    StageArgs baux = base;                                   // the second stream keeps its own step slots
    baux.slots = (Slot *)slotmem;
    baux.fin = (Final *)((Slot *)slotmem + 2);
    int rc;
    // Stage l of step nn (step j of the segment in buffer b), keeping every
    // stage state and its partial statistics; (inC, inD, inP) is the undamped
    // input and its partials.
    auto seg_stage = [&](const StageArgs &sa, int b, long long nn, long long j, int l, const double *inC,
                         const double *inD, double *inP, bool first, hipStream_t s) {
        StageArgs a = sa;
        a.l = l;
        a.par = (int)(nn & 1);
        a.first = first;
        const int sp = (a.par + l) & 1;
        double *out = st(b, j, 2 * l + 1);
        a.BC[sp] = const_cast<double *>(inC);
        a.BD[sp] = const_cast<double *>(inD);
        a.BC[sp ^ 1] = out;
        a.BD[sp ^ 1] = out + S;
        a.UC = st(b, j, 0);
        a.UD = st(b, j, 0) + S;
        a.DC = nullptr;                                      // s_1, s_2 are formed again by the reverse stages
        a.DD = nullptr;
        a.part[sp] = pp(b, j, l);
        a.part[sp ^ 1] = inP;
        for (const auto &g : h->groups) {
            StageArgs c = a;
            c.tbeg = g.tbeg;
            c.tend = g.tend;
            HIPCHK(h, launch_stage_1d(c, g.k, h->flux, h->tile, s));
        }
        return (int)OECDG_OK;
    };
    // pass 1: forward from u^0, keeping u^n at n = 0, ckpt, 2 ckpt, ... and
    // every stage of the last segment (which then needs no recomputation)
    const int bL = (int)((nseg - 1) & 1);
    HIPCHK(h, hipMemcpyAsync(ck, uC0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(ck + S, uD0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(base.BC[0], uC0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(base.BD[0], uD0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, launch_init_1d(base, 1, h->stream));
    HIPCHK(h, launch_init_1d(baux, 1, h->stream));
    for (long long nn = 0; nn < nsteps; ++nn) {
        for (int l = 0; l < 3; ++l) {
            if (nn >= n0L) {
                const long long j = nn - n0L;
                if (l > 0)
                    rc = seg_stage(base, bL, nn, j, l, st(bL, j, 2 * l - 1), st(bL, j, 2 * l - 1) + S, pp(bL, j, l - 1),
                                   false, h->stream);
                else if (j > 0)
                    rc = seg_stage(base, bL, nn, j, 0, st(bL, j - 1, 5), st(bL, j - 1, 5) + S, pp(bL, j - 1, 2), false,
                                   h->stream);
                else {
                    const int sp = (int)(nn & 1);
                    rc = seg_stage(base, bL, nn, 0, 0, base.BC[sp], base.BD[sp], base.part[sp ^ 1], nn == 0,
                                   h->stream);
                }
                if (rc != OECDG_OK) return rc;
                continue;
            }
            StageArgs a = base;
            a.l = l;
            a.par = (int)(nn & 1);
            a.first = nn == 0;
            if (nn % ckpt == 0) {                            // u^n is read back by stages 1 and 2
                a.UC = ck + (nn / ckpt) * S2;
                a.UD = a.UC + S;
            }
            if ((rc = stage_all(h, a)) != OECDG_OK) return rc;
        }
        if (nseg >= 2 && nn == (nseg - 2) * ckpt)           // the last checkpoint a recomputation reads
            HIPCHK(h, hipEventRecord(ckdone, h->stream));
    }
    // Recompute segment sg (all of its steps are whole) into buffer sg & 1 on
    // the second stream, once the reverse stages have released that buffer.
    auto recompute = [&](long long sg) -> int {
        const int b = (int)(sg & 1);
        if (sg == nseg - 2) HIPCHK(h, hipStreamWaitEvent(h->aux, ckdone, 0));
        else HIPCHK(h, hipStreamWaitEvent(h->aux, freed[b], 0));
        const long long n0 = sg * ckpt;
        for (long long j = 0; j < ckpt; ++j)
            for (int l = 0; l < 3; ++l) {
                const long long nn = n0 + j;
                int r;
                if (l > 0)
                    r = seg_stage(baux, b, nn, j, l, st(b, j, 2 * l - 1), st(b, j, 2 * l - 1) + S, pp(b, j, l - 1),
                                  false, h->aux);
                else if (j > 0)
                    r = seg_stage(baux, b, nn, j, 0, st(b, j - 1, 5), st(b, j - 1, 5) + S, pp(b, j - 1, 2), false,
                                  h->aux);
                else                                         // the checkpoint is already damped
                    r = seg_stage(baux, b, nn, 0, 0, ck + sg * S2, ck + sg * S2 + S, pp(b, 0, 2), true, h->aux);
                if (r != OECDG_OK) return r;
            }
        HIPCHK(h, hipEventRecord(ready[b], h->aux));
        return OECDG_OK;
    };
    // backward
    HIPCHK(h, hipMemcpyAsync(lamA, gCT, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(lamA + S, gDT, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    double *lam = lamA, *lam_next = lamB;
    AdjArgs q;
    memset(&q, 0, sizeof(q));
    q.k = I.k;
    q.flux = I.flux;
    q.n = n;
    q.nb = nb;
    q.nbp = nb * adj_waves();
    q.S = (long long)S;
    q.hinv = 1.0 / I.h;
    q.p0 = I.p0;
    q.tau = dt;
    q.inv_tm = 1.0 / dt;
    q.inv_n = 1.0 / n;
    q.ftile0 = I.tile0;
    q.fntiles = I.npart;
    q.acc = acc;
    q.oe = I.oe && I.k > 0;
    static const double AL[3] = {0.0, 0.75, 1.0 / 3.0}, BL[3] = {1.0, 0.25, 2.0 / 3.0};
    int cur = 0;                                             // the preparation set the next launch reads
    auto set_out = [&](AdjArgs &a, int w) {
        a.lp = prepv[w][0], a.cr = prepv[w][1], a.cl = prepv[w][2], a.bp = bpv[w];
    };
    auto set_in = [&](AdjArgs &a, int r) {
        a.lp_in = prepv[r][0], a.cr_in = prepv[r][1], a.cl_in = prepv[r][2], a.bp_in = bpv[r];
    };
    // the reverse stages of segment sg, from buffer sg & 1
    auto reverse = [&](long long sg) -> int {
        const int b = (int)(sg & 1);
        const long long m = std::min<long long>(ckpt, nsteps - sg * ckpt);
        if (sg != nseg - 1) HIPCHK(h, hipStreamWaitEvent(h->stream, ready[b], 0));
        if (q.oe) {                                          // prepare the OE of the segment's last stage
            AdjArgs a = q;
            a.do_rk = 0;
            a.do_prep = 1;
            a.lam = lam;
            a.h = st(b, m - 1, 5);
            a.fpart = pp(b, m - 1, 2);
            set_out(a, cur);
            HIPCHK(h, launch_adj(a, h->stream));
        }
        for (long long j = m - 1; j >= 0; --j)
            for (int l = 2; l >= 0; --l) {
                AdjArgs a = q;
                a.do_rk = 1;
                // s_l is read for the first stage of a step (u^n, damped); for
                // l > 0 the pointer is h_l, damped inside the reverse stage
                a.s = l == 0 ? st(b, j, 0) : st(b, j, 2 * l - 1);
                a.lam = lam;
                a.out = lam_next;
                a.al = AL[l];
                a.bl = BL[l];
                a.stage0 = l == 0;
                a.acc_init = l == 2;
                set_in(a, cur);
                set_out(a, cur ^ 1);
                a.do_prep = l > 0 || j > 0;
                a.h = l > 0 ? st(b, j, 2 * l - 1) : (j > 0 ? st(b, j - 1, 5) : nullptr);
                a.fpart = l > 0 ? pp(b, j, l - 1) : (j > 0 ? pp(b, j - 1, 2) : nullptr);
                HIPCHK(h, launch_adj(a, h->stream));
                cur ^= 1;
                std::swap(lam, lam_next);
            }
        HIPCHK(h, hipEventRecord(freed[b], h->stream));
        return OECDG_OK;
    };
    // recompute(sg - 1) is issued before reverse(sg): the two run side by side
    rc = OECDG_OK;
    if (nseg >= 2) rc = recompute(nseg - 2);
    for (long long sg = nseg - 1; sg >= 0 && rc == OECDG_OK; --sg) {
        if ((rc = reverse(sg)) != OECDG_OK) break;
        if (sg >= 2) rc = recompute(sg - 2);
    }
    if (rc != OECDG_OK) {                                    // nothing may still write the workspace
        (void)hipStreamSynchronize(h->aux);
        return rc;
    }
    HIPCHK(h, hipMemcpyAsync(gC0, lam, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(gD0, lam + S, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    return check_errors(h);
}

hipStream_t oecdg::handle_stream(oecdg_handle *h) { return h->stream; }
const oecdg_desc &oecdg::handle_desc(oecdg_handle *h) { return h->desc[0]; }
void *&oecdg::handle_ext2d(oecdg_handle *h) { return h->ext2d; }
void *&oecdg::handle_extnu(oecdg_handle *h) { return h->extnu; }
int oecdg::handle_nbatch(oecdg_handle *h) { return h->nbatch; }
int oecdg::handle_fail(oecdg_handle *h, int code, const char *msg) { return fail(h, code, msg); }

// ============================================================== C ABI ===

extern "C" {

int oecdg_state_size(const oecdg_desc *d, int64_t *n_primal, int64_t *n_dual) {
    if (!d || !n_primal || !n_dual) return OECDG_EINVAL;
    const char *why = "";
    int rc = validate(*d, why);
    if (rc != OECDG_OK) return rc;
    sizes(*d, *n_primal, *n_dual);
    return OECDG_OK;
}

int oecdg_init(const oecdg_desc *d, int32_t nbatch, void *stream, oecdg_handle **out) {
    if (!d || !out || nbatch < 1) return OECDG_EINVAL;
    *out = nullptr;
    oecdg_handle *h = new (std::nothrow) oecdg_handle();
    if (!h) return OECDG_ENOMEM;
    h->nbatch = nbatch;
    h->stream = (hipStream_t)stream;
    h->desc.assign(d, d + nbatch);
    h->dim = d[0].dim;
    for (int b = 0; b < nbatch; ++b) {
        const char *why = "";
        int rc = validate(d[b], why);
        if (rc == OECDG_OK && d[b].dim != h->dim) rc = OECDG_EINVAL, why = "mixed dimensions in one batch";
        if (rc == OECDG_OK && nbatch > 1 && d[b].dim != 1) rc = OECDG_EUNSUPPORTED, why = "batches are 1D only";
        if (rc == OECDG_OK && d[b].flux != d[0].flux) rc = OECDG_EUNSUPPORTED, why = "one flux per batch";
        if (rc == OECDG_OK && (d[b].rk == 0 ? 3 : d[b].rk) != (d[0].rk == 0 ? 3 : d[0].rk))
            rc = OECDG_EUNSUPPORTED, why = "one RK method per batch";
        if (rc != OECDG_OK) {
            delete h;
            return rc;
        }
    }
    int rc = OECDG_OK;
    h->rk = d[0].rk == 0 ? 3 : d[0].rk;
    if (h->dim == 2) {
        rc = oecdg::create_2d(h, d);
        if (rc != OECDG_OK) {
            oecdg::destroy_2d(h);
            delete h;
            return rc;
        }
        *out = h;
        return OECDG_OK;
    }
    h->flux = d[0].flux;
    for (int b = 0; b < nbatch; ++b)       // kernels with the ghost code only where an instance has walls or inflow
        if (d[b].bc == OECDG_BC_REFLECTIVE || d[b].bc == OECDG_BC_INFLOW) h->flux = 3;
    h->inflow_set.assign(nbatch, 0);
    h->rk = d[0].rk == 0 ? 3 : d[0].rk;
    h->offC.assign(nbatch + 1, 0);
    h->offD.assign(nbatch + 1, 0);
    for (int b = 0; b < nbatch; ++b) {
        const oecdg_desc &e = d[b];
        Inst1D I = make_inst(e);
        int64_t np, nd;
        sizes(e, np, nd);
        I.offC = h->offC[b];
        I.offD = h->offD[b];
        h->offC[b + 1] = h->offC[b] + np;
        h->offD[b + 1] = h->offD[b] + nd;
        h->inst_h.push_back(I);
        if (e.k > h->kmax) h->kmax = e.k;
    }
    h->totC = h->offC[nbatch];
    h->totD = h->offD[nbatch];
    int64_t maxn = 0;
    for (auto &I : h->inst_h) maxn = I.nd > maxn ? I.nd : maxn;
    h->tile = default_tile(maxn, nbatch);
#define ALLOC(ptr, bytes)                                                    \
    do {                                                                     \
        if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                      \
            oecdg_destroy(h);                                                \
            return OECDG_ENOMEM;                                             \
        }                                                                    \
    } while (0)
    ALLOC(h->inst_d, sizeof(Inst1D) * nbatch);
    ALLOC(h->slots, sizeof(Slot) * 2 * nbatch);
    // the step records and, right after them, the four error flags: one block,
    // so that one copy brings both to the host
    ALLOC(h->fin, rec_bytes(nbatch));
    h->err = reinterpret_cast<int *>(reinterpret_cast<char *>(h->fin) + sizeof(Final) * nbatch);
    ALLOC(h->B, sizeof(double) * 2 * (h->totC + h->totD));
    ALLOC(h->U, sizeof(double) * (h->totC + h->totD));
    if (h->rk == 4) ALLOC(h->A, sizeof(double) * (h->totC + h->totD));
    ALLOC(h->bar, sizeof(unsigned) * 2);
    ALLOC(h->red, sizeof(double) * NSTAT * nbatch);
#undef ALLOC
    if (hipHostMalloc((void **)&h->fin_h, rec_bytes(nbatch), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&h->fin_hd, h->fin_h, 0) != hipSuccess) {
        oecdg_destroy(h);
        return OECDG_ENOMEM;
    }
    h->err_h = reinterpret_cast<int *>(reinterpret_cast<char *>(h->fin_h) + sizeof(Final) * nbatch);
    h->err_hd = reinterpret_cast<int *>(reinterpret_cast<char *>(h->fin_hd) + sizeof(Final) * nbatch);
    rc = build_tiles(h);
    if (rc != OECDG_OK) {
        oecdg_destroy(h);
        return rc;
    }
    *out = h;
    return OECDG_OK;
}

int oecdg_batch_offsets(oecdg_handle *h, int64_t *off_primal, int64_t *off_dual) {
    if (!h || !off_primal || !off_dual) return OECDG_EINVAL;
    if (h->dim != 1) {
        int64_t np, nd;
        sizes(h->desc[0], np, nd);
        off_primal[0] = off_dual[0] = 0;
        off_primal[1] = np;
        off_dual[1] = nd;
        return OECDG_OK;
    }
    for (int b = 0; b <= h->nbatch; ++b) {
        off_primal[b] = h->offC[b];
        off_dual[b] = h->offD[b];
    }
    return OECDG_OK;
}

int oecdg_set_option(oecdg_handle *h, int32_t key, int64_t value) {
    if (!h) return OECDG_EINVAL;
    switch (key) {
    case OECDG_OPT_MODE:
        if (value < 0 || value > 3) return fail(h, OECDG_EINVAL, "unknown mode");
        h->mode = (int)value;
        return OECDG_OK;
    case OECDG_OPT_TILE:
        if (value != 32 && value != 64 && value != 128) return fail(h, OECDG_EINVAL, "tile must be 32, 64 or 128");
        if (h->dim != 1) return OECDG_OK;
        h->tile = (int)value;
        return build_tiles(h);
    case OECDG_OPT_GRAPH_STEPS:
        if (value < 1 || value > 4096) return fail(h, OECDG_EINVAL, "graph steps must be 1..4096");
        h->graph_steps = (int)((value + 1) / 2 * 2);       // even: parities of the captured nodes repeat
        return OECDG_OK;
    case OECDG_OPT_GRID:
        if (value < 0 || value > (1 << 20)) return fail(h, OECDG_EINVAL, "grid out of range");
        h->grid = (int)value;
        return OECDG_OK;
    case OECDG_OPT_FOLD:
        if (value < 0 || value > 2) return fail(h, OECDG_EINVAL, "fold must be 0 (auto), 1 (in-kernel) or 2 (fold kernel)");
        h->fold = (int)value;
        return OECDG_OK;
    }
    return fail(h, OECDG_EINVAL, "unknown option");
}

int oecdg_set_inflow(oecdg_handle *h, int32_t instance, const double *left, const double *right) {
    if (!h || !left || !right) return OECDG_EINVAL;
    if (h->dim != 1 || instance < 0 || instance >= h->nbatch) return fail(h, OECDG_EINVAL, "instance out of range");
    Inst1D &I = h->inst_h[instance];
    if (I.bc != OECDG_BC_INFLOW) return fail(h, OECDG_EINVAL, "the instance has no inflow boundaries");
    for (int q = 0; q < I.nc; ++q) {
        I.gin[0][q] = left[q];
        I.gin[1][q] = right[q];
    }
    HIPCHK(h, hipMemcpy(h->inst_d + instance, &I, sizeof(Inst1D), hipMemcpyHostToDevice));
    h->inflow_set[instance] = 1;
    drop_graphs(h);                          // single-instance graphs hold the instance in their arguments
    return OECDG_OK;
}

int oecdg_dt(oecdg_handle *h, const double *uC, const double *uD, double *dt_out) {
    if (!h || !uC || !uD || !dt_out) return OECDG_EINVAL;
    if (h->dim != 1) {
        return oecdg::dt_2d(h, uC, uD, dt_out);
    }
    StageArgs a = base_args(h);
    a.srcC = uC;
    a.srcD = uD;
    int rcs = stats_all(h, a);
    if (rcs != OECDG_OK) return rcs;
    const Inst1D &I = h->inst_h[0];
    std::vector<double> recs((size_t)NSTAT * I.npart);        // the instance's tile records
    HIPCHK(h, hipMemcpyAsync(recs.data(), a.part[1] + (size_t)I.tile0 * NSTAT, sizeof(double) * recs.size(),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double beta = 0.0;
    for (int t = 0; t < I.npart; ++t)
        for (int j = 0; j < 2; ++j) beta = std::fmax(beta, recs[(size_t)t * NSTAT + ST_BETA + j]);
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(h, OECDG_ENONFINITE, "wave speed is zero or not finite");
    *dt_out = I.cfl * I.h / beta;
    return OECDG_OK;
}

int oecdg_stage(oecdg_handle *h, int32_t stage, double dt, double tau_max, const double *uC_n, const double *uD_n,
                const double *uC_l, const double *uD_l, double *uC_out, double *uD_out) {
    if (!h || !uC_n || !uD_n || !uC_out || !uD_out) return OECDG_EINVAL;
    const int ns = rk_stages(h->rk);
    if (stage < 0 || stage >= ns) return fail(h, OECDG_EINVAL, "stage out of range for the RK method");
    if (h->rk == 4 && stage == 3)
        return fail(h, OECDG_EUNSUPPORTED, "the last stage of classical RK4 reads the earlier stages");
    if (!(dt > 0.0) || !(tau_max > 0.0)) return fail(h, OECDG_EINVAL, "dt and tau_max must be positive");
    if (stage > 0 && (!uC_l || !uD_l)) return fail(h, OECDG_EINVAL, "stages after the first need u_l");
    if (h->dim != 1) {
        return oecdg::stage_2d(h, stage, dt, tau_max, uC_n, uD_n, uC_l, uD_l, uC_out, uD_out);
    }
    if (h->nbatch != 1) return fail(h, OECDG_EUNSUPPORTED, "oecdg_stage takes single-instance handles");
    StageArgs a = base_args(h);
    const int sp = stage & 1;                 // step index 0: global stage parity = stage
    a.l = stage;                              // a.rk, a.ns: the handle's method (base_args)
    a.par = 0;
    a.first = 0;
    a.tau_override = dt;
    a.taumax_override = tau_max;
    a.damp_input = 0;
    a.red = nullptr;                          // no statistics enter a single stage
    a.BC[sp] = const_cast<double *>(stage == 0 ? uC_n : uC_l);
    a.BD[sp] = const_cast<double *>(stage == 0 ? uD_n : uD_l);
    a.UC = const_cast<double *>(uC_n);
    a.UD = const_cast<double *>(uD_n);
    // the library's stage buffers receive the undamped output
    a.BC[sp ^ 1] = h->B + (sp ^ 1) * h->totC;
    a.BD[sp ^ 1] = h->B + 2 * h->totC + (sp ^ 1) * h->totD;
    HIPCHK(h, launch_init_1d(a, 1, h->stream));
    int rcs = stage_all(h, a);
    if (rcs != OECDG_OK) return rcs;
    // final OE with (tau, executed steps) chosen so that it reads that output:
    // counted as stage + 1 steps of a three-stage method, the buffer parity of
    // the final kernel is that of the stage's output
    Final f{0.0, dt, (long long)stage + 1};
    HIPCHK(h, hipMemcpyAsync(h->fin, &f, sizeof(Final), hipMemcpyHostToDevice, h->stream));
    a.ns = 3;
    a.dstC = uC_out;
    a.dstD = uD_out;
    int rcf = final_all(h, a);
    if (rcf != OECDG_OK) return rcf;
    return check_errors(h);
}

int oecdg_run(oecdg_handle *h, double *uC, double *uD, double t_end, int64_t nsteps, double dt_fixed, double *t_out,
              int64_t *steps_out) {
    if (!h || !uC || !uD) return OECDG_EINVAL;
    if (h->dim != 1) {
        return oecdg::run_2d(h, uC, uD, t_end, nsteps, dt_fixed, t_out, steps_out);
    }
    return run_1d(h, uC, uD, t_end, nsteps, dt_fixed, t_out, steps_out);
}

int oecdg_run_nonuniform(oecdg_handle *h, const double *edges, double *uC, double *uD, double t_end, int64_t nsteps,
                         double dt_fixed, double *t_out, int64_t *steps_out) {
    if (!h) return OECDG_EINVAL;
    return oecdg::run_nonuniform(h, edges, uC, uD, t_end, nsteps, dt_fixed, t_out, steps_out);
}

int oecdg_adjoint(oecdg_handle *h, const double *uC0, const double *uD0, int64_t nsteps, double dt,
                  const double *gC_T, const double *gD_T, double *gC0, double *gD0, int32_t checkpoint_every) {
    if (!h || !uC0 || !uD0 || !gC_T || !gD_T || !gC0 || !gD0) return OECDG_EINVAL;
    if (h->dim != 1 || h->nbatch != 1) return fail(h, OECDG_EUNSUPPORTED, "adjoint: 1D single instance only");
    if (h->rk != 3) return fail(h, OECDG_EUNSUPPORTED, "adjoint: SSP-RK3 only");
    if (nsteps < 0 || !(dt > 0.0) || checkpoint_every < 1) return fail(h, OECDG_EINVAL, "adjoint: bad nsteps/dt/checkpoint");
    return oecdg::adjoint_1d(h, uC0, uD0, nsteps, dt, gC_T, gD_T, gC0, gD0, checkpoint_every);
}

void oecdg_destroy(oecdg_handle *h) {
    if (!h) return;
    drop_graphs(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->aux) (void)hipStreamSynchronize(h->aux), (void)hipStreamDestroy(h->aux);
    for (hipEvent_t e : h->adj_ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(h->adj_ws);
    (void)hipFree(h->inst_d);
    (void)hipFree(h->tiles_d);
    (void)hipFree(h->slots);
    (void)hipFree(h->fin);
    (void)hipFree(h->part);
    (void)hipFree(h->B);
    (void)hipFree(h->U);
    (void)hipFree(h->A);
    (void)hipFree(h->bar);
    (void)hipFree(h->red);
    if (h->fin_h) (void)hipHostFree(h->fin_h);
    if (h->ext2d) {
        oecdg::destroy_2d(h);
    }
    if (h->extnu) oecdg::destroy_nu(h);
    delete h;
}

const char *oecdg_strerror(int code) {
    switch (code) {
    case OECDG_OK: return "success";
    case OECDG_EINVAL: return "invalid argument";
    case OECDG_ENOMEM: return "out of memory";
    case OECDG_EHIP: return "HIP runtime error";
    case OECDG_ENONFINITE: return "non-finite value produced";
    case OECDG_ENONPHYSICAL: return "non-physical state (density or pressure <= 0)";
    case OECDG_EUNSUPPORTED: return "unsupported configuration";
    case OECDG_ETIMEOUT: return "device barrier timeout";
    case OECDG_ETOOBIG: return "problem larger than the fixed device scratch of oecdg_run_noalloc";
    }
    return "unknown error";
}

const char *oecdg_last_error(oecdg_handle *h) { return h ? h->last.c_str() : "null handle"; }

}  // extern "C"
