// oecdg_1d.hip -- gfx950 kernels of the 1D RK-OECDG stage update.
//
// One workgroup owns a tile of T primal cells [i0, i0+T) and the T dual cells
// [i0, i0+T) that interleave with them (dual cell j is centred on the left
// edge of primal cell j), one thread per cell, and one more wave whose lanes
// take the cells next to the tile that its operator reads (the primal cells
// i0-1 and i0+T, the dual cell i0+T) and the dual cells i0-1 and i0+T+1 that
// the damping of those primal cells reads.  A stage kernel for stage l of step n
//   1. issues every independent load at once: the step records, the previous
//      stage's per-tile partial statistics, each thread's cell, undamped (ghost
//      cells at non-periodic ends built from the end cells), and its u^n; the
//      undamped cells go to an LDS image, from which each thread takes the two
//      cells of the other mesh that overlap its own;
//   2. reduces the partial statistics (fixed order, so every workgroup gets
//      bit-identical avg/sigma/beta), and at l = 0 derives tau^n and
//      tau_max^n (Sec. 2.1, tau = C h / beta);
//   3. applies the OE step F_tau of the previous stage to its cell in
//      registers (Sec. 2.2, OEstep2D: delta_K^m from the primal/dual
//      difference at the cell edges, then the exact exponential
//      a_j *= exp(-tau sum_{m<=j} delta^m)) and puts the damped cell in LDS;
//   4. evaluates the CDG operator (equcdg) on its cell from the damped cells in
//      LDS: the overlap coupling with 1/tau_max, the volume integral of f(w)
//      with k+1 Gauss nodes on each half cell, and the point fluxes of the other
//      mesh at the cell edges;
//   5. forms the RK combination of eq:RKCDG (SSP-RK3 by default; forward
//      Euler, SSP-RK2 or classical RK4 on request) and writes the stage output;
//   6. writes the tile's partial statistics of that output for the next stage
//      (DPP reductions within the waves that hold each mesh; the wave speeds
//      only after a step's last stage, the one whose output sets the next tau).
// The OE of the last stage of a run is applied by the final kernel.
#include "oecdg_device.h"
#include "oecdg_internal.h"
#include "oecdg_tables.h"

#include <math.h>
#include <string.h>

namespace oecdg {

// Threads per workgroup: one per cell for the T primal and the T dual cells of
// a tile, and one wave for the cells next to it.
__host__ __device__ constexpr int nthreads(int T) { return 2 * T + WAVE; }

// ------------------------------------------------------------ cell kernels ---

// Damping factors of one cell: fac[j] = exp(-tau * sum_{m<=j} delta^m), j >= 1,
// delta^m = (2m+1) 2^m / ((2k-1) m! h) * max_q beta (|dR_q| + |dL_q|) / sigma_q
// with dR, dL the xi-derivatives of order m of (own trace - other mesh at its
// centre) at the right and left edge; components with sigma_q = 0 are skipped.
template <int K, int NC>
__device__ inline void oe_factors(const double (&own)[NC][K + 1], const double (&nl)[NC][K + 1],
                                  const double (&nr)[NC][K + 1], double beta, const double *sig, double hinv,
                                  double tau, double (&fac)[K + 1]) {
    constexpr Tab<K> tb = make_tab<K>();
    fac[0] = 1.0;
    double S = 0.0;
#pragma unroll
    for (int m = 0; m <= K; ++m) {
        double dm = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            double ur = 0.0, ul = 0.0, vr = 0.0, vl = 0.0;
#pragma unroll
            for (int n = m; n <= K; ++n) {
                const double d1 = tb.D1[m][n];
                ur += own[q][n] * d1;
                ul += own[q][n] * (((n + m) & 1) ? -d1 : d1);
                vr += nr[q][n] * tb.D0[m][n];
                vl += nl[q][n] * tb.D0[m][n];
            }
            if (sig[q] != 0.0) {
                const double val = beta * (fabs(ur - vr) + fabs(ul - vl)) / sig[q];
                dm = fmax(dm, val);
            }
        }
        S += tb.C[m] * hinv * dm;
        if (m >= 1) fac[m] = exp(-tau * S);
    }
}

// Contribution of one half of a cell to tau_max times the time derivative of
// its modal coefficients (equcdg), without the cell's own coupling term -a_m:
//   (2m+1)/2 int_half w P_m + tau_max (2m+1)/h (int_half f(w) P_m' + edge term)
// The projection of w uses the exact overlap integrals of the Legendre modes
// (OV), so a component that is one constant on both meshes and carries no
// flux gets exactly zero rate once the caller subtracts a_m.  Right half
// (hf = 1): nb is the overlapping cell on the right, nodes xi_g = (s_g+1)/2,
// edge term -f(w(x_R)).  Left half (hf = 0): evaluated as the mirror image with
// the same nodes through P_n(-x) = (-1)^n P_n(x): the neighbour's odd modes,
// the test functions P_m (odd m) and P_m' (even m) change sign, and the edge
// term is +(-1)^m f(w(x_L)).  ft = tau_max / h.
template <int K, int FLUX>
__device__ inline void cdg_rate_half(const double (&nb)[FluxT<FLUX>::NC][K + 1], int hf, double p0, double ft,
                                     double (&r)[FluxT<FLUX>::NC][K + 1]) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC;
    constexpr Tab<K> tb = make_tab<K>();
    const double flip = hf ? 1.0 : -1.0;
    double c[NC][K + 1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int n = 0; n <= K; ++n) c[q][n] = (n & 1) ? flip * nb[q][n] : nb[q][n];
    double accf[NC][K + 1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m <= K; ++m) accf[q][m] = 0.0;
#pragma unroll
    for (int g = 0; g <= K; ++g) {
        double w[NC], fw[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            double v = 0.0;
#pragma unroll
            for (int n = 0; n <= K; ++n) v += c[q][n] * tb.E[1][g][n];
            w[q] = v;
        }
        F::f(w, fw, p0);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m <= K; ++m) accf[q][m] += tb.WD[1][g][m] * fw[q];
    }
    double wc[NC], fc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        double v = 0.0;
#pragma unroll
        for (int n = 0; n <= K; ++n) v += c[q][n] * tb.D0[0][n];
        wc[q] = v;
    }
    F::f(wc, fc, p0);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const double edge = hf ? -fc[q] : fc[q];
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            const double sw = (m & 1) ? flip : 1.0;
            const double sf = (m & 1) ? 1.0 : flip;
            double pw = 0.0;
#pragma unroll
            for (int n = 0; n <= K; ++n) pw += tb.OV[m][n] * c[q][n];
            r[q][m] = (m + 0.5) * (sw * pw) + (2.0 * m + 1.0) * ft * (sf * accf[q][m] + sw * edge);
        }
    }
}

// ------------------------------------------------------------ tile pieces ---

// Sign of coefficient (q, m) of a reflective ghost: (-1)^m, and -1 more for
// the momentum (q = 1 of the Euler system).
__device__ inline double mirror_sign(int q, int m) { return ((m & 1) ^ (q == 1)) ? -1.0 : 1.0; }

// Pre-damping coefficients of cell g of mesh `mesh` of instance I (input
// arrays inC, inD of the instance).  A primal index outside [0, np) (the ends
// of non-periodic meshes) is the ghost next to the end cell e: outflow the
// mean of e with zero higher modes, inflow the instance's fixed ghost state,
// reflective walls the mirror image of e (kernels of the walled Euler flux,
// FLUX == 3, which alone carry the wall and inflow ghosts).  A dual index
// outside [0, nd) reads as zeros.  Every load is of a valid element, with no
// branch between the loads.
template <int K, int FLUX>
__device__ inline void cell_pre(const Inst1D &I, int mesh, int g, const double *__restrict__ inC,
                                const double *__restrict__ inD, double (&u)[FluxT<FLUX>::NC][K + 1]) {
    constexpr int NC = FluxT<FLUX>::NC, K1 = K + 1;
    const int n = mesh == 0 ? I.np : I.nd;
    const bool in = g >= 0 && g < n;
    const int e = g < 0 ? 0 : (g >= n ? n - 1 : g);
    const double *src = mesh == 0 ? inC : inD;
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) {
            const double x = src[(long long)(q * K1 + m) * n + e];
            double v = m == 0 ? x : 0.0;                 // outflow ghost: constant extension
            if constexpr (FLUX == 3) {
                if (I.bc == 2) v = mirror_sign(q, m) * x;
                else if (I.bc == 3) v = m == 0 ? I.gin[g < 0 ? 0 : 1][q] : 0.0;
            }
            u[q][m] = in ? x : (mesh == 1 ? 0.0 : v);
        }
}

// The cell of this thread in the tile of instance I that starts at index i0,
// and its LDS column (both meshes: column g - i0 + 1 of cell g).  Threads
// [0, T): primal cell i0 + tid; [T, 2T): dual cell i0 + tid - T; the last
// wave: lane 0 the primal cell i0 - 1, lane 1 the dual cell i0 + T, lane 2 the
// primal cell i0 + T (the neighbours that the tile's operator reads, damped),
// lanes 3 and 4 the dual cells i0 - 1 and i0 + T + 1 (which the damping of
// lanes 0 and 2 reads, undamped).  g is wrapped on periodic meshes; elsewhere a
// primal g of -1 or np is a ghost and a dual g of nd or more no cell.  damps:
// the thread damps its cell; owned: it also updates it (the dual cell i0 + T
// only as the instance's dual cell np carried by its last tile in a launch
// with xwl).
struct TCell {
    int mesh, col, g;
    bool has, damps, owned;
};
template <int T>
__device__ inline TCell tile_cell(const Inst1D &I, int tile, int i0, bool xwl) {
    const int tid = threadIdx.x;
    TCell c;
    int g;
    if (tid < 2 * T) {
        c.mesh = tid < T ? 0 : 1;
        const int s = tid - c.mesh * T;
        g = i0 + s;
        c.col = s + 1;
        c.has = c.damps = true;
        c.owned = g < (c.mesh == 0 ? I.np : I.nd);
    } else {
        const int lane = tid - 2 * T;
        c.mesh = (lane == 1 || lane == 3 || lane == 4) ? 1 : 0;
        g = (lane == 0 || lane == 3) ? i0 - 1 : (lane == 4 ? i0 + T + 1 : i0 + T);
        c.col = (lane == 0 || lane == 3) ? 0 : (lane == 4 ? T + 2 : T + 1);
        c.has = lane < 5;
        c.damps = lane < 3;
        c.owned = xwl && lane == 1 && I.tail && tile == I.tile0 + I.ntiles - 1 && g < I.nd;
    }
    if (I.bc == 0) {                         // periodic (meshes shorter than a tile too)
        const int n = c.mesh == 0 ? I.np : I.nd;
        g = g < 0 ? g + n : (g >= n ? g - n : g);
        if (g < 0 || g >= n) g = ((g % n) + n) % n;
    }
    c.g = g;
    return c;
}

// Indices of the two cells of the other mesh that overlap cell g of `mesh`
// (left, right): primal g -> dual g, g + 1; dual g -> primal g - 1, g
// (periodic meshes wrapped; a primal -1 or np is a ghost for cell_pre).
__device__ inline void overlap_cells(const Inst1D &I, int mesh, int g, int &l, int &r) {
    if (mesh == 0) {
        l = g;
        r = g + 1;
        if (I.bc == 0 && r >= I.nd) r -= I.nd;
    } else {
        l = g - 1;
        r = g;
        if (I.bc == 0 && l < 0) l += I.np;
    }
}

template <int K, int NC, int W>
__device__ inline void lds_cell(const double *s, int col, double (&c)[NC][K + 1]) {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m <= K; ++m) c[q][m] = s[(q * (K + 1) + m) * W + col];
}

template <int K, int NC, int W>
__device__ inline void lds_put(double *s, int col, const double (&c)[NC][K + 1]) {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m <= K; ++m) s[(q * (K + 1) + m) * W + col] = c[q][m];
}

// This thread's cell, damped: its undamped coefficients and those of the two
// cells of the other mesh that overlap it are loaded (issued together), and
// after the caller has the statistics, damp_cell applies F_tau.  A primal ghost
// of a reflective wall is the mirror image of the damped end cell, so its
// thread damps the end cell and mirrors it; the other ghosts need no damping
// (their only nonzero mode is the mean).
template <int K, int FLUX>
struct CellIn {
    static constexpr int NC = FluxT<FLUX>::NC;
    double own[NC][K + 1], nl[NC][K + 1], nr[NC][K + 1];
    bool real;                               // a cell of the mesh (not a ghost, not beyond nd)
    bool mirror;                             // a reflective-wall ghost: damp the end cell, then mirror it
};

template <int K, int FLUX>
__device__ inline void load_cell_in(const Inst1D &I, const TCell &c, const double *__restrict__ inC,
                                    const double *__restrict__ inD, CellIn<K, FLUX> &ci) {
    const int n = c.mesh == 0 ? I.np : I.nd;
    ci.real = c.has && c.g >= 0 && c.g < n;
    ci.mirror = false;
    if constexpr (FLUX == 3) ci.mirror = c.has && c.mesh == 0 && !ci.real && I.bc == 2;
    // the cell whose values (and neighbours) are loaded: itself, or the end
    // cell next to a wall ghost
    const int sg = ci.mirror ? (c.g < 0 ? 0 : I.np - 1) : c.g;
    cell_pre<K, FLUX>(I, c.mesh, sg, inC, inD, ci.own);
    int l, r;
    overlap_cells(I, c.mesh, ci.real || ci.mirror ? sg : 0, l, r);
    cell_pre<K, FLUX>(I, 1 - c.mesh, l, inC, inD, ci.nl);
    cell_pre<K, FLUX>(I, 1 - c.mesh, r, inC, inD, ci.nr);
}

// The stage kernel's variant: only the thread's own cell from memory (a wall
// ghost's thread: the end cell); the overlapping cells come from the tile's
// undamped image in LDS (lds_overlaps).
template <int K, int FLUX>
__device__ inline void load_own(const Inst1D &I, const TCell &c, const double *__restrict__ inC,
                                const double *__restrict__ inD, CellIn<K, FLUX> &ci) {
    const int n = c.mesh == 0 ? I.np : I.nd;
    ci.real = c.has && c.g >= 0 && c.g < n;
    ci.mirror = false;
    if constexpr (FLUX == 3)
        ci.mirror = c.damps && c.mesh == 0 && I.bc == 2 && (c.g == -1 || c.g == I.np);
    cell_pre<K, FLUX>(I, c.mesh, ci.mirror ? (c.g < 0 ? 0 : I.np - 1) : c.g, inC, inD, ci.own);
}

// The overlapping cells of the cell that the thread damps, from the undamped
// image (uo: the other mesh's image, columns g - i0 + 1): a primal cell in
// column x has dual x, x + 1; a dual cell in column x has primal x - 1, x; a
// wall ghost's end cell sits next to the ghost's column.
template <int K, int FLUX, int W>
__device__ inline void lds_overlaps(const TCell &c, const double *uo, CellIn<K, FLUX> &ci) {
    constexpr int NC = FluxT<FLUX>::NC;
    int x = c.col;
    if (c.mesh == 0 && ci.mirror) x = c.g < 0 ? x + 1 : x - 1;
    const int l = c.mesh == 0 ? x : x - 1;
    lds_cell<K, NC, W>(uo, l, ci.nl);
    lds_cell<K, NC, W>(uo, l + 1, ci.nr);
}

template <int K, int FLUX>
__device__ inline void damp_cell(const Inst1D &I, const TCell &c, CellIn<K, FLUX> &ci, const double (*sig)[3],
                                 double tau, bool damp) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1;
    if (damp && c.damps && (ci.real || ci.mirror)) {
        double ubar[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) ubar[q] = ci.own[q][0];
        const double beta = F::speed(ubar, I.p0);
        double fac[K1];
        oe_factors<K, NC>(ci.own, ci.nl, ci.nr, beta, sig[c.mesh], 1.0 / I.h, tau, fac);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 1; m <= K; ++m) ci.own[q][m] *= fac[m];
    }
    if (ci.mirror) {
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m <= K; ++m) ci.own[q][m] *= mirror_sign(q, m);
    }
}

// Partial statistics of one cell's output (valid: an owned cell; otherwise the
// identities): the cell average, max and min over the sigma sample points
// (both halves: the right-half nodes and xi = 1, and their mirror images
// through the sign flip of odd modes), and the wave speed at the average (beta:
// only a step's last stage, whose output gives the next step's tau).
template <int K, int FLUX>
__device__ inline void cell_stats(const Inst1D &I, bool valid, const double (&out)[FluxT<FLUX>::NC][K + 1],
                                  double (&v)[3 * FluxT<FLUX>::NC + 1], bool beta = true) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC;
    constexpr Tab<K> tb = make_tab<K>();
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        double mx = -INFINITY, mn = INFINITY;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const double flip = hf ? 1.0 : -1.0;
#pragma unroll
            for (int sidx = K + 2; sidx < 2 * K + 4; ++sidx) {
                double x = 0.0;
#pragma unroll
                for (int n = 0; n <= K; ++n) x += ((n & 1) ? flip * out[q][n] : out[q][n]) * tb.SP[sidx][n];
                mx = fmax(mx, x);
                mn = fmin(mn, x);
            }
        }
        v[3 * q] = valid ? out[q][0] : 0.0;
        v[3 * q + 1] = valid ? mx : -INFINITY;
        v[3 * q + 2] = valid ? mn : INFINITY;
    }
    double ubar[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) ubar[q] = out[q][0];
    v[3 * NC] = valid && beta ? F::speed(ubar, I.p0) : -INFINITY;
}

// Kind of value j of cell_stats: sum, max, min per component, then max.
template <int NC>
__device__ constexpr int cell_stat_kind(int j) { return j == 3 * NC ? 1 : j % 3; }

// Reduction over the 32 lanes of each half of a wave (the first five levels
// of wave_reduce); the results are in lanes 31 and 63.
__device__ inline double half_wave_reduce(int kind, double v) {
    const double id = stat_identity(kind);
    v = stat_op(kind, v, dpp_all<0xB1>(v));
    v = stat_op(kind, v, dpp_all<0x4E>(v));
    v = stat_op(kind, v, dpp_all<0x141>(v));
    v = stat_op(kind, v, dpp_all<0x140>(v));
    v = stat_op(kind, v, dpp_d<0x142, 0xa>(v, id));
    return v;
}

// The tile's partial statistics (cell_stats of its owned cells) reduced per
// mesh in a fixed order and written to the record of `tile` in part: the T
// cells of a mesh are half a wave (T = 32), a wave (T = 64) or two waves
// (T = 128, combined in order through LDS).  The instance's dual cell np, when
// the last tile carries it (lane 1 of the last wave, xcell), gets the next
// column, as a tile of its own would have written it.
template <int K, int FLUX, int T>
__device__ inline void tile_partials(const Inst1D &I, const TCell &c, const double (&out)[FluxT<FLUX>::NC][K + 1],
                                     double *part, int tile, double *scratch, bool xcell,
                                     bool write = true, bool beta = true) {
    constexpr int NC = FluxT<FLUX>::NC, NV = 3 * NC + 1;
    const int tid = threadIdx.x, lane = tid % WAVE;
    double v[NV];
    cell_stats<K, FLUX>(I, c.owned, out, v, beta);
    auto put = [&](int mesh, int j, double x) {
        const int row = j == 3 * NC ? ST_BETA + mesh : stat_index(mesh, j / 3, j % 3);
        if (write) part[(long long)tile * NSTAT + row] = x;
    };
    if constexpr (T == 32) {
        if (tid < WAVE) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double x = half_wave_reduce(cell_stat_kind<NC>(j), v[j]);
                if (lane == 31) put(0, j, x);
                if (lane == 63) put(1, j, x);
            }
        }
    } else if constexpr (T == 64) {
        if (tid < 2 * WAVE) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double x = wave_reduce(cell_stat_kind<NC>(j), v[j]);
                if (lane == WAVE - 1) put(tid / WAVE, j, x);
            }
        }
    } else {
        const int wave = tid / WAVE;
        if (tid < 2 * T) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double x = wave_reduce(cell_stat_kind<NC>(j), v[j]);
                if (lane == WAVE - 1) scratch[wave * NV + j] = x;
            }
        }
        __syncthreads();
        if (tid < 2 * NV) {                  // one thread per (mesh, value): waves 2 mesh, 2 mesh + 1
            const int mesh = tid / NV, j = tid % NV;
            const double x = stat_op(cell_stat_kind<NC>(j), scratch[(2 * mesh) * NV + j],
                                     scratch[(2 * mesh + 1) * NV + j]);
            put(mesh, j, x);
        }
    }
    if (write && xcell && tid == 2 * T + 1) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int row1 = j == 3 * NC ? ST_BETA + 1 : stat_index(1, j / 3, j % 3);
            const int row0 = j == 3 * NC ? ST_BETA : stat_index(0, j / 3, j % 3);
            part[(long long)(tile + 1) * NSTAT + row1] = v[j];
            part[(long long)(tile + 1) * NSTAT + row0] = j == 3 * NC ? -INFINITY : stat_identity(j % 3);
        }
    }
}

// Reduced statistics -> avg and sigma per mesh and component.
template <int NC>
__device__ inline void finish_stats(const Inst1D &I, const double *red, double (*sig)[3]) {
#pragma unroll
    for (int mesh = 0; mesh < 2; ++mesh) {
        const double ncell = mesh == 0 ? (double)I.np : (double)I.nd;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double avg = red[stat_index(mesh, q, 0)] / ncell;
            sig[mesh][q] = fmax(red[stat_index(mesh, q, 1)] - avg, avg - red[stat_index(mesh, q, 2)]);
        }
    }
}

// LDS of a tile: the damped and the undamped image of both meshes, columns
// 0 .. T + 2 (cells i0 - 1 .. i0 + T + 1).
constexpr int lds_width(int T) { return T + 3; }
constexpr int lds_doubles(int K, int NC, int T) { return 4 * NC * (K + 1) * lds_width(T); }
constexpr int scratch_doubles(int T) { return NSTAT * ((nthreads(T) + WAVE - 1) / WAVE) + NSTAT; }

// ---------------------------------------------------------- stage tile ---

// folded: the instance's statistics were reduced by k_fold into a.red (batched
// launches); otherwise every workgroup reduces the per-tile records itself.
// COH: the persistent launch, whose step records other workgroups of the same
// launch write (read with device-scope atomic loads after the grid barrier).
template <int K, int FLUX, int T, bool COH = false>
__device__ void stage_tile(const StageArgs &a, int l, int par, int first, int tile, double *smem, bool xwl,
                           bool folded) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, W = lds_width(T), PER = NC * K1 * W, NT = nthreads(T);
    const int tid = threadIdx.x;
    constexpr bool coh = COH;
    Tile1D tl;
    Inst1D I;
    if (a.ninst == 1) {                      // single instance: everything from the kernel arguments
        tl.inst = 0;
        tl.i0 = tile * T;
        I = a.inst0;
        // keeps the two branches apart: merged, they become one load through a
        // selected pointer (vector loads, waited for before anything else)
        asm volatile("" ::: "memory");
    } else {
        tl = a.tiles[tile];
        I = a.inst[tl.inst];
    }
    const int i0 = tl.i0;
    const bool lead = (tile == I.tile0) && tid == 0;
    Slot *S = a.slots + 2 * tl.inst;
    const bool single = a.tau_override > 0.0;
    const int sp = ((a.ns & 1 ? par : 0) + l) & 1;   // parity of the global stage index ns n + l
    // LDS images, [damped C, damped D, undamped C, undamped D] x PER (offsets,
    // not selected pointers: the compiler mishandles a select of LDS pointers)
    double *scratch = smem + lds_doubles(K, NC, T) + NSTAT;

    const TCell c = tile_cell<T>(I, tile, i0, xwl);
    const bool xcell = xwl && I.tail && tile == I.tile0 + I.ntiles - 1;
    const int ncell = c.mesh == 0 ? I.np : I.nd;
    const int gi = c.owned ? c.g : 0;        // a valid index for the owned-cell loads and stores
    double *UM = (c.mesh == 0 ? a.UC + I.offC : a.UD + I.offD);
    const bool damp = a.damp_input && I.oe && K > 0 && !(l == 0 && first);
    const bool need_beta = l == 0 && !single && a.dt_fixed <= 0.0;
    const bool need_red = damp || need_beta;
    const int ns = need_beta ? Partials<NC>::NS : Partials<NC>::NS - 2;
    const RKStage rs = COH ? rk_stage(a.rk, l) : a.rs;   // (l = a.l outside the persistent launch)
    double *AM = (rs.acc_read || rs.ca != 0.0) ? (c.mesh == 0 ? a.AC + I.offC : a.AD + I.offD) : nullptr;

    // One round trip for every load that does not depend on another (issued
    // before any test on them, the selects after): this step's and the
    // previous step's scalars, the thread's cell and its overlapping cells, u^n
    // and the RK4 sum of the cell, the previous stage's partial statistics.
    const Slot cur = ld_slot(&S[par], coh), prev = ld_slot(&S[par ^ 1], coh);
    CellIn<K, FLUX> ci;
    load_own<K, FLUX>(I, c, a.BC[sp] + I.offC, a.BD[sp] + I.offD, ci);
    double un[NC][K1], acc[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) {
            un[q][m] = UM[(long long)(q * K1 + m) * ncell + gi];   // gi: a valid index
            acc[q][m] = 0.0;
        }
    if (rs.acc_read) {
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) acc[q][m] = AM[(long long)(q * K1 + m) * ncell + gi];
    }
    Partials<NC> pv;
    double redv = 0.0;                       // folded: row tid of the instance's reduced statistics
    if (need_red) {
        if (folded) {
            if (tid < NSTAT) redv = a.red[(long long)tl.inst * NSTAT + tid];
        } else {
            load_partials_raw<NT, NC>(a.part[sp ^ 1], I.tile0, I.npart, pv);
        }
    }

    // A step that is not taken (t_end reached) carries the time over; its
    // stages compute but store nothing.  (No early return: a return here would
    // let the compiler sink the loads above below it, one round trip later.)
    const bool skip = !single && ((l == 0 && cur.t >= a.t_end) || (l > 0 && cur.done));
    if (!single && l == 0 && skip && lead) {
        S[par].done = 1;
        S[par ^ 1].t = cur.t;
    }
    // the undamped image (a wall ghost: the mirror image of its end cell), for
    // the overlapping cells of every damped cell; the barrier of the
    // reduction below covers it
    if (c.has) {
        double g[NC][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) g[q][m] = ci.mirror ? mirror_sign(q, m) * ci.own[q][m] : ci.own[q][m];
        lds_put<K, NC, W>(smem + (2 + c.mesh) * PER, c.col, g);
    }
    double red[NSTAT];                       // the reduced statistics, in every thread
    if (need_red) {
        if (folded) {
            if (tid < NSTAT) scratch[tid] = redv;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NSTAT; ++i) red[i] = scratch[i];
        } else {
            finish_partials_all<NT, NC>(pv, a.part[sp ^ 1], I.tile0, I.npart, ns, red, scratch);
        }
    } else {
        __syncthreads();
    }

    double tau, taumax;
    int last = 0;
    if (single) {
        tau = a.tau_override;
        taumax = a.taumax_override;
    } else if (l == 0) {
        taumax = a.dt_fixed > 0.0 ? a.dt_fixed : I.cfl * I.h / fmax(red[ST_BETA], red[ST_BETA + 1]);
        tau = taumax;
        if (cur.t + tau >= a.t_end) {
            tau = a.t_end - cur.t;
            last = 1;
        }
        if (lead && !skip) {
            S[par].tau = tau;
            S[par].tau_max = taumax;
            S[par].done = 0;
            S[par].last = last;
        }
    } else {
        tau = cur.tau;
        taumax = cur.tau_max;
        last = cur.last;
    }
    if (!single && l == a.ns - 1 && lead && !skip) {   // the step's last stage: time and step count
        const double tnext = last ? a.t_end : cur.t + tau;
        S[par ^ 1].t = tnext;
        Final *f = a.fin + tl.inst;
        f->t = tnext;
        f->tau = tau;
        f->nexec = ld_ll(&f->nexec, coh) + 1;
    }

    double sig[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (damp) {
        finish_stats<NC>(I, red, sig);
        if (c.damps && (ci.real || ci.mirror)) lds_overlaps<K, FLUX, W>(c, smem + (3 - c.mesh) * PER, ci);
    }
    damp_cell<K, FLUX>(I, c, ci, sig, (l == 0) ? prev.tau : tau, damp);
    if (c.damps) lds_put<K, NC, W>(smem + c.mesh * PER, c.col, ci.own);
    __syncthreads();

    double out[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) out[q][m] = 0.0;
    if (c.owned && !skip) {
        const double(&own)[NC][K1] = ci.own;
        if (l == 0 && !single) {
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m) UM[(long long)(q * K1 + m) * ncell + gi] = own[q][m];
        }
        if (l > 0 && a.DC) {                 // damped stage input, kept for the adjoint
            double *DM = c.mesh == 0 ? a.DC + I.offC : a.DD + I.offD;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m) DM[(long long)(q * K1 + m) * ncell + gi] = own[q][m];
        }
        // the damped cells of the other mesh that overlap this one (left, right)
        double nb[NC][K1], rl[NC][K1], rr[NC][K1];
        const double ft = taumax * (1.0 / I.h);
        lds_cell<K, NC, W>(smem + (1 - c.mesh) * PER, c.mesh == 0 ? c.col : c.col - 1, nb);
        cdg_rate_half<K, FLUX>(nb, 0, I.p0, ft, rl);
        lds_cell<K, NC, W>(smem + (1 - c.mesh) * PER, c.mesh == 0 ? c.col + 1 : c.col, nb);
        cdg_rate_half<K, FLUX>(nb, 1, I.p0, ft, rr);

        // eq:RKCDG: out = c_{l0} u^n [+ accumulated earlier stages] + c_{ll} u^l + tau d_{ll} L(u^l)
        const double inv_tm = 1.0 / taumax;
        const double td = tau * rs.d;
        bool finite = true;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                const double both = rl[q][m] + rr[q][m];      // the two halves of the cell
                const double rate = inv_tm * (both - own[q][m]);
                const double v = fma(td, rate, rs.cw * own[q][m]);
                double o = v;
                if (l > 0) {                 // (u^n at stage 0 is the input itself)
                    double base = rs.cn * un[q][m];
                    if (rs.acc_read) base += acc[q][m];
                    o = base + v;
                }
                out[q][m] = o;
                finite = finite && isfinite(o);
            }
        if (rs.ca != 0.0) {                  // classical RK4: this stage's damped input joins the sum
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m) {
                    double *p = AM + (long long)(q * K1 + m) * ncell + gi;
                    *p = rs.acc_first ? rs.ca * own[q][m] : fma(rs.ca, own[q][m], *p);
                }
        }
        double *OM = (c.mesh == 0 ? a.BC[sp ^ 1] + I.offC : a.BD[sp ^ 1] + I.offD);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) OM[(long long)(q * K1 + m) * ncell + gi] = out[q][m];
        double ubar[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) ubar[q] = out[q][0];
        // a tolerated non-positive pressure (OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE) leaves the density
        const bool phys = (I.flags & OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE) ? ubar[0] > 0.0 : F::physical(ubar, I.p0);
        if (!finite || !phys) {
            if (!finite) a.err[0] = 1;
            if (!phys) a.err[1] = 1;
            a.err[3] = (int)(a.fin[tl.inst].nexec + 1);
        }
    }
    // the wave speeds only where a step's tau reads them: after its last stage
    // (a single-stage call writes them always)
    tile_partials<K, FLUX, T>(I, c, out, a.part[sp], tile, scratch, xcell, !skip, single || l == a.ns - 1);
    if (tile + (int)gridDim.x < a.tend) __syncthreads();   // (persistent launch) the next tile reuses the LDS
}

// Statistics of a given state (srcC/srcD) into part[1]: the partials that the
// first stage of a run reads (beta for tau^0).
template <int K, int FLUX, int T>
__device__ void stats_tile(const StageArgs &a, int tile, double *smem, bool xwl) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1;
    const Tile1D tl = a.ninst == 1 ? Tile1D{0, tile * T} : a.tiles[tile];
    const Inst1D I = a.ninst == 1 ? a.inst0 : a.inst[tl.inst];
    const TCell c = tile_cell<T>(I, tile, tl.i0, xwl);
    const int ncell = c.mesh == 0 ? I.np : I.nd;
    const double *src = c.mesh == 0 ? a.srcC + I.offC : a.srcD + I.offD;
    double u[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) u[q][m] = c.owned ? src[(long long)(q * K1 + m) * ncell + c.g] : 1.0;
    tile_partials<K, FLUX, T>(I, c, u, a.part[1], tile, smem + NSTAT,
                              xwl && I.tail && tile == I.tile0 + I.ntiles - 1);
    __syncthreads();
}

// Final OE: u_sigma^N = F_tau(output of the last stage of step N-1) into (dstC, dstD); copy if no step ran.
template <int K, int FLUX, int T>
__device__ void final_tile(const StageArgs &a, int tile, double *smem, bool xwl) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1;
    const Tile1D tl = a.ninst == 1 ? Tile1D{0, tile * T} : a.tiles[tile];
    const Inst1D I = a.ninst == 1 ? a.inst0 : a.inst[tl.inst];
    const long long N = a.fin[tl.inst].nexec;
    const double tau = a.fin[tl.inst].tau;
    const int bp = (int)((a.ns * N) & 1);   // buffer holding the last stage's output (or the input when N = 0)
    double *red = smem + lds_doubles(K, NC, T);
    double *scratch = red + NSTAT;
    const bool damp = N > 0 && I.oe && K > 0;
    const TCell c = tile_cell<T>(I, tile, tl.i0, xwl);
    CellIn<K, FLUX> ci;
    load_cell_in<K, FLUX>(I, c, a.BC[bp] + I.offC, a.BD[bp] + I.offD, ci);
    double sig[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (damp) {
        reduce_instance<nthreads(T), NC>(a.part[(int)((a.ns * N - 1) & 1)], I.tile0, I.npart, false, red,
                                         scratch);
        finish_stats<NC>(I, red, sig);
    }
    damp_cell<K, FLUX>(I, c, ci, sig, tau, damp);
    if (c.owned) {
        const int ncell = c.mesh == 0 ? I.np : I.nd;
        double *dst = c.mesh == 0 ? a.dstC + I.offC : a.dstD + I.offD;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) dst[(long long)(q * K1 + m) * ncell + c.g] = ci.own[q][m];
    }
    __syncthreads();
}

// --------------------------------------------------------------- kernels ---

// Kernels of one degree KM, flux and tile.
template <int KM, int FLUX, int T>
struct Disp {
    static constexpr int LDS = lds_doubles(KM, FluxT<FLUX>::NC, T) + scratch_doubles(T);
    template <template <int, int, int> class Fn, typename... Args>
    __device__ static void run(Args &&...args) {
        Fn<KM, FLUX, T>::go(args...);
    }
};

template <int K, int FLUX, int T> struct StageFn {
    __device__ static void go(const StageArgs &a, int l, int par, int first, int tile, double *smem, bool xwl,
                              bool folded) {
        stage_tile<K, FLUX, T>(a, l, par, first, tile, smem, xwl, folded);
    }
};
template <int K, int FLUX, int T> struct StageCohFn {
    __device__ static void go(const StageArgs &a, int l, int par, int first, int tile, double *smem, bool xwl,
                              bool folded) {
        stage_tile<K, FLUX, T, true>(a, l, par, first, tile, smem, xwl, folded);
    }
};
template <int K, int FLUX, int T> struct StatsFn {
    __device__ static void go(const StageArgs &a, int tile, double *smem, bool xwl) {
        stats_tile<K, FLUX, T>(a, tile, smem, xwl);
    }
};
template <int K, int FLUX, int T> struct FinalFn {
    __device__ static void go(const StageArgs &a, int tile, double *smem, bool xwl) {
        final_tile<K, FLUX, T>(a, tile, smem, xwl);
    }
};

// One tile per workgroup (launched with one workgroup per tile): no loop
// keeps the stage's uniform values alive across tiles, which had spilled them
// from scalar registers into vector lanes.
template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(nthreads(T)) void k_stage(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    const int tile = a.tbeg + xcd_tile(blockIdx.x, a.tend - a.tbeg);
    if (tile < a.tend) D::template run<StageFn>(a, a.l, a.par, a.first, tile, smem, XW, false);
}

// The stage kernel of batched launches (one degree per launch): the
// instance's statistics come reduced from k_fold (one fixed-order reduction
// per instance and stage) instead of every workgroup reducing all of its
// instance's per-tile records.  One tile per workgroup, as in k_stage: a
// loop over tiles kept the stage's uniform values alive across iterations
// and spilled them from scalar registers into vector lanes.
template <int K, int FLUX, int T>
__global__ __launch_bounds__(nthreads(T), T == 64 && K <= 2 ? 3 : 1) void k_stage_folded(StageArgs a) {
    __shared__ double smem[lds_doubles(K, FluxT<FLUX>::NC, T) + scratch_doubles(T)];
    const int tile = a.tbeg + xcd_tile(blockIdx.x, a.tend - a.tbeg);     // one tile per workgroup
    if (tile < a.tend) stage_tile<K, FLUX, T>(a, a.l, a.par, a.first, tile, smem, false, true);
}

// One workgroup per instance: the partial columns of the state the next stage
// reads (part[src]) reduced in the same fixed order as a stage kernel's own
// reduction (same thread count, same tree), so batched instances keep the bits
// of single-instance runs.  All NSTAT rows go to red[instance][row].
template <int NC, int T>
__global__ __launch_bounds__(nthreads(T)) void k_fold(StageArgs a, int src) {
    __shared__ double red[NSTAT];
    __shared__ double scratch[scratch_doubles(T)];
    const int b = blockIdx.x, tid = threadIdx.x;
    if (tid < NSTAT) red[tid] = 0.0;
    __syncthreads();
    const Inst1D I = a.ninst == 1 ? a.inst0 : a.inst[b];
    reduce_instance<nthreads(T), NC>(a.part[src], I.tile0, I.npart, true, red, scratch);
    if (tid < NSTAT) a.red[(long long)b * NSTAT + tid] = red[tid];
}

// Step records (both parities), final record of instance i, and with i = 0
// the error flags and the grid-barrier counters, cleared: the start of a run.
__device__ inline void clear_records(const StageArgs &a, int i, int ninst) {
    if (i < ninst) {
        a.slots[2 * i].t = 0.0;
        a.slots[2 * i].tau = 0.0;
        a.slots[2 * i].tau_max = 0.0;
        a.slots[2 * i].done = 0;
        a.slots[2 * i].last = 0;
        a.slots[2 * i + 1] = a.slots[2 * i];
        a.fin[i].t = 0.0;
        a.fin[i].tau = 0.0;
        a.fin[i].nexec = 0;
    }
    if (i == 0) {
        a.err[0] = a.err[1] = a.err[2] = a.err[3] = 0;
        a.bar[0] = 0;
        a.bar[1] = 0;
    }
}

template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(nthreads(T)) void k_stats(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    if (a.init_records && blockIdx.x == 0)   // a run's start: no kernel of its own for the records
        for (int i = threadIdx.x; i < a.ninst; i += blockDim.x) clear_records(a, i, a.ninst);
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        D::template run<StatsFn>(a, tile, smem, XW);
    }
}

template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(nthreads(T)) void k_final(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    if (a.fin_host && blockIdx.x == 0) {     // the run's records (complete: the stages wrote them) to the host
        for (int i = threadIdx.x; i < a.ninst; i += blockDim.x) a.fin_host[i] = a.fin[i];
        if (threadIdx.x < 4) a.err_host[threadIdx.x] = a.err[threadIdx.x];
    }
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        D::template run<FinalFn>(a, tile, smem, XW);
    }
}

// Grid-wide barrier for the persistent launch (all workgroups co-resident by
// cooperative launch).  Sense by generation counter; bounded spin so that every
// workgroup always terminates (a timeout is reported through err[2]).
__device__ inline void grid_barrier(const StageArgs &a) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *count = a.bar, *gen = a.bar + 1;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > a.spin_limit) {
                    a.err[2] = 1;
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// Persistent launch: every workgroup walks all steps and stages; a grid
// barrier separates consecutive stages.  The statistics a workgroup reads after
// a barrier are read coherently (stage_tile with COH).
template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(nthreads(T)) void k_persistent(StageArgs a, long long nsteps, int single_instance) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    for (long long n = 0; n < nsteps; ++n) {
        const int par = (int)(n & 1);
        for (int l = 0; l < a.ns; ++l) {
            for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
                D::template run<StageCohFn>(a, l, par, n == 0, tile, smem, XW, false);
            }
            grid_barrier(a);
            if (l == 0 && single_instance && ld_i(&a.slots[par].done, true)) return;
            if (ld_i(&a.err[2], true)) return;
        }
    }
}

__global__ void k_init(StageArgs a, int ninst) {
    clear_records(a, blockIdx.x * blockDim.x + threadIdx.x, ninst);
}

// ------------------------------------------------------------ host side ---

static int tile_index(int tile) { return tile == 32 ? 0 : (tile == 64 ? 1 : (tile == 128 ? 2 : -1)); }
// kernel table index: the tile (0, 1, 2 for 32, 64, 128), or 3 / 4 for tiles
// of 32 / 64 whose launches carry the dual cell np in an instance's last tile
static int kernel_index(int tile, bool tailwave) {
    const int ti = tile_index(tile);
    return (ti >= 0 && tailwave && tail_mode(tile)) ? ti + 3 : ti;
}

// Kernel pointers by (kernel, degree, flux, tile).  XW: launches with the extra
// wave (tail tiles) use kernels whose launch bounds allow it; the others keep
// the bounds of four waves per tile of T.  WHICH 4: the folded stage kernel.
template <int WHICH, int KM, int FLUX, int T, bool XW>
static void *kptr() {
    if constexpr (WHICH == 0) return (void *)k_stage<KM, FLUX, T, XW>;
    else if constexpr (WHICH == 1) return (void *)k_stats<KM, FLUX, T, XW>;
    else if constexpr (WHICH == 2) return (void *)k_final<KM, FLUX, T, XW>;
    else if constexpr (WHICH == 3) return (void *)k_persistent<KM, FLUX, T, XW>;
    else return (void *)k_stage_folded<KM, FLUX, T>;
}

template <int WHICH, int KM, int FLUX>
static void *pick_t(int ti) {
    if constexpr (WHICH == 4) {              // no extra-wave variants
        switch (ti) {
        case 0: return kptr<WHICH, KM, FLUX, 32, false>();
        case 1: return kptr<WHICH, KM, FLUX, 64, false>();
        default: return kptr<WHICH, KM, FLUX, 128, false>();
        }
    } else {
        switch (ti) {
        case 0: return kptr<WHICH, KM, FLUX, 32, false>();
        case 1: return kptr<WHICH, KM, FLUX, 64, false>();
        case 3: return kptr<WHICH, KM, FLUX, 32, true>();
        case 4: return kptr<WHICH, KM, FLUX, 64, true>();
        default: return kptr<WHICH, KM, FLUX, 128, false>();
        }
    }
}

template <int WHICH, int KM>
static void *pick_f(int flux, int ti) {
    switch (flux) {
    case 0: return pick_t<WHICH, KM, 0>(ti);
    case 1: return pick_t<WHICH, KM, 1>(ti);
    case 2: return pick_t<WHICH, KM, 2>(ti);
    default: return pick_t<WHICH, KM, 3>(ti);   // Euler with reflective walls
    }
}

template <int WHICH>
static void *pick(int k, int flux, int ti) {   // batches of mixed degree launch one kernel per degree group
    switch (k) {
    case 0: return pick_f<WHICH, 0>(flux, ti);
    case 1: return pick_f<WHICH, 1>(flux, ti);
    case 2: return pick_f<WHICH, 2>(flux, ti);
    default: return pick_f<WHICH, 3>(flux, ti);
    }
}

static hipError_t launch(void *fn, int grid, int tile, const StageArgs &a, hipStream_t s) {
    StageArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(nthreads(tile)), args, 0, s);
}

hipError_t launch_init_1d(const StageArgs &a, int ninst, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3((ninst + 255) / 256), dim3(256), 0, s, a, ninst);
    return hipGetLastError();
}

hipError_t launch_stats_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s) {
    int ti = kernel_index(tile, a.tailwave);
    if (ti < 0) return hipErrorInvalidValue;
    return launch(pick<1>(kmax, flux, ti), a.tend - a.tbeg, tile, a, s);
}

hipError_t launch_stage_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s) {
    int ti = kernel_index(tile, a.tailwave);
    if (ti < 0) return hipErrorInvalidValue;
    StageArgs b = a;
    b.rs = rk_stage(a.rk, a.l);              // the stage's coefficients, ready in the kernel arguments
    if (a.red) {                             // statistics folded by launch_fold_1d
        if (a.tailwave) return hipErrorInvalidValue;
        return launch(pick<4>(kmax, flux, ti), b.tend - b.tbeg, tile, b, s);   // one workgroup per tile
    }
    return launch(pick<0>(kmax, flux, ti), b.tend - b.tbeg, tile, b, s);   // one workgroup per tile
}

hipError_t launch_fold_1d(const StageArgs &a, int flux, int tile, hipStream_t s) {
    // the reduction uses nthreads(tile) threads, as a stage workgroup does
    // (an extra-wave launch's fifth wave takes no part in it either)
    if (!a.red || tile_index(tile) < 0) return hipErrorInvalidValue;
    // the partials the stage (a.l, a.par) reads: those of the previous global stage
    const int src = ((((a.ns & 1) ? a.par : 0) + a.l) & 1) ^ 1;
    void *fn = nullptr;
    const int nc = flux == 0 || flux == 1 ? 1 : 3;
    if (nc == 1) fn = tile == 32 ? (void *)k_fold<1, 32> : (tile == 64 ? (void *)k_fold<1, 64> : (void *)k_fold<1, 128>);
    else fn = tile == 32 ? (void *)k_fold<3, 32> : (tile == 64 ? (void *)k_fold<3, 64> : (void *)k_fold<3, 128>);
    StageArgs copy = a;
    int srcv = src;
    void *args[] = {&copy, &srcv};
    return hipLaunchKernel(fn, dim3(a.ninst), dim3(nthreads(tile)), args, 0, s);
}

hipError_t launch_final_1d(const StageArgs &a, int kmax, int flux, int tile, hipStream_t s) {
    int ti = kernel_index(tile, a.tailwave);
    if (ti < 0) return hipErrorInvalidValue;
    return launch(pick<2>(kmax, flux, ti), a.tend - a.tbeg, tile, a, s);
}

int persistent_max_grid_1d(int kmax, int flux, int tile, bool tailwave) {
    int ti = kernel_index(tile, tailwave);
    if (ti < 0) return 0;
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int nthr = nthreads(tile);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pick<3>(kmax, flux, ti), nthr, 0) !=
        hipSuccess)
        return 0;
    return per_cu * ncu;
}

hipError_t launch_persistent_1d(const StageArgs &a, int kmax, int flux, int tile, int grid,
                                long long nsteps, hipStream_t s) {
    int ti = kernel_index(tile, a.tailwave);
    if (ti < 0) return hipErrorInvalidValue;
    StageArgs copy = a;
    int single = a.ninst == 1;
    void *args[] = {&copy, &nsteps, &single};
    const int nthr = nthreads(tile);
    return hipLaunchCooperativeKernel(pick<3>(kmax, flux, ti), dim3(grid), dim3(nthr), args, 0, s);
}

}  // namespace oecdg
