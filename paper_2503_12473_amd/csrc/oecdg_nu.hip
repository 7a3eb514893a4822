// oecdg_nu.hip -- 1D OECDG on a non-uniform periodic mesh.
//
// Meshes of the 1D setting of Sec. 2.1: primal cells [x_{i-1/2}, x_{i+1/2}] of
// width h_i, dual cells [x_{i-1}, x_i] between neighbouring primal centres, so a
// dual cell holds the primal edge x_{i-1/2} off its centre.  Every cell carries
// its own geometry (centre, width, and the point where the other mesh has its
// edge); the Legendre values at the mapped quadrature nodes are evaluated at run
// time.
//
// One launch per RK stage (k_nu_step), as the uniform stage kernel: a workgroup
// owns CPB = 64 consecutive indices of both meshes, one thread per cell (wave 0
// primal, wave 1 dual; two lanes of wave 2 take the primal cell left of the
// range and the dual cell right of it, which the operator of the owned cells
// reads; 256 workgroups at N = 16384, one per CU).  In order:
//   - the statistics of the stage input (the previous stage's undamped output)
//     from the per-workgroup partials, in the same fixed order in every
//     workgroup: avg = width-weighted domain mean and sigma per mesh and
//     component (Sec. 2.2), and at a step's first stage the wave speed beta,
//     tau_max = C h_max / beta and tau (every workgroup computes the same tau;
//     the first workgroup records the step);
//   - delta_K^m (h_{e,K} = the width of K) and the exact damping F_tau of each
//     thread's cell into LDS (not at the run's first stage: the initial data
//     enter undamped); at the first stage the damped u^n is also stored;
//   - the operator of eq:1D_H on the owned cells from the damped cells in LDS,
//     the c/d combination of eq:RKCDG, the undamped output, and the partials of
//     its statistics (one DPP wave reduction per mesh).
// A step's last output stays undamped until the next step's first stage (or
// k_nu_final at the end of the call) damps it.  Stage inputs and outputs
// alternate between two buffers with the parity of the global stage index; the
// step record alternates with the parity of the step index.  No host
// synchronisation inside a step; the host polls the record every few steps when
// it marches to a final time.
#include "oecdg_device.h"
#include "oecdg_tables.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace oecdg {
namespace {

constexpr int NB = 3 * WAVE;            // threads per workgroup: a wave per mesh, and one for the two end cells
constexpr int CPB = WAVE;               // owned indices per workgroup
constexpr int POLL = 16;                // steps between host checks of the record when marching to t_end

// Run-time Legendre values: d-th derivative of P_m at x, m <= 3.
__device__ inline double legr(int m, int d, double x) {
    if (d == 0) return m == 0 ? 1.0 : m == 1 ? x : m == 2 ? 1.5 * x * x - 0.5 : (2.5 * x * x - 1.5) * x;
    if (d == 1) return m == 0 ? 0.0 : m == 1 ? 1.0 : m == 2 ? 3.0 * x : 7.5 * x * x - 1.5;
    if (d == 2) return m < 2 ? 0.0 : m == 2 ? 3.0 : 15.0 * x;
    return m == 3 ? 15.0 : 0.0;
}

// The start of a step (t, stop) and, once its first stage has run, the step
// itself (tau, tau_max, run).  Two records, by the parity of the step index.
struct NuSlot {
    double t, tau, tau_max;
    int stop, run;
};

struct NuArgs {
    int n, k, flux, oe, ns;
    double L, hmax, cfl, p0, t_end, dt_fixed;
    const double *edges;                 // [n+1]
    const double *cC, *wC;               // primal centres and widths [n]
    const double *cD, *wD;               // dual centres and widths [n] (dual 0 starts below xlo)
    double *TC[2], *TD[2];               // undamped stage states, by the parity of the global stage index
    double *UC, *UD;                     // damped u^n of the current step
    double *dstC, *dstD;                 // k_nu_final: the caller's arrays
    double *part;                        // partial statistics [2 parities][2 meshes][RW rows][nblk]
    NuSlot *slot;                        // [2]
    long long *nexec;                    // steps executed
    int *err;                            // [0] non-finite, [1] non-physical, [2] bad wave speed
    int nblk;
    // per launch
    int l, gp, sp, first;                // stage, parity of the global stage index, parity of the step, step 0
    double cn, cw, dd;                   // c_{l0}, c_{ll}, d_{ll} (l = 0: cn = 0)
};

// Geometry of the cell of the other mesh that overlaps piece p of cell i of mesh
// M, shifted by a period across the seam.
__device__ inline void neighbour(const NuArgs &a, int M, int i, int p, int &j, double &c, double &w) {
    if (M == 0) {                        // primal i: dual i (left), dual i+1 (right)
        j = p == 0 ? i : (i + 1 == a.n ? 0 : i + 1);
        c = a.cD[j] + ((p == 1 && i + 1 == a.n) ? a.L : 0.0);
        w = a.wD[j];
    } else {                             // dual i: primal i-1 (left), primal i (right)
        j = p == 0 ? (i == 0 ? a.n - 1 : i - 1) : i;
        c = a.cC[j] - ((p == 0 && i == 0) ? a.L : 0.0);
        w = a.wC[j];
    }
}

// The cell's ends and the split point where the other mesh has its edge.
__device__ inline void pieces(const NuArgs &a, int M, int i, double &lo, double &split, double &hi) {
    if (M == 0) {
        lo = a.edges[i];
        hi = a.edges[i + 1];
        split = a.cC[i];
    } else {
        lo = i == 0 ? a.cC[a.n - 1] - a.L : a.cC[i - 1];
        hi = a.cC[i];
        split = a.edges[i];
    }
}

template <int K, int NC>
__device__ inline void load_cell(const double *u, int n, int i, double (&c)[NC][K + 1]) {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m <= K; ++m) c[q][m] = u[(long long)(q * (K + 1) + m) * n + i];
}

template <int K, int NC>
__device__ inline void eval(const double (&c)[NC][K + 1], int d, double xi, double scale, double *v) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m <= K; ++m) s += c[q][m] * legr(m, d, xi);
        v[q] = scale * s;
    }
}

template <int NC>
struct Rows {
    static constexpr int RW = 3 * NC + 1;   // per mesh: (sum, max, min) per component, then max beta
};

// Kind of partial row j (both meshes): sum, max, min per component, then max beta.
template <int NC>
__device__ constexpr int nu_row_kind(int j) {
    return j % Rows<NC>::RW == Rows<NC>::RW - 1 ? 1 : (j % Rows<NC>::RW) % 3;
}

// This thread's share of the partials of parity gp: partials t and t + NB of
// every row, loaded together (unconditional loads of valid elements, then
// selects).
template <int NC>
struct NuPart {
    double x[2 * Rows<NC>::RW], y[2 * Rows<NC>::RW];
};
template <int NC>
__device__ inline void nu_stat_load(const NuArgs &a, int gp, NuPart<NC> &pt) {
    constexpr int NR = 2 * Rows<NC>::RW;
    const double *part = a.part + (long long)gp * NR * a.nblk;
    const int b0 = min((int)threadIdx.x, a.nblk - 1), b1 = min((int)threadIdx.x + NB, a.nblk - 1);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        pt.x[j] = part[(long long)j * a.nblk + b0];
        pt.y[j] = part[(long long)j * a.nblk + b1];
    }
}

// Reduce the partials into avg and sigma of both meshes ([mesh][q]) and the
// largest wave speed: this thread's share, a DPP tree per wave, then the waves
// in order; every workgroup gets the same bits.  All threads must take part.
template <int NC>
__device__ inline void nu_statistics(const NuArgs &a, int gp, const NuPart<NC> &pt, double *sh,
                                     double (&avg)[2][NC], double (&sig)[2][NC], double &beta) {
    constexpr int RW = Rows<NC>::RW, NR = 2 * RW, NW = NB / WAVE;
    const int t = threadIdx.x, lane = t % WAVE, wave = t / WAVE;
    const double *part = a.part + (long long)gp * NR * a.nblk;
    double v[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kd = nu_row_kind<NC>(j);
        v[j] = t < a.nblk ? pt.x[j] : stat_identity(kd);
        v[j] = t + NB < a.nblk ? stat_op(kd, v[j], pt.y[j]) : v[j];
    }
    for (int b = t + 2 * NB; b < a.nblk; b += NB) {  // meshes of more than 2 NB CPB cells
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = stat_op(nu_row_kind<NC>(j), v[j], part[(long long)j * a.nblk + b]);
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kd = nu_row_kind<NC>(j);
        v[j] = wave_reduce(kd, v[j]);
        if (lane == WAVE - 1) sh[j * NW + wave] = v[j];
    }
    __syncthreads();
    double r[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kd = nu_row_kind<NC>(j);
        r[j] = sh[j * NW];
        for (int w = 1; w < NW; ++w) r[j] = stat_op(kd, r[j], sh[j * NW + w]);
    }
#pragma unroll
    for (int M = 0; M < 2; ++M)
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            avg[M][q] = r[M * RW + 3 * q] / a.L;
            sig[M][q] = fmax(r[M * RW + 3 * q + 1] - avg[M][q], avg[M][q] - r[M * RW + 3 * q + 2]);
        }
    beta = fmax(r[RW - 1], r[2 * RW - 1]);
}

// Geometry of cell i of mesh M: centre, width, its ends and split point, and
// the overlapping cells of the other mesh (indices, centres shifted across the
// seam, widths), with the reciprocal widths.
struct NuGeo {
    double c, w, iw, lo, split, hi, cn[2], wn[2], iwn[2];
    int j[2];
};
__device__ inline NuGeo nu_geo(const NuArgs &a, int M, int i) {
    NuGeo g;
    g.c = M == 0 ? a.cC[i] : a.cD[i];
    g.w = M == 0 ? a.wC[i] : a.wD[i];
    pieces(a, M, i, g.lo, g.split, g.hi);
#pragma unroll
    for (int p = 0; p < 2; ++p) neighbour(a, M, i, p, g.j[p], g.cn[p], g.wn[p]);
    g.iw = 1.0 / g.w;
#pragma unroll
    for (int p = 0; p < 2; ++p) g.iwn[p] = 1.0 / g.wn[p];
    return g;
}

// delta_K^m of a cell (Sec. 2.2) from its undamped coefficients u and those of
// the two overlapping cells of the other mesh (nb), and the exact damping
// F_tau of u in place.  isig: 1 / sigma per component (0 where sigma = 0,
// whose component then takes no part).
template <int K, int FLUX>
__device__ inline void nu_damp(const NuArgs &a, const NuGeo &g, const double (&nb)[2][FluxT<FLUX>::NC][K + 1],
                               double tau, const double (&isig)[FluxT<FLUX>::NC],
                               double (&u)[FluxT<FLUX>::NC][K + 1]) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC;
    double ub[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) ub[q] = u[q][0];
    const double beta = F::speed(ub, a.p0);
    const double xl = 2.0 * (g.lo - g.c) * g.iw, xr = 2.0 * (g.hi - g.c) * g.iw;
    const double yl = 2.0 * (g.lo - g.cn[0]) * g.iwn[0], yr = 2.0 * (g.hi - g.cn[1]) * g.iwn[1];
    double S = 0.0, wp = g.iw;                        // w^{m-1}
    double so = 1.0, sl = 1.0, sr = 1.0;              // (2/w)^m of the cell and of both neighbours
    double fact = 1.0;
#pragma unroll
    for (int m = 0; m <= K; ++m) {
        if (m > 0) {
            so *= 2.0 * g.iw;
            sl *= 2.0 * g.iwn[0];
            sr *= 2.0 * g.iwn[1];
        }
        if (m > 1) fact *= m;
        double oL[NC], oR[NC], vL[NC], vR[NC];
        eval<K, NC>(u, m, xl, so, oL);
        eval<K, NC>(u, m, xr, so, oR);
        eval<K, NC>(nb[0], m, yl, sl, vL);
        eval<K, NC>(nb[1], m, yr, sr, vR);
        const double cm = (2.0 * m + 1.0) / ((2.0 * K - 1.0) * fact) * wp;
        double dm = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q)
            dm = fmax(dm, cm * beta * (fabs(oL[q] - vL[q]) + fabs(oR[q] - vR[q])) * isig[q]);
        S += dm;
        wp *= g.w;
        if (m >= 1) {
            const double fac = exp(-tau * S);
#pragma unroll
            for (int q = 0; q < NC; ++q) u[q][m] *= fac;
        }
    }
}

// Partial statistics of one cell's undamped coefficients o: width-weighted
// average, max and min at the ends and the quadrature nodes of both pieces, and
// the wave speed at the average; plus the error flags.
template <int K, int FLUX>
__device__ inline void nu_cell_stats(const NuArgs &a, const NuGeo &g, const double (&o)[FluxT<FLUX>::NC][K + 1],
                                     double *st, bool flag) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, Q = K + 1;
    constexpr ct::Gauss<Q> G = ct::gauss<Q>();
#pragma unroll
    for (int q = 0; q < NC; ++q) st[3 * q] = g.w * o[q][0], st[3 * q + 1] = -INFINITY, st[3 * q + 2] = INFINITY;
    double xs[2 * Q + 2];
    xs[0] = g.lo;
    xs[2 * Q + 1] = g.hi;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        xs[1 + k] = 0.5 * (g.lo + g.split) + 0.5 * (g.split - g.lo) * G.s[k];
        xs[1 + Q + k] = 0.5 * (g.split + g.hi) + 0.5 * (g.hi - g.split) * G.s[k];
    }
#pragma unroll
    for (int j = 0; j < 2 * Q + 2; ++j) {
        double v[NC];
        eval<K, NC>(o, 0, 2.0 * (xs[j] - g.c) * g.iw, 1.0, v);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            st[3 * q + 1] = fmax(st[3 * q + 1], v[q]);
            st[3 * q + 2] = fmin(st[3 * q + 2], v[q]);
        }
    }
    double ub[NC];
    bool finite = true;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        ub[q] = o[q][0];
#pragma unroll
        for (int m = 0; m < K1; ++m) finite = finite && isfinite(o[q][m]);
    }
    double b = F::speed(ub, a.p0);
    if (!(b >= 0.0)) b = INFINITY;       // NaN: a bad wave speed at the next step
    st[3 * NC] = b;
    if (flag) {
        if (!finite) __hip_atomic_store(&a.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!F::physical(ub, a.p0)) __hip_atomic_store(&a.err[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The block of CPB cells of this workgroup (a band of consecutive blocks per
// XCD); it also names the workgroup's column of the partial statistics.
__device__ inline int nu_block(const NuArgs &a) { return xcd_tile(blockIdx.x, a.nblk); }

// One wave's reduction of its cells' partial rows (waves 0 and 1 hold one mesh
// each; wave 2 owns no cell) into the workgroup's column of the partials of
// parity gp.
template <int NC>
__device__ inline void nu_store_partials(const NuArgs &a, int gp, int M, double *st) {
    constexpr int RW = Rows<NC>::RW;
    if (threadIdx.x >= 2 * WAVE) return;             // uniform over the wave
    double *part = a.part + (long long)gp * 2 * RW * a.nblk;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int kd = r == RW - 1 ? 1 : r % 3;
        const double v = wave_reduce(kd, st[r]);
        if (threadIdx.x % WAVE == WAVE - 1) part[((long long)M * RW + r) * a.nblk + nu_block(a)] = v;
    }
}

// This thread's cell and its LDS slot, for the owned range [i0, i1): wave 0
// the primal cells i0 + lane (slot lane + 1), wave 1 the dual cells i0 + lane
// (slot lane); wave 2 lane 0 the primal cell i0 - 1 (slot 0), lane 1 the dual
// cell i1 (slot i1 - i0); periodic wrap.  owned: the operator's cells.
struct NuCell {
    int M, s, i;
    bool has, owned;
};
__device__ inline NuCell nu_cell(const NuArgs &a) {
    NuCell c;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int i0 = nu_block(a) * CPB, span = min(a.n, i0 + CPB) - i0;
    int i;
    if (wave < 2) {
        c.M = wave;
        c.has = c.owned = lane < span;
        c.s = wave == 0 ? lane + 1 : lane;
        i = i0 + lane;
    } else {
        c.M = lane == 1 ? 1 : 0;
        c.has = lane < 2;
        c.owned = false;
        c.s = lane == 0 ? 0 : span;
        i = lane == 0 ? i0 - 1 : i0 + span;
    }
    i = i < 0 ? i + a.n : (i >= a.n ? i - a.n : i);
    c.i = c.has ? i : i0;                // threads without a cell read a valid one and store nothing
    return c;
}

// Statistics of the initial data (stage input of step 0).
template <int K, int FLUX>
__global__ void __launch_bounds__(NB) k_nu_init(NuArgs a) {
    constexpr int NC = FluxT<FLUX>::NC, K1 = K + 1, RW = Rows<NC>::RW;
    const NuCell c = nu_cell(a);
    const NuGeo g = nu_geo(a, c.M, c.i);
    double u[NC][K1];
    load_cell<K, NC>(c.M == 0 ? a.TC[0] : a.TD[0], a.n, c.i, u);
    double st[RW];
    nu_cell_stats<K, FLUX>(a, g, u, st, false);
    if (!c.owned) {
#pragma unroll
        for (int r = 0; r < RW; ++r) st[r] = stat_identity(r == RW - 1 ? 1 : r % 3);
    }
    nu_store_partials<NC>(a, 0, c.M, st);
}

// One RK stage (see the top of the file).
template <int K, int FLUX>
__global__ void __launch_bounds__(NB) k_nu_step(NuArgs a) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, Q = K + 1, RW = Rows<NC>::RW;
    constexpr ct::Gauss<Q> G = ct::gauss<Q>();
    __shared__ double dmp[2][NC * K1][WAVE + 1];     // damped input of the workgroup's cells, [mesh][coefficient][slot]
    __shared__ double sh[2 * RW * (NB / WAVE)];
    // every independent load before the first test on any of them: the step
    // record, the error flags, the partial statistics of the input, geometry,
    // the cell, the two overlapping cells of the other mesh, u^n (later stages)
    const NuSlot cur = a.slot[a.sp];
    const double tau_prev = a.slot[a.sp ^ 1].tau;    // the previous step's (damps the input of its first stage)
    const int errs = a.err[0] | a.err[1] | a.err[2];
    NuPart<NC> pt;
    nu_stat_load<NC>(a, a.gp, pt);
    const NuCell c = nu_cell(a);
    const int M = c.M, i = c.i;
    const double *own = M == 0 ? a.TC[a.gp] : a.TD[a.gp], *oth = M == 0 ? a.TD[a.gp] : a.TC[a.gp];
    const NuGeo g = nu_geo(a, M, i);
    double u[NC][K1], nb[2][NC][K1], un[NC][K1];
    load_cell<K, NC>(own, a.n, i, u);
#pragma unroll
    for (int p = 0; p < 2; ++p) load_cell<K, NC>(oth, a.n, g.j[p], nb[p]);
    if (a.l > 0) load_cell<K, NC>(M == 0 ? a.UC : a.UD, a.n, i, un);
    if (a.l > 0 && !cur.run) return;                 // uniform over the grid
    if (a.l == 0 && (cur.stop || errs || cur.t >= a.t_end)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.slot[a.sp].run = 0;
            a.slot[a.sp ^ 1].t = cur.t;
            a.slot[a.sp ^ 1].stop = 1;
        }
        return;
    }
    double avg[2][NC], sig[2][NC], beta;
    nu_statistics<NC>(a, a.gp, pt, sh, avg, sig, beta);
    double tau = cur.tau, tau_max = cur.tau_max;
    if (a.l == 0) {                                  // the step's tau, the same in every workgroup
        tau_max = a.dt_fixed;
        if (!(a.dt_fixed > 0.0)) {
            if (!(beta > 0.0) || !isfinite(beta)) {
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    a.err[2] = 1;
                    a.slot[a.sp].run = 0;
                    a.slot[a.sp ^ 1].t = cur.t;
                    a.slot[a.sp ^ 1].stop = 1;
                }
                return;
            }
            tau_max = a.cfl * a.hmax / beta;
        }
        tau = tau_max;
        bool last = false;
        if (cur.t + tau >= a.t_end) tau = a.t_end - cur.t, last = true;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.slot[a.sp].tau = tau;
            a.slot[a.sp].tau_max = tau_max;
            a.slot[a.sp].run = 1;
            a.slot[a.sp ^ 1].t = last ? a.t_end : cur.t + tau;
            a.slot[a.sp ^ 1].stop = last;
            *a.nexec += 1;
        }
    }
    if (a.oe && K > 0 && !a.first) {
        double isig[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) isig[q] = sig[M][q] != 0.0 ? 1.0 / sig[M][q] : 0.0;
        nu_damp<K, FLUX>(a, g, nb, a.l == 0 ? tau_prev : tau, isig, u);
    }
    if (c.has) {
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) dmp[M][q * K1 + m][c.s] = u[q][m];
    }
    if (a.l == 0 && c.owned) {                       // u^n, damped, for the later stages
        double *dn = M == 0 ? a.UC : a.UD;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) dn[(long long)(q * K1 + m) * a.n + i] = u[q][m];
    }
    __syncthreads();
    // operator of eq:1D_H on the owned cell, from the damped cells in LDS: primal
    // i in slot s has dual i, i+1 in dual slots s-1, s; dual i in slot s has
    // primal i-1, i in primal slots s, s+1
    double st[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) st[r] = stat_identity(r == RW - 1 ? 1 : r % 3);
    if (c.owned) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int ns = M == 0 ? c.s - 1 + p : c.s + p;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m) nb[p][q][m] = dmp[1 - M][q * K1 + m][ns];
        }
        const double itm = 1.0 / tau_max;
        double R[NC][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) R[q][m] = 0.0;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const double x0 = p == 0 ? g.lo : g.split, x1 = p == 0 ? g.split : g.hi;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double x = 0.5 * (x0 + x1) + 0.5 * (x1 - x0) * G.s[k], jac = 0.5 * (x1 - x0) * G.w[k];
                const double xi = 2.0 * (x - g.c) * g.iw, xn = 2.0 * (x - g.cn[p]) * g.iwn[p];
                double v[NC], uk[NC], fv[NC];
                eval<K, NC>(nb[p], 0, xn, 1.0, v);
                eval<K, NC>(u, 0, xi, 1.0, uk);
                F::f(v, fv, a.p0);
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int m = 0; m < K1; ++m)
                        R[q][m] += jac * ((v[q] - uk[q]) * itm * legr(m, 0, xi) + fv[q] * (2.0 * g.iw) * legr(m, 1, xi));
            }
        }
        double vl[NC], vr[NC], fl[NC], fr[NC];
        eval<K, NC>(nb[0], 0, 2.0 * (g.lo - g.cn[0]) * g.iwn[0], 1.0, vl);
        eval<K, NC>(nb[1], 0, 2.0 * (g.hi - g.cn[1]) * g.iwn[1], 1.0, vr);
        F::f(vl, fl, a.p0);
        F::f(vr, fr, a.p0);
        double *out = M == 0 ? a.TC[a.gp ^ 1] : a.TD[a.gp ^ 1];
        double o[NC][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                const double sgn = (m % 2 == 0) ? 1.0 : -1.0;
                const double Lm = (2.0 * m + 1.0) * g.iw * (R[q][m] - (fr[q] - fl[q] * sgn));
                const double base = a.l > 0 ? a.cn * un[q][m] : 0.0;
                o[q][m] = base + (a.cw * u[q][m] + tau * a.dd * Lm);
                out[(long long)(q * K1 + m) * a.n + i] = o[q][m];
            }
        nu_cell_stats<K, FLUX>(a, g, o, st, true);
    }
    nu_store_partials<NC>(a, a.gp ^ 1, M, st);
}

// The end of a call: the state after the executed steps, damped unless no step
// ran, into the caller's arrays.
template <int K, int FLUX>
__global__ void __launch_bounds__(NB) k_nu_final(NuArgs a) {
    constexpr int NC = FluxT<FLUX>::NC, K1 = K + 1;
    __shared__ double sh[2 * Rows<NC>::RW * (NB / WAVE)];
    const long long done = *a.nexec;
    const int gp = (int)((done * a.ns) & 1);
    const NuCell c = nu_cell(a);
    const int M = c.M, i = c.i;
    const double *own = M == 0 ? a.TC[gp] : a.TD[gp], *oth = M == 0 ? a.TD[gp] : a.TC[gp];
    const NuGeo g = nu_geo(a, M, i);
    double u[NC][K1], nb[2][NC][K1];
    load_cell<K, NC>(own, a.n, i, u);
    if (a.oe && K > 0 && done > 0) {                 // uniform over the grid
#pragma unroll
        for (int p = 0; p < 2; ++p) load_cell<K, NC>(oth, a.n, g.j[p], nb[p]);
        NuPart<NC> pt;
        nu_stat_load<NC>(a, gp, pt);
        double avg[2][NC], sig[2][NC], beta;
        nu_statistics<NC>(a, gp, pt, sh, avg, sig, beta);
        double isig[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) isig[q] = sig[M][q] != 0.0 ? 1.0 / sig[M][q] : 0.0;
        nu_damp<K, FLUX>(a, g, nb, a.slot[(int)(done & 1) ^ 1].tau, isig, u);
    }
    if (!c.owned) return;
    double *dst = M == 0 ? a.dstC : a.dstD;
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) dst[(long long)(q * K1 + m) * a.n + i] = u[q][m];
}

struct NuState {
    int n = 0, nc = 0, k = 0;
    double *geo = nullptr;          // edges [n+1] | cC | wC | cD | wD
    double *buf = nullptr;          // T0 (C|D) | T1 (C|D) | U (C|D)
    double *part = nullptr;
    NuSlot *slot = nullptr;
    long long *nexec = nullptr;
    int *err = nullptr;
    long long *nexec_h = nullptr;
    NuSlot *slot_h = nullptr;
    int *err_h = nullptr;
    // POLL steps from an even step index, captured once per (t_end, fixed step, h_max)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    double g_tend = 0.0, g_dt = 0.0, g_hmax = 0.0;
};

void free_state(NuState *s) {
    if (!s) return;
    (void)hipFree(s->geo);
    (void)hipFree(s->buf);
    (void)hipFree(s->part);
    (void)hipFree(s->slot);
    (void)hipFree(s->nexec);
    (void)hipFree(s->err);
    if (s->nexec_h) (void)hipHostFree(s->nexec_h);
    if (s->slot_h) (void)hipHostFree(s->slot_h);
    if (s->err_h) (void)hipHostFree(s->err_h);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    delete s;
}

// which: 0 initial statistics, 1 stage, 2 final
template <int FLUX>
void launch_flux(int which, const NuArgs &a, hipStream_t st) {
    const dim3 grid(a.nblk), block(NB);
    switch (a.k) {
#define NU_CASE(K)                                                                              \
    case K:                                                                                     \
        if (which == 0) hipLaunchKernelGGL((k_nu_init<K, FLUX>), grid, block, 0, st, a);        \
        else if (which == 1) hipLaunchKernelGGL((k_nu_step<K, FLUX>), grid, block, 0, st, a);   \
        else hipLaunchKernelGGL((k_nu_final<K, FLUX>), grid, block, 0, st, a);                  \
        break;
    NU_CASE(0)
    NU_CASE(1)
    NU_CASE(2)
    default:
    NU_CASE(3)
#undef NU_CASE
    }
}

void launch_kind(int which, const NuArgs &a, hipStream_t st) {
    if (a.flux == OECDG_FLUX_ADVECTION) launch_flux<0>(which, a, st);
    else if (a.flux == OECDG_FLUX_BURGERS) launch_flux<1>(which, a, st);
    else launch_flux<2>(which, a, st);
}

}  // namespace

void destroy_nu(oecdg_handle *h) {
    free_state(static_cast<NuState *>(handle_extnu(h)));
    handle_extnu(h) = nullptr;
}

#define NUCHK(h, call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) return handle_fail(h, OECDG_EHIP, hipGetErrorString(e_)); \
    } while (0)

int run_nonuniform(oecdg_handle *h, const double *edges_h, double *uC, double *uD, double t_end, int64_t nsteps,
                   double dt_fixed, double *t_out, int64_t *steps_out) {
    const oecdg_desc &d = handle_desc(h);
    if (handle_nbatch(h) != 1 || d.dim != 1 || d.bc != OECDG_BC_PERIODIC)
        return handle_fail(h, OECDG_EUNSUPPORTED, "non-uniform mesh: one periodic 1D instance only");
    const int rk = d.rk == 0 ? 3 : d.rk;
    if (rk == 4) return handle_fail(h, OECDG_EUNSUPPORTED, "non-uniform mesh: forward Euler, SSP-RK2 or SSP-RK3");
    if (!edges_h || !uC || !uD) return handle_fail(h, OECDG_EINVAL, "null pointer");
    if (!(t_end >= 0.0) || (std::isinf(t_end) && nsteps < 0) || std::isnan(dt_fixed))
        return handle_fail(h, OECDG_EINVAL, "bad t_end / nsteps / dt_fixed");
    const int n = (int)d.nx, k = d.k, K1 = k + 1;
    const int nc = d.flux == OECDG_FLUX_EULER ? 3 : 1;
    const double L = d.xhi - d.xlo;
    if (edges_h[0] != d.xlo || edges_h[n] != d.xhi) return handle_fail(h, OECDG_EINVAL, "edges must span [xlo, xhi]");
    double hmax = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(edges_h[i + 1] > edges_h[i])) return handle_fail(h, OECDG_EINVAL, "edges must increase strictly");
        hmax = fmax(hmax, edges_h[i + 1] - edges_h[i]);
    }
    hipStream_t st = handle_stream(h);
    NuState *s = static_cast<NuState *>(handle_extnu(h));
    const int nblk = (n + CPB - 1) / CPB;
    const int rows = 2 * (3 * nc + 1);          // partial rows of both meshes
    const size_t S1 = (size_t)nc * K1 * n;      // one mesh
    if (!s) {
        s = new NuState();
        s->n = n, s->nc = nc, s->k = k;
        handle_extnu(h) = s;
        if (hipMalloc(&s->geo, sizeof(double) * (5 * (size_t)n + 1)) != hipSuccess ||
            hipMalloc(&s->buf, sizeof(double) * 6 * S1) != hipSuccess ||
            hipMalloc(&s->part, sizeof(double) * 2 * rows * (size_t)nblk) != hipSuccess ||
            hipMalloc(&s->slot, 2 * sizeof(NuSlot)) != hipSuccess || hipMalloc(&s->err, sizeof(int) * 4) != hipSuccess ||
            hipMalloc(&s->nexec, sizeof(long long)) != hipSuccess ||
            hipHostMalloc(&s->nexec_h, sizeof(long long)) != hipSuccess ||
            hipHostMalloc(&s->slot_h, 2 * sizeof(NuSlot)) != hipSuccess ||
            hipHostMalloc(&s->err_h, sizeof(int) * 4) != hipSuccess) {
            destroy_nu(h);
            return handle_fail(h, OECDG_ENOMEM, "non-uniform mesh buffers");
        }
    }
    // geometry: edges, primal centres/widths, dual centres/widths (dual 0 reaches below xlo)
    std::vector<double> g(5 * (size_t)n + 1);
    double *e = g.data(), *cC = e + n + 1, *wC = cC + n, *cD = wC + n, *wD = cD + n;
    std::memcpy(e, edges_h, sizeof(double) * (n + 1));
    for (int i = 0; i < n; ++i) cC[i] = 0.5 * (e[i] + e[i + 1]), wC[i] = e[i + 1] - e[i];
    for (int j = 0; j < n; ++j) {
        const double cl = j == 0 ? cC[n - 1] - L : cC[j - 1], wl = j == 0 ? wC[n - 1] : wC[j - 1];
        cD[j] = 0.5 * (cl + cC[j]);
        wD[j] = 0.5 * (wl + wC[j]);
    }
    NuArgs a{};
    a.n = n, a.k = k, a.flux = d.flux, a.oe = d.oe;
    const int ns = rk == 1 ? 1 : rk == 2 ? 2 : 3;
    a.ns = ns;
    a.L = L, a.hmax = hmax, a.cfl = d.cfl, a.t_end = t_end, a.dt_fixed = dt_fixed;
    a.p0 = d.flux_param[0];                      // advection speed or gamma
    a.edges = s->geo, a.cC = s->geo + n + 1, a.wC = a.cC + n, a.cD = a.wC + n, a.wD = a.cD + n;
    a.part = s->part, a.slot = s->slot, a.nexec = s->nexec, a.err = s->err, a.nblk = nblk;
    a.TC[0] = s->buf, a.TD[0] = a.TC[0] + S1, a.TC[1] = a.TD[0] + S1, a.TD[1] = a.TC[1] + S1;
    a.UC = a.TD[1] + S1, a.UD = a.UC + S1;
    a.dstC = uC, a.dstD = uD;

    NUCHK(h, hipMemcpyAsync(s->geo, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, st));
    const NuSlot s0[2] = {{0.0, 0.0, 0.0, 0, 0}, {0.0, 0.0, 0.0, 0, 0}};
    NUCHK(h, hipMemcpyAsync(s->slot, s0, sizeof(s0), hipMemcpyHostToDevice, st));
    NUCHK(h, hipMemsetAsync(s->err, 0, sizeof(int) * 4, st));
    NUCHK(h, hipMemsetAsync(s->nexec, 0, sizeof(long long), st));
    NUCHK(h, hipMemcpyAsync(a.TC[0], uC, sizeof(double) * S1, hipMemcpyDeviceToDevice, st));
    NUCHK(h, hipMemcpyAsync(a.TD[0], uD, sizeof(double) * S1, hipMemcpyDeviceToDevice, st));
    launch_kind(0, a, st);                       // statistics of the initial data (parity 0)

    // the stage launches of step n; they depend on n only through the parities
    // of n and of n * ns, and through n == 0
    auto enqueue_step = [&](int64_t n_step, hipStream_t q) {
        NuArgs b = a;
        b.sp = (int)(n_step & 1);
        b.first = n_step == 0;
        for (int l = 0; l < ns; ++l) {
            const RKStage r = rk_stage(rk, l);
            b.l = l;
            b.gp = (int)((n_step * ns + l) & 1);
            b.cn = l == 0 ? 0.0 : r.cn, b.cw = r.cw, b.dd = r.d;
            b.first = n_step == 0 && l == 0;
            launch_kind(1, b, q);
        }
    };
    // whole blocks of POLL steps from a multiple of POLL (even, > 0) replay a captured graph
    if (s->gexec && (s->g_tend != t_end || s->g_dt != dt_fixed || s->g_hmax != hmax))
        (void)hipGraphExecDestroy(s->gexec), s->gexec = nullptr;
    auto ensure_graph = [&]() -> int {
        if (s->gexec) return OECDG_OK;
        if (!s->cap) NUCHK(h, hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        NUCHK(h, hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < POLL; ++j) enqueue_step(POLL + j, s->cap);
        NUCHK(h, hipStreamEndCapture(s->cap, &gr));
        const hipError_t e = hipGraphInstantiate(&s->gexec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        NUCHK(h, e);
        s->g_tend = t_end, s->g_dt = dt_fixed, s->g_hmax = hmax;
        return OECDG_OK;
    };
    int64_t step = 0;
    while (nsteps < 0 || step < nsteps) {
        if (step > 0 && step % POLL == 0 && !std::isinf(t_end)) {
            NUCHK(h, hipMemcpyAsync(s->slot_h, s->slot, 2 * sizeof(NuSlot), hipMemcpyDeviceToHost, st));
            NUCHK(h, hipStreamSynchronize(st));
            if (s->slot_h[step & 1].stop) break;
        }
        if (step > 0 && step % POLL == 0 && (nsteps < 0 || nsteps - step >= POLL)) {
            const int rc = ensure_graph();
            if (rc != OECDG_OK) return rc;
            NUCHK(h, hipGraphLaunch(s->gexec, st));
            step += POLL;
        } else {
            enqueue_step(step, st);
            ++step;
        }
        NUCHK(h, hipGetLastError());
    }
    launch_kind(2, a, st);                       // the state reached, damped, into (uC, uD)
    NUCHK(h, hipGetLastError());
    NUCHK(h, hipMemcpyAsync(s->slot_h, s->slot, 2 * sizeof(NuSlot), hipMemcpyDeviceToHost, st));
    NUCHK(h, hipMemcpyAsync(s->err_h, s->err, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    NUCHK(h, hipMemcpyAsync(s->nexec_h, s->nexec, sizeof(long long), hipMemcpyDeviceToHost, st));
    NUCHK(h, hipStreamSynchronize(st));
    if (s->err_h[2]) return handle_fail(h, OECDG_EINVAL, "wave speed is zero or not finite");
    if (s->err_h[0]) return handle_fail(h, OECDG_ENONFINITE, "non-finite coefficient");
    if (s->err_h[1]) return handle_fail(h, OECDG_ENONPHYSICAL, "non-physical cell average");
    if (t_out) *t_out = s->slot_h[step & 1].t;
    if (steps_out) *steps_out = *s->nexec_h;
    return OECDG_OK;
}

}  // namespace oecdg
