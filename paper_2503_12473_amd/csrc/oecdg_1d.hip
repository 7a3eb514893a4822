// oecdg_1d.hip -- gfx950 kernels of the 1D RK-OECDG stage update.
//
// One workgroup owns a tile of T primal cells [i0, i0+T) and the T dual cells
// [i0, i0+T) that interleave with them (dual cell j is centred on the left
// edge of primal cell j).  A stage kernel for stage l of step n
//   1. reduces the per-tile partial statistics left by the previous stage
//      (fixed order, so every workgroup gets bit-identical avg/sigma/beta),
//      and at l = 0 derives tau^n and tau_max^n (Sec. 2.1, tau = C h / beta);
//   2. stages its tile plus a two-cell halo of the pre-damping input into LDS
//      (coalesced structure-of-arrays loads);
//   3. applies the OE step F_tau of the previous stage in LDS (Sec. 2.2,
//      OEstep2D: delta_K^m from the primal/dual difference at the cell edges,
//      then the exact exponential a_j *= exp(-tau sum_{m<=j} delta^m));
//   4. evaluates the CDG operator (equcdg): the overlap coupling with
//      1/tau_max, the volume integral of f(w) with k+1 Gauss nodes on each
//      half cell, and the point fluxes of the other mesh at the cell edges;
//   5. forms the RK combination of eq:RKCDG (SSP-RK3 by default; forward
//      Euler, SSP-RK2 or classical RK4 on request) and writes the stage output;
//   6. writes the tile's partial statistics of that output for the next stage.
// The OE of the last stage of a run is applied by the final kernel.
#include "oecdg_device.h"
#include "oecdg_internal.h"
#include "oecdg_tables.h"

#include <math.h>
#include <string.h>

namespace oecdg {

// Threads per workgroup: two per cell (one per half cell) for the T primal
// and the T dual cells of a tile.
__host__ __device__ constexpr int nthreads(int T) { return 4 * T; }
// A mesh with nd = np + 1 dual cells and np a multiple of T has one dual cell
// (np) beyond np / T full tiles.  Rather than a tile of its own (one
// workgroup more than there are CUs for the 16384-cell workload: 15.0 instead
// of 12.8 us per stage), launches of such handles carry one more wave, whose
// first lane pair updates that cell in the instance's last tile.  Tiles of
// 128 keep the extra tile (a fifth wave per SIMD would cap the registers).
__host__ __device__ constexpr int max_threads(int T) { return nthreads(T) + tail_threads(T); }

// Segmented reduction over the two halves of a workgroup (primal threads
// [0, H), dual threads [H, 2H)), H a multiple of the wave size.  NV values per
// thread, kinds given.  On return the threads tid == 0 (primal) and tid == H
// (dual) hold the half's result (waves combined in order).  xwave: the
// launch's extra wave (threads [2H, 2H + WAVE)) carries a cell and reduces its
// own values, left in scratch at wave 2H / WAVE; otherwise it does no work here.
// scratch: NV * (2H / WAVE + 1) doubles of LDS.
template <int H, int NV>
__device__ void reduce_halves(double (&v)[NV], const int (&kind)[NV], double *scratch, bool xwave, bool xwl) {
    static_assert(H % WAVE == 0, "halves are whole waves");
    constexpr int WPH = H / WAVE;          // waves per half
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    if (!xwl || tid < 2 * H || xwave) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = wave_reduce(kind[j], v[j]);
        if (lane == WAVE - 1) {
#pragma unroll
            for (int j = 0; j < NV; ++j) scratch[wave * NV + j] = v[j];
        }
    }
    __syncthreads();
    if (tid == 0 || tid == H) {
        const int w0 = tid / WAVE;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double x = scratch[w0 * NV + j];
            for (int w = 1; w < WPH; ++w) x = stat_op(kind[j], x, scratch[(w0 + w) * NV + j]);
            v[j] = x;
        }
    }
    __syncthreads();
}

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

template <int K, int NC, int W>
__device__ inline void lds_cell(const double *s, int li, double (&c)[NC][K + 1]) {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m <= K; ++m) c[q][m] = s[(q * (K + 1) + m) * W + li];
}

// Element e of the tile's LDS image of the pre-damping input: primal cells
// [i0-1, i0+T] (rows q*(k+1)+m of length T+2), then dual cells [i0-1, i0+T].
// Periodic wrap; outflow: constant-extension ghosts for primal -1 and np
// (reflective walls load the same and mirror_ghosts overwrites them); inflow:
// the instance's fixed ghost states; zeros for dual cells that do not exist.
// Sign of coefficient (q, m) of a reflective ghost: (-1)^m, and -1 more for
// the momentum (q = 1 of the Euler system).
__device__ inline double mirror_sign(int q, int m) { return ((m & 1) ^ (q == 1)) ? -1.0 : 1.0; }

// GH: kernels of the Euler flux with wall or inflow ghosts (FluxT<3>), the
// only ones that carry the inflow ghost states.
template <int K, int NC, int T, bool GH>
__device__ inline double tile_elem(const Inst1D &I, int i0, const double *__restrict__ inC,
                                   const double *__restrict__ inD, int e) {
    constexpr int W = T + 2, K1 = K + 1, PER = NC * K1 * W;
    const int mesh = e >= PER;
    const int r = e - mesh * PER;
    const int qm = r / W;
    const int li = r - qm * W;
    int gi = i0 - 1 + li;
    if (mesh == 0) {
        const int np = I.np;
        if (I.bc == 0) {
            gi = gi < 0 ? gi + np : (gi >= np ? gi - np : gi);
            if (gi < 0 || gi >= np) gi = ((gi % np) + np) % np;   // mesh shorter than a tile
            return inC[(long long)qm * np + gi];
        }
        if (gi < 0 || gi >= np) {
            if (qm % K1 != 0) return 0.0;
            if constexpr (GH) {
                if (I.bc == 3) return I.gin[gi < 0 ? 0 : 1][qm / K1];
            }
            return inC[(long long)qm * np + (gi < 0 ? 0 : np - 1)];
        }
        return inC[(long long)qm * np + gi];
    }
    const int nd = I.nd;
    if (I.bc == 0) {
        gi = gi < 0 ? gi + nd : (gi >= nd ? gi - nd : gi);
        if (gi < 0 || gi >= nd) gi = ((gi % nd) + nd) % nd;
    }
    return (gi >= 0 && gi < nd) ? inD[(long long)qm * nd + gi] : 0.0;
}

// Reflective walls (Euler): primal ghosts -1 and np in the LDS tile become the
// mirror images of cells 0 and np-1 (mode m times (-1)^m, the momentum
// negated).  Only kernels of the walled Euler flux (FluxT<3>) contain this,
// and only their tiles that hold a ghost call it (a workgroup-uniform test),
// followed by a barrier; damp_tile mirrors the damped end cells again.
template <int K, int NC, int T>
__device__ inline bool has_wall_ghost(const Inst1D &I, int i0) {
    return I.bc == 2 && (i0 == 0 || I.np - i0 <= T);
}

template <int K, int NC, int T>
__device__ inline void mirror_ghosts(const Inst1D &I, int i0, double *sC) {
    constexpr int W = T + 2, K1 = K + 1;
    const int t = threadIdx.x;
    if (t < NC * K1) {
        const double sg = mirror_sign(t / K1, t % K1);
        if (i0 == 0) sC[t * W] = sg * sC[t * W + 1];
        const int lr = I.np - i0;                  // LDS column of cell np-1; its ghost is the next one
        if (lr >= 0 && lr <= T) sC[t * W + lr + 1] = sg * sC[t * W + lr];
    }
}

template <int K, int NC, int T, bool GH>
__device__ inline void load_tile(const Inst1D &I, int i0, const double *__restrict__ inC,
                                 const double *__restrict__ inD, double *s, bool xwl) {
    constexpr int PER = NC * (K + 1) * (T + 2);
    if (!xwl || threadIdx.x < nthreads(T))
        for (int e = threadIdx.x; e < 2 * PER; e += nthreads(T)) s[e] = tile_elem<K, NC, T, GH>(I, i0, inC, inD, e);
}

// Apply F_tau in LDS to primal cells [i0-1, i0+T-1] and dual cells [i0, i0+T]
// (the cells whose damped values the tile's operator needs), one cell per
// thread, all damping factors computed from the pre-damping values first.
template <int K, int FLUX, int T>
__device__ inline void damp_tile(const Inst1D &I, int i0, double *sC, double *sD, const double (*sig)[3],
                                 double tau) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, W = T + 2, K1 = K + 1;
    static_assert(nthreads(T) >= 2 * T + 2, "one damping item per thread");
    const double hinv = 1.0 / I.h;
    double fac[K1];
    const int w = threadIdx.x;
    const int mesh = w < T + 1 ? 0 : 1;
    const int li = mesh == 0 ? w : w - T;          // primal 0..T, dual 1..T+1
    const int gi = i0 - 1 + li;
    bool active = w < 2 * T + 2;
    if (active && I.bc != 0) active = mesh == 0 ? (gi >= 0 && gi < I.np) : (gi >= 0 && gi < I.nd);
    if (active) {
        double own[NC][K1], nl[NC][K1], nr[NC][K1];
        if (mesh == 0) {
            lds_cell<K, NC, W>(sC, li, own);
            lds_cell<K, NC, W>(sD, li, nl);
            lds_cell<K, NC, W>(sD, li + 1, nr);
        } else {
            lds_cell<K, NC, W>(sD, li, own);
            lds_cell<K, NC, W>(sC, li - 1, nl);
            lds_cell<K, NC, W>(sC, li, nr);
        }
        double ubar[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) ubar[q] = own[q][0];
        const double beta = F::speed(ubar, I.p0);
        oe_factors<K, NC>(own, nl, nr, beta, sig[mesh], hinv, tau, fac);
    }
    __syncthreads();
    if (active) {
        double *s = mesh == 0 ? sC : sD;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 1; m <= K; ++m) s[(q * K1 + m) * W + li] *= fac[m];
        // reflective walls: the ghost next to an end cell mirrors its damped values
        if constexpr (FLUX == 3) {
            if (I.bc == 2 && mesh == 0 && (gi == 0 || gi == I.np - 1)) {
                const int lg = gi == 0 ? li - 1 : li + 1;
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int m = 1; m <= K; ++m)
                        s[(q * K1 + m) * W + lg] = mirror_sign(q, m) * s[(q * K1 + m) * W + li];
            }
        }
    }
    __syncthreads();
}

// Partial statistics of the tile's output: each thread of a cell's pair takes
// half of the sigma sample points (hf = 1: the right-half nodes and xi = 1;
// hf = 0: their mirror images, through the sign flip of odd modes); the cell
// average counts once (hf = 0).  Reduced over the primal and dual halves of the
// workgroup and written to column tile of part[row][tile].
template <int K, int FLUX, int T>
__device__ inline void tile_partials(const Inst1D &I, bool valid, int mesh, int hf,
                                     const double (&out)[FluxT<FLUX>::NC][K + 1], double *part, long long ntot,
                                     int tile, double *scratch, bool xwave, bool xwl) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, NV = 3 * NC + 1;
    constexpr Tab<K> tb = make_tab<K>();
    const double flip = hf ? 1.0 : -1.0;
    double v[NV];
    int kind[NV];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        kind[3 * q] = 0;
        kind[3 * q + 1] = 1;
        kind[3 * q + 2] = 2;
        double mx = -INFINITY, mn = INFINITY;
#pragma unroll
        for (int sidx = K + 2; sidx < 2 * K + 4; ++sidx) {
            double x = 0.0;
#pragma unroll
            for (int n = 0; n <= K; ++n) x += ((n & 1) ? flip * out[q][n] : out[q][n]) * tb.SP[sidx][n];
            mx = fmax(mx, x);
            mn = fmin(mn, x);
        }
        v[3 * q] = (valid && hf == 0) ? out[q][0] : 0.0;
        v[3 * q + 1] = valid ? mx : -INFINITY;
        v[3 * q + 2] = valid ? mn : INFINITY;
    }
    double ubar[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) ubar[q] = out[q][0];
    kind[NV - 1] = 1;
    v[NV - 1] = valid ? F::speed(ubar, I.p0) : -INFINITY;
    reduce_halves<2 * T, NV>(v, kind, scratch, xwave, xwl);
    if (threadIdx.x == 0 || threadIdx.x == 2 * T) {
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int kd = 0; kd < 3; ++kd) part[stat_index(mesh, q, kd) * ntot + tile] = v[3 * q + kd];
        part[(ST_BETA + mesh) * ntot + tile] = v[NV - 1];
    }
    // the extra wave's dual cell np gets the next column, as the separate
    // tile of that cell would have written it (no primal cells: identities)
    if (xwave && threadIdx.x == 4 * T) {
        const double *xs = scratch + (4 * T / WAVE) * NV;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int kd = 0; kd < 3; ++kd) {
                part[stat_index(0, q, kd) * ntot + tile + 1] = stat_identity(kd);
                part[stat_index(1, q, kd) * ntot + tile + 1] = xs[3 * q + kd];
            }
        part[ST_BETA * ntot + tile + 1] = -INFINITY;
        part[(ST_BETA + 1) * ntot + tile + 1] = xs[NV - 1];
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

constexpr int lds_doubles(int K, int NC, int T) { return 2 * NC * (K + 1) * (T + 2); }
constexpr int scratch_doubles(int T) { return NSTAT * ((max_threads(T) + WAVE - 1) / WAVE) + NSTAT; }

// Cell of thread tid in a tile: primal cell tid/2 < T, dual cell tid/2 - T < T
// (both relative to i0); the extra wave's first lane pair takes dual cell T of
// a tail tile (the instance's dual cell np), its other lanes no cell.  c is
// kept within the LDS tile; returns whether the thread has a cell.
template <int T>
__device__ inline bool cell_of(const Inst1D &I, int tile, int i0, int tid, int &mesh, int &c, int &gi, bool xwl) {
    const int cidx = tid >> 1;
    mesh = cidx < T ? 0 : 1;
    c = cidx - mesh * T;
    if (xwl && c >= T) {
        const bool tail = I.tail && tile == I.tile0 + I.ntiles - 1 && c == T;
        c = T;
        gi = i0 + T;
        return tail && gi < I.nd;
    }
    gi = i0 + c;
    return gi < (mesh == 0 ? I.np : I.nd);
}

// ---------------------------------------------------------- stage tile ---
// Thread tid works on cell tid/2 of the tile (primal cells first) and on the
// half cell tid%2 of it.

// Doubles of a tile's LDS image (with its halo) that each thread loads.
template <int K, int FLUX, int T>
constexpr int tile_loads() { return (2 * FluxT<FLUX>::NC * (K + 1) * (T + 2) + nthreads(T) - 1) / nthreads(T); }

// Issue the loads of tile `tile`'s LDS image (stage input of parity sp) into pre.
template <int K, int FLUX, int T>
__device__ inline void load_pre(const StageArgs &a, int tile, int sp, double (&pre)[tile_loads<K, FLUX, T>()]) {
    constexpr int NC = FluxT<FLUX>::NC, PER = NC * (K + 1) * (T + 2), NT = nthreads(T);
    const Tile1D tl = a.tiles[tile];
    const Inst1D I = a.inst[tl.inst];
    const double *inC = a.BC[sp] + I.offC, *inD = a.BD[sp] + I.offD;
#pragma unroll
    for (int i = 0; i < tile_loads<K, FLUX, T>(); ++i) {
        const int e = threadIdx.x + i * NT;
        pre[i] = e < 2 * PER ? tile_elem<K, NC, T, FLUX == 3>(I, tl.i0, inC, inD, e) : 0.0;
    }
}

// folded: the instance's statistics were reduced by k_fold into a.red (batched
// launches); otherwise every workgroup reduces the partial columns itself.
// have_pre: the tile's LDS image is already in pre (loaded while the previous
// tile of this workgroup was computed); next_tile >= 0: once this tile's image
// is in LDS, the loads of next_tile's image are issued into pre, so they are in
// flight while this tile is damped and updated (batched launches).
// Returns whether next_tile's loads were issued.
template <int K, int FLUX, int T>
__device__ bool stage_tile(const StageArgs &a, int l, int par, int first, int tile, double *smem, bool xwl,
                           bool folded, double (&pre)[tile_loads<K, FLUX, T>()], bool have_pre = false,
                           int next_tile = -1) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, W = T + 2, PER = NC * K1 * W, NT = nthreads(T);
    constexpr int NLD = tile_loads<K, FLUX, T>();
    const int tid = threadIdx.x;
    const bool coh = a.coherent;
    Tile1D tl;
    Inst1D I;
    if (a.ninst == 1) {                      // single instance: everything from the kernel arguments
        tl.inst = 0;
        tl.i0 = tile * T;
        I = a.inst0;
    } else {
        tl = a.tiles[tile];
        I = a.inst[tl.inst];
    }
    const int i0 = tl.i0;
    const bool lead = (tile == I.tile0) && tid == 0;
    Slot *S = a.slots + 2 * tl.inst;
    const bool single = a.tau_override > 0.0;
    const int sp = ((a.ns & 1 ? par : 0) + l) & 1;   // parity of the global stage index ns n + l
    double *sC = smem, *sD = smem + PER;
    double *red = smem + lds_doubles(K, NC, T);
    double *scratch = red + NSTAT;

    const int hf = tid & 1;
    int mesh, c, gi;
    const bool valid = cell_of<T>(I, tile, i0, tid, mesh, c, gi, xwl);
    const bool mainthr = !xwl || tid < NT;      // not the launch's extra wave
    const int ncell = mesh == 0 ? I.np : I.nd;
    double *UM = (mesh == 0 ? a.UC + I.offC : a.UD + I.offD);
    const bool damp = a.damp_input && I.oe && K > 0 && !(l == 0 && first);
    const bool need_beta = l == 0 && !single && a.dt_fixed <= 0.0;
    const bool need_red = damp || need_beta;
    const int ns = need_beta ? Partials<NC>::NS : Partials<NC>::NS - 2;

    // One round trip for every load that does not depend on another: this
    // step's and the previous step's scalars, the tile's pre-damping input and
    // the previous stage's partial statistics (issued before any test on them).
    const Slot cur = ld_slot(&S[par], coh), prev = ld_slot(&S[par ^ 1], coh);
    if (!have_pre) {
        const double *inC = a.BC[sp] + I.offC, *inD = a.BD[sp] + I.offD;
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int e = tid + i * NT;
            pre[i] = (e < 2 * PER && mainthr) ? tile_elem<K, NC, T, FLUX == 3>(I, i0, inC, inD, e) : 0.0;
        }
    }
    Partials<NC> pv;
    double redv = 0.0;                       // folded: row tid of the instance's reduced statistics
    if (need_red) {
        if (folded) {
            if (tid < NSTAT) redv = a.red[(long long)tl.inst * NSTAT + tid];
        } else {
            load_partials<NT, NC>(a.part[sp ^ 1], a.ntiles, I.tile0, I.npart, ns, pv, xwl);
        }
    }

    if (!single) {
        if (l == 0 && cur.t >= a.t_end) {    // a step that is not taken: carry the time over
            if (lead) {
                S[par].done = 1;
                S[par ^ 1].t = cur.t;
            }
            return false;
        }
        if (l > 0 && cur.done) return false;
    }
    if (need_red) {
        if (folded) {
            if (tid < NSTAT) red[tid] = redv;
            __syncthreads();
        } else {
            finish_partials<NT, NC>(pv, a.part[sp ^ 1], a.ntiles, I.tile0, I.npart, ns, red, scratch, xwl);
        }
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
        if (lead) {
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
    if (!single && l == a.ns - 1 && lead) {   // the step's last stage: time and step count
        const double tnext = last ? a.t_end : cur.t + tau;
        S[par ^ 1].t = tnext;
        Final *f = a.fin + tl.inst;
        f->t = tnext;
        f->tau = tau;
        f->nexec = ld_ll(&f->nexec, coh) + 1;
    }

    double sig[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (damp) finish_stats<NC>(I, red, sig);
    const double tau_in = (l == 0) ? prev.tau : tau;

#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * NT;
        if (e < 2 * PER && mainthr) smem[e] = pre[i];
    }
    // u^n of this thread's cell: its latency overlaps the damping below
    double un[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) un[q][m] = (l > 0 && valid) ? UM[(long long)(q * K1 + m) * ncell + gi] : 0.0;
    const bool prefetched = next_tile >= 0;    // workgroup-uniform
    if (prefetched) load_pre<K, FLUX, T>(a, next_tile, sp, pre);
    __syncthreads();
    if constexpr (FLUX == 3) {
        if (has_wall_ghost<K, NC, T>(I, i0)) {
            mirror_ghosts<K, NC, T>(I, i0, sC);
            __syncthreads();
        }
    }
    if (damp) damp_tile<K, FLUX, T>(I, i0, sC, sD, sig, tau_in);

    // A launch's extra wave computes only in the tile that carries dual cell np.
    const bool tail_tile = I.tail && tile == I.tile0 + I.ntiles - 1;
    double out[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) out[q][m] = 0.0;
    if (mainthr || tail_tile) {
        // own cell; the overlapping cell of this thread's half
        double own[NC][K1], nb[NC][K1];
        if (mesh == 0) {
            lds_cell<K, NC, W>(sC, c + 1, own);
            lds_cell<K, NC, W>(sD, c + 1 + hf, nb);
        } else {
            lds_cell<K, NC, W>(sD, c + 1, own);
            lds_cell<K, NC, W>(sC, c + hf, nb);
        }
        if (l == 0 && !single && valid) {
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m)
                    if (((q * K1 + m) & 1) == hf) UM[(long long)(q * K1 + m) * ncell + gi] = own[q][m];
        }
        if (l > 0 && a.DC && valid) {          // damped stage input, kept for the adjoint
            double *DM = mesh == 0 ? a.DC + I.offC : a.DD + I.offD;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m)
                    if (((q * K1 + m) & 1) == hf) DM[(long long)(q * K1 + m) * ncell + gi] = own[q][m];
        }

        const double inv_tm = 1.0 / taumax;
        double r[NC][K1];
        cdg_rate_half<K, FLUX>(nb, hf, I.p0, taumax * (1.0 / I.h), r);

        // eq:RKCDG: out = c_{l0} u^n [+ accumulated earlier stages] + c_{ll} u^l + tau d_{ll} L(u^l)
        const RKStage rs = rk_stage(a.rk, l);
        const double td = tau * rs.d;
        double *AM = nullptr;
        if (rs.acc_read || rs.ca != 0.0) AM = mesh == 0 ? a.AC + I.offC : a.AD + I.offD;
        bool finite = true;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                const double both = r[q][m] + pair_swap(r[q][m]);   // the two halves (a + b == b + a)
                const double rate = inv_tm * (both - own[q][m]);
                const double v = fma(td, rate, rs.cw * own[q][m]);
                double o = v;
                if (l > 0) {
                    double base = rs.cn * un[q][m];
                    if (rs.acc_read) base += valid ? AM[(long long)(q * K1 + m) * ncell + gi] : 0.0;
                    o = base + v;
                }
                out[q][m] = o;
                finite = finite && isfinite(o);
            }
        if (rs.ca != 0.0 && valid) {           // classical RK4: this stage's damped input joins the sum
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m)
                    if (((q * K1 + m) & 1) == hf) {
                        double *p = AM + (long long)(q * K1 + m) * ncell + gi;
                        *p = rs.acc_first ? rs.ca * own[q][m] : fma(rs.ca, own[q][m], *p);
                    }
        }
        double *OM = (mesh == 0 ? a.BC[sp ^ 1] + I.offC : a.BD[sp ^ 1] + I.offD);
        if (valid) {
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int m = 0; m < K1; ++m)
                    if (((q * K1 + m) & 1) == hf) OM[(long long)(q * K1 + m) * ncell + gi] = out[q][m];
            double ubar[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) ubar[q] = out[q][0];
            // a tolerated non-positive pressure (OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE) leaves the density
            const bool phys = (I.flags & OECDG_FLAG_ALLOW_NEGATIVE_PRESSURE) ? ubar[0] > 0.0 : F::physical(ubar, I.p0);
            if (hf == 0 && (!finite || !phys)) {
                if (!finite) a.err[0] = 1;
                if (!phys) a.err[1] = 1;
                a.err[3] = (int)(a.fin[tl.inst].nexec + 1);
            }
        }
    }
    tile_partials<K, FLUX, T>(I, valid, mesh, hf, out, a.part[sp], a.ntiles, tile, scratch, xwl && tail_tile, xwl);
    __syncthreads();
    return prefetched;
}

// Statistics of a given state (srcC/srcD) into part[1]: the partials that the
// first stage of a run reads (beta for tau^0).
template <int K, int FLUX, int T>
__device__ void stats_tile(const StageArgs &a, int tile, double *smem, bool xwl) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1;
    const Tile1D tl = a.ninst == 1 ? Tile1D{0, tile * T} : a.tiles[tile];
    const Inst1D I = a.ninst == 1 ? a.inst0 : a.inst[tl.inst];
    const int tid = threadIdx.x, hf = tid & 1;
    int mesh, c, gi;
    const bool valid = cell_of<T>(I, tile, tl.i0, tid, mesh, c, gi, xwl);
    const int ncell = mesh == 0 ? I.np : I.nd;
    const double *src = mesh == 0 ? a.srcC + I.offC : a.srcD + I.offD;
    double u[NC][K1];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int m = 0; m < K1; ++m) u[q][m] = valid ? src[(long long)(q * K1 + m) * ncell + gi] : 1.0;
    tile_partials<K, FLUX, T>(I, valid, mesh, hf, u, a.part[1], a.ntiles, tile, smem + NSTAT,
                              xwl && I.tail && tile == I.tile0 + I.ntiles - 1, xwl);
    __syncthreads();
}

// Final OE: u_sigma^N = F_tau(output of the last stage of step N-1) into (dstC, dstD); copy if no step ran.
template <int K, int FLUX, int T>
__device__ void final_tile(const StageArgs &a, int tile, double *smem, bool xwl) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, W = T + 2;
    const int tid = threadIdx.x;
    const Tile1D tl = a.ninst == 1 ? Tile1D{0, tile * T} : a.tiles[tile];
    const Inst1D I = a.ninst == 1 ? a.inst0 : a.inst[tl.inst];
    const long long N = a.fin[tl.inst].nexec;
    const double tau = a.fin[tl.inst].tau;
    const int bp = (int)((a.ns * N) & 1);   // buffer holding the last stage's output (or the input when N = 0)
    double *sC = smem, *sD = smem + NC * K1 * W;
    double *red = smem + lds_doubles(K, NC, T);
    double *scratch = red + NSTAT;
    const bool damp = N > 0 && I.oe && K > 0;
    double sig[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (damp) {
        reduce_instance<nthreads(T), NC>(a.part[(int)((a.ns * N - 1) & 1)], a.ntiles, I.tile0, I.npart, false, red,
                                         scratch, xwl);
        finish_stats<NC>(I, red, sig);
    }
    load_tile<K, NC, T, FLUX == 3>(I, tl.i0, a.BC[bp] + I.offC, a.BD[bp] + I.offD, smem, xwl);
    __syncthreads();
    if constexpr (FLUX == 3) {
        if (has_wall_ghost<K, NC, T>(I, tl.i0)) {
            mirror_ghosts<K, NC, T>(I, tl.i0, sC);
            __syncthreads();
        }
    }
    if (damp) damp_tile<K, FLUX, T>(I, tl.i0, sC, sD, sig, tau);
    const int hf = tid & 1;
    int mesh, c, gi;
    const bool valid = cell_of<T>(I, tile, tl.i0, tid, mesh, c, gi, xwl);
    const int ncell = mesh == 0 ? I.np : I.nd;
    if (valid) {
        const double *s = mesh == 0 ? sC : sD;
        double *dst = mesh == 0 ? a.dstC + I.offC : a.dstD + I.offD;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m)
                if (((q * K1 + m) & 1) == hf) dst[(long long)(q * K1 + m) * ncell + gi] = s[(q * K1 + m) * W + c + 1];
    }
    __syncthreads();
}

// --------------------------------------------------------------- kernels ---

// KM < 0: mixed-degree batch, dispatch on the instance's k per tile.
template <int KM, int FLUX, int T>
struct Disp {
    static constexpr int KL = KM < 0 ? MAXK : KM;
    static constexpr int LDS = lds_doubles(KL, FluxT<FLUX>::NC, T) + scratch_doubles(T);
    template <template <int, int, int> class Fn, typename... Args>
    __device__ static void run(int k, Args &&...args) {
        if constexpr (KM >= 0) {
            Fn<KM, FLUX, T>::go(args...);
        } else {
            switch (k) {
            case 0: Fn<0, FLUX, T>::go(args...); break;
            case 1: Fn<1, FLUX, T>::go(args...); break;
            case 2: Fn<2, FLUX, T>::go(args...); break;
            default: Fn<3, FLUX, T>::go(args...); break;
            }
        }
    }
};

template <int K, int FLUX, int T> struct StageFn {
    __device__ static void go(const StageArgs &a, int l, int par, int first, int tile, double *smem, bool xwl,
                              bool folded) {
        double pre[tile_loads<K, FLUX, T>()];
        stage_tile<K, FLUX, T>(a, l, par, first, tile, smem, xwl, folded, pre);
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

template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(XW ? max_threads(T) : nthreads(T)) void k_stage(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        const int k = a.ninst == 1 ? a.inst0.k : a.inst[a.tiles[tile].inst].k;
        D::template run<StageFn>(k, a, a.l, a.par, a.first, tile, smem, XW, false);
    }
}

// The stage kernel of batched launches (one degree per launch): the
// instance's statistics come reduced from k_fold (one fixed-order reduction
// per instance and stage) instead of every workgroup reducing all of its
// instance's partial columns, and a workgroup walks the tiles tbeg +
// blockIdx.x, + gridDim.x, ..., loading each tile's input while the previous
// one is damped and updated.
template <int K, int FLUX, int T>
__global__ __launch_bounds__(nthreads(T)) void k_stage_folded(StageArgs a) {
    __shared__ double smem[lds_doubles(K, FluxT<FLUX>::NC, T) + scratch_doubles(T)];
    double pre[tile_loads<K, FLUX, T>()];
    bool have = false;
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        const int next = tile + (int)gridDim.x < a.tend ? tile + (int)gridDim.x : -1;
        have = stage_tile<K, FLUX, T>(a, a.l, a.par, a.first, tile, smem, false, true, pre, have, next);
    }
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
    reduce_instance<nthreads(T), NC>(a.part[src], a.ntiles, I.tile0, I.npart, true, red, scratch);
    if (tid < NSTAT) a.red[(long long)b * NSTAT + tid] = red[tid];
}

template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(XW ? max_threads(T) : nthreads(T)) void k_stats(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        const int k = a.ninst == 1 ? a.inst0.k : a.inst[a.tiles[tile].inst].k;
        D::template run<StatsFn>(k, a, tile, smem, XW);
    }
}

template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(XW ? max_threads(T) : nthreads(T)) void k_final(StageArgs a) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
        const int k = a.ninst == 1 ? a.inst0.k : a.inst[a.tiles[tile].inst].k;
        D::template run<FinalFn>(k, a, tile, smem, XW);
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
// a barrier are read coherently (a.coherent).
template <int KM, int FLUX, int T, bool XW>
__global__ __launch_bounds__(XW ? max_threads(T) : nthreads(T)) void k_persistent(StageArgs a, long long nsteps, int single_instance) {
    using D = Disp<KM, FLUX, T>;
    __shared__ double smem[D::LDS];
    for (long long n = 0; n < nsteps; ++n) {
        const int par = (int)(n & 1);
        for (int l = 0; l < a.ns; ++l) {
            for (int tile = a.tbeg + blockIdx.x; tile < a.tend; tile += gridDim.x) {
                const int k = a.ninst == 1 ? a.inst0.k : a.inst[a.tiles[tile].inst].k;
                D::template run<StageFn>(k, a, l, par, n == 0, tile, smem, XW, false);
            }
            grid_barrier(a);
            if (l == 0 && single_instance && ld_i(&a.slots[par].done, true)) return;
            if (ld_i(&a.err[2], true)) return;
        }
    }
}

__global__ void k_init(StageArgs a, int ninst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// ------------------------------------------------------------ host side ---

static int tile_index(int tile) { return tile == 32 ? 0 : (tile == 64 ? 1 : (tile == 128 ? 2 : -1)); }
// kernel table index: the tile (0, 1, 2 for 32, 64, 128), or 3 / 4 for tiles
// of 32 / 64 launched with the extra wave
static int kernel_index(int tile, bool tailwave) {
    const int ti = tile_index(tile);
    return (ti >= 0 && tailwave && tail_threads(tile) > 0) ? ti + 3 : ti;
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
    return hipLaunchKernel(fn, dim3(grid), dim3(nthreads(tile) + (a.tailwave ? tail_threads(tile) : 0)), args, 0, s);
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

hipError_t launch_stage_1d(const StageArgs &a, int kmax, int flux, int tile, int grid, hipStream_t s) {
    int ti = kernel_index(tile, a.tailwave);
    if (ti < 0) return hipErrorInvalidValue;
    if (a.red) {                             // statistics folded by launch_fold_1d
        if (a.tailwave) return hipErrorInvalidValue;
        return launch(pick<4>(kmax, flux, ti), grid > 0 ? grid : a.tend - a.tbeg, tile, a, s);
    }
    return launch(pick<0>(kmax, flux, ti), grid > 0 ? grid : a.tend - a.tbeg, tile, a, s);
}

int folded_grid_1d(int k, int flux, int tile) {
    const int ti = tile_index(tile);
    if (ti < 0) return 0;
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pick<4>(k, flux, ti), nthreads(tile), 0) !=
        hipSuccess)
        return 0;
    return per_cu * ncu;
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
    const int nthr = nthreads(tile) + (tailwave ? tail_threads(tile) : 0);
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
    const int nthr = nthreads(tile) + (a.tailwave ? tail_threads(tile) : 0);
    return hipLaunchCooperativeKernel(pick<3>(kmax, flux, ti), dim3(grid), dim3(nthr), args, 0, s);
}

}  // namespace oecdg
