// oecdg_2d.hip -- 2D RK-OECDG on periodic Cartesian primal and dual meshes,
// tensor-product Q^k Legendre modes or the total-degree P^k (k = 1, 2, 3),
// linear advection or Euler.
//
// Per RK stage (eq:RKCDG) one tile kernel and one statistics kernel:
//   k_reduce2d  one workgroup folds the per-tile partial statistics of the
//               stage input into the global scalars: per mesh and component
//               the domain average and sigma (Sec. 2.2), the largest x and y
//               wave speeds, and at a step start tau and tau_max
//               (tau_max = C_CFL / (beta_x/h_x + beta_y/h_y), Sec. 2.1);
//   k_stage2d   one workgroup per tile of TX x TY primal cells and the dual
//               cells with the same indices.  It stages both meshes'
//               pre-damping input with a one-cell halo in LDS, applies the
//               OE step of the previous stage in place (OEstep2D solved
//               exactly, delta_K^m from the edge integrals of Sec. 2.2),
//               evaluates the operator of eq:2D_H on its cells, takes the
//               RK combination (the c/d table of eq:RKCDG: SSP-RK3 by
//               default, forward Euler, SSP-RK2 or classical RK4) and writes
//               the undamped stage output;
//   k_delta2d   the damping numerators and the tile's partial statistics of
//               that output.
// The same tile kernel, in other modes, damps a state without a stage (the
// end of a run or of a single stage) or only computes statistics.
//
// Work split inside a tile: four lanes (a quad) per cell.  For the operator
// lane t takes quadrant t (coupling and volume integrals against the one
// overlapping cell of the other mesh) and edge t (half-edge flux integrals
// on the other mesh's centre line); for the damping coefficients lane t takes
// edge t.  The quad sums with order-fixed DPP exchanges.  Lanes run the same
// instructions; what differs per lane (quadrant, edge direction) is chosen by
// selects, so the quad never diverges.
//
// Layout (global): u[(((q*(k+1) + a)*(k+1) + b)*ny + iy)*nx + ix]; dual cell
// (ix, iy) is centred on the lower-left vertex of primal cell (ix, iy), so
// primal (i, j) overlaps dual (i..i+1, j..j+1) and dual (i, j) overlaps
// primal (i-1..i, j-1..j).
#include "oecdg_device.h"
#include "oecdg_internal.h"
#include "oecdg_tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace oecdg {

// ---------------------------------------------------------------- fluxes ---

struct FPar2 {
    double a, b, gamma;      // advection velocity (a, b); ideal-gas gamma
};

template <int FLUX> struct Flux2D;

template <> struct Flux2D<OECDG_FLUX_ADVECTION> {
    static constexpr int NC = 1;
    // flux along direction dir (0 = x, 1 = y), selected per lane
    __device__ static inline void f(int dir, const double *w, double *o, const FPar2 &p) {
        o[0] = (dir ? p.b : p.a) * w[0];
    }
    __device__ static inline double speed(int dir, const double *, const FPar2 &p) { return fabs(dir ? p.b : p.a); }
    __device__ static inline bool physical(const double *, const FPar2 &) { return true; }
};

template <> struct Flux2D<OECDG_FLUX_EULER> {
    static constexpr int NC = 4;    // rho, rho u, rho v, E
    __device__ static inline void f(int dir, const double *w, double *o, const FPar2 &p) {
        const double ir = 1.0 / w[0];
        const double u = w[1] * ir, v = w[2] * ir;
        const double pr = (p.gamma - 1.0) * (w[3] - 0.5 * (w[1] * u + w[2] * v));
        const double un = dir ? v : u;
        o[0] = dir ? w[2] : w[1];
        o[1] = w[1] * un + (dir ? 0.0 : pr);
        o[2] = w[2] * un + (dir ? pr : 0.0);
        o[3] = (w[3] + pr) * un;
    }
    __device__ static inline double speed(int dir, const double *w, const FPar2 &p) {
        const double ir = 1.0 / w[0];
        const double u = w[1] * ir, v = w[2] * ir;
        const double pr = (p.gamma - 1.0) * (w[3] - 0.5 * (w[1] * u + w[2] * v));
        return fabs(dir ? v : u) + sqrt(p.gamma * pr * ir);
    }
    __device__ static inline bool physical(const double *w, const FPar2 &p) {
        if (!(w[0] > 0.0)) return false;
        const double pr = (p.gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
        return pr > 0.0;
    }
};

// ---------------------------------------------------------------- tables ---

template <int K>
struct Tab2 {
    static constexpr int K1 = K + 1, Q = K + 1, NSP = 2 * K + 4;
    double w[Q];                  // Gauss-Legendre weights on [-1, 1]
    double own[K1][2][Q][K1];     // [d][half][g][n]: P_n^(d) at node g of the half, own coordinate
    double nb[K1][2][Q][K1];      // the same point in the overlapping cell's coordinate (+1 / -1)
    double e1[K1][K1];            // [d][n]: P_n^(d)(1)
    double e0[K1][K1];            // [d][n]: P_n^(d)(0)
    double sp[NSP][K1];           // P_n at the sigma sample points (-1, half nodes, +1)
    double cdel[K1];              // (2m+1) / ((2K-1) m!)
};

template <int K>
constexpr Tab2<K> make_tab2() {
    Tab2<K> t{};
    constexpr int K1 = K + 1, Q = K + 1;
    constexpr auto g = ct::gauss<Q>();
    for (int i = 0; i < Q; ++i) t.w[i] = g.w[i];
    for (int d = 0; d < K1; ++d)
        for (int hf = 0; hf < 2; ++hf)
            for (int i = 0; i < Q; ++i) {
                const double xi = hf == 0 ? 0.5 * (g.s[i] - 1.0) : 0.5 * (g.s[i] + 1.0);
                const double xn = hf == 0 ? xi + 1.0 : xi - 1.0;
                for (int n = 0; n < K1; ++n) {
                    t.own[d][hf][i][n] = ct::legd(n, d, xi);
                    t.nb[d][hf][i][n] = ct::legd(n, d, xn);
                }
            }
    for (int d = 0; d < K1; ++d)
        for (int n = 0; n < K1; ++n) {
            t.e1[d][n] = ct::legd(n, d, 1.0);
            t.e0[d][n] = ct::legd(n, d, 0.0);
        }
    double pts[2 * K + 4] = {};
    pts[0] = -1.0;
    for (int i = 0; i < Q; ++i) pts[1 + i] = 0.5 * (g.s[i] - 1.0);
    for (int i = 0; i < Q; ++i) pts[1 + Q + i] = 0.5 * (g.s[i] + 1.0);
    pts[2 * K + 3] = 1.0;
    for (int j = 0; j < 2 * K + 4; ++j)
        for (int n = 0; n < K1; ++n) t.sp[j][n] = ct::leg(n, pts[j]);
    double fact = 1.0;
    for (int m = 0; m < K1; ++m) {
        if (m > 1) fact *= m;
        t.cdel[m] = K > 0 ? (2.0 * m + 1.0) / ((2.0 * K - 1.0) * fact) : 0.0;
    }
    return t;
}

// ------------------------------------------------------- device structs ---

// Global scalars of the current stage (written by k_reduce2d).
struct Stats2 {
    double avg[2][4], sig[2][4];  // per mesh and component
    double bx, by;                // largest x / y wave speeds at cell averages (both meshes)
    double t;                     // start time of the current step
    double tau, tau_max;          // the current step
    double tau_damp;              // tau of the OE step applied to the next tile kernel's input
    long long nexec;              // completed steps
    int done, pending, last, bad; // bad: no admissible time step
};

enum { M2_STAGE = 0, M2_FINAL = 1 };
enum { R2_STEP = 0, R2_STAGE = 1, R2_FINAL = 2, R2_SINGLE = 3, R2_STATS = 4 };

struct Stage2Args {
    int nx, ny, ntx, nty;
    long long plane;              // nx * ny
    double hx, hy;
    FPar2 fp;
    const double *inC, *inD;      // tile input (pre-damping, or damped when damp == 0)
    double *outC, *outD;          // stage output (undamped) or damped state (final mode)
    double *UC, *UD;              // damped u^n: written at stage 0 (write_u), read at stages 1, 2
    double *part;                 // [row][tile] partial statistics (k_delta2d)
    double *numC, *numD;          // damping numerators [m*NC + q][ny][nx]: written by k_delta2d, read by k_stage2d
    double *AC, *AD;              // classical RK4: weighted sum of the damped inputs of stages 1 and 2
    const Stats2 *st;
    int *err;                     // [0] non-finite, [1] non-physical, [2] no admissible step
    int l, mode, damp, write_u;
    RKStage rs;                   // c/d coefficients of stage l of the RK method (eq:RKCDG)
};

// Stage output of eq:RKCDG from the damped input s0, its rate Lv and (l > 0)
// the damped u^n un and the accumulated earlier stages acc (classical RK4):
//   c_{l0} u^n [+ acc] + c_{ll} s0 + tau d_{ll} L(s0)
__device__ inline double rk_out(const RKStage &rs, int l, double s0, double Lv, double tau, double un, double acc) {
    const double v = fma(tau * rs.d, Lv, rs.cw * s0);
    if (l == 0) return v;
    return (rs.acc_read ? rs.cn * un + acc : rs.cn * un) + v;
}

struct Red2Args {
    const double *part;
    int ntiles, mode;
    long long ncell;
    double t_end, dt_fixed, cfl, hx, hy;
    double tau_o, taumax_o;       // single-stage call
    Stats2 *st;
    int *err;
};

template <int NC> __host__ __device__ constexpr int nrow2() { return 2 * NC * 3 + 2; }
__host__ __device__ constexpr int row2(int nc, int mesh, int q, int kind) { return (mesh * nc + q) * 3 + kind; }

// ------------------------------------------------------------ helpers ---

// Sum over the four lanes of a quad; every lane gets ((l0 + l1) + (l2 + l3)).
__device__ inline double quad_sum(double v) {
    v += dpp_all<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_all<0x4E>(v);          // quad_perm [2,3,0,1]
    return v;
}

__device__ inline double quad_max(double v) {
    v = fmax(v, dpp_all<0xB1>(v));
    v = fmax(v, dpp_all<0x4E>(v));
    return v;
}

// 1/x from the hardware estimate and two Newton steps (within an ulp or so of
// the correctly rounded quotient; the flux divisions do not need the full
// IEEE division sequence).
__device__ inline double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ inline int wrap_idx(int i, int n, bool small) {
    if (small) return ((i % n) + n) % n;
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// (-1)^(n+d) P_n^(d)(1) = P_n^(d)(-1)
__device__ inline double edge_val(double v1, int n, int d, int side) { return (side || !((n + d) & 1)) ? v1 : -v1; }

// ---------------------------------------------------------- tile kernels ---

// Tile of primal cells [i0, i0+TX) x [j0, j0+TY) and the dual cells with the
// same indices; a band of consecutive tiles per XCD (xcd_tile).
__device__ inline int tile_of_block(int nt) { return xcd_tile(blockIdx.x, nt); }

// Both meshes' state of a tile with a one-cell halo into LDS:
// tile[(mesh*NE + entry)*NCELL + ly*W + lx], global cell (i0-1+lx, j0-1+ly).
// A thread keeps one cell of the tile (its wrapped global index computed
// once) and walks the rows (mesh, entry) in steps of NT / NCELL, so that each
// load costs a pointer select and one multiply-add.
template <int NE, int TX, int TY, int NT>
__device__ inline void stage_tile2d(double *tile, const double *inC, const double *inD, int i0, int j0, int nx,
                                    int ny, long long plane) {
    constexpr int W = TX + 2, H = TY + 2, NCELL = W * H, NROW = 2 * NE;
    constexpr int RPT = NT / NCELL, NIT = (NROW + RPT - 1) / RPT;    // rows per pass, passes
    static_assert(RPT >= 1, "one pass covers every cell of the tile");
    const int tid = threadIdx.x;
    if (tid >= RPT * NCELL) return;
    const int cell = tid % NCELL, r0 = tid / NCELL;
    const bool small = nx < W || ny < H;
    const int gx = wrap_idx(i0 - 1 + cell % W, nx, small);
    const int gy = wrap_idx(j0 - 1 + cell / W, ny, small);
    const long long g = (long long)gy * nx + gx;
    double v[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int r = min(r0 + i * RPT, NROW - 1);                   // past the last row: a valid duplicate
        v[i] = (r < NE ? inC + r * plane : inD + (r - NE) * plane)[g];
    }
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int r = r0 + i * RPT;
        if (r < NROW) tile[r * NCELL + cell] = v[i];
    }
}

// Stage kernel: OE step of the previous stage on the staged input (from the
// damping numerators of k_delta2d and sigma), then the operator of eq:2D_H
// and the RK combination on the owned cells (stage mode), or only the
// damped owned cells (final mode).
// PK: the total-degree space P^K.  Modes with a + b > K are zero in every
// state, so the unrolled loops skip them at compile time (kept()).
template <int K, bool PK>
__device__ constexpr bool kept(int a, int b) { return !PK || a + b <= K; }

template <int K, int FLUX, int TX, int TY, bool PK>
__global__ __launch_bounds__(8 * TX * TY) void k_stage2d(Stage2Args a) {
    using F = Flux2D<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, Q = K + 1, NE = NC * K1 * K1;
    constexpr int W = TX + 2, H = TY + 2, NCELL = W * H, NT = 8 * TX * TY;
    constexpr int ND1 = (TX + 1) * (TY + 1), NDAMP = 2 * ND1;
    constexpr Tab2<K> tb = make_tab2<K>();
    static_assert(NT % WAVE == 0 && NT <= 1024 && NDAMP <= NT, "one damped cell per thread");
    __shared__ double tile[2 * NE * NCELL];      // [mesh][entry][cell]
    __shared__ double fac[2 * K * NCELL];        // [mesh][j-1][cell]: exp(-tau sum_{m<=j} delta^m)

    const int tid = threadIdx.x, lane4 = tid & 3;
    const int nt = a.ntx * a.nty, tileid = tile_of_block(nt);
    const int i0 = (tileid % a.ntx) * TX, j0 = (tileid / a.ntx) * TY;
    const Stats2 *st = a.st;
    if (a.mode == M2_STAGE && st->done) return;

    // damping factors of the damped set (owned cells and one ring): one
    // thread per cell, delta^m = max_q N^m_q / sigma_q
    double fj[K];
    int fcell = -1, fmesh = 0;
    if (a.damp && tid < NDAMP) {
        fmesh = tid / ND1;
        const int rr = tid % ND1;
        const int lx = rr % (TX + 1) + fmesh, ly = rr / (TX + 1) + fmesh;
        fcell = ly * W + lx;
        const bool small = a.nx < W || a.ny < H;
        const int gx = wrap_idx(i0 - 1 + lx, a.nx, small), gy = wrap_idx(j0 - 1 + ly, a.ny, small);
        const double *N = fmesh == 0 ? a.numC : a.numD;
        const long long g = (long long)gy * a.nx + gx;
        double nv[K1][NC];
#pragma unroll
        for (int m = 0; m < K1; ++m)
#pragma unroll
            for (int q = 0; q < NC; ++q) nv[m][q] = N[(m * NC + q) * a.plane + g];
        const double tau = st->tau_damp;
        double S = 0.0;
#pragma unroll
        for (int m = 0; m < K1; ++m) {
            double dm = 0.0;
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                const double sg = st->sig[fmesh][q];
                dm = fmax(dm, sg != 0.0 ? nv[m][q] / sg : 0.0);
            }
            S += dm;
            if (m >= 1) fj[m - 1] = exp(-tau * S);
        }
    }
    stage_tile2d<NE, TX, TY, NT>(tile, a.inC, a.inD, i0, j0, a.nx, a.ny, a.plane);
    if (a.damp) {
        if (fcell >= 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) fac[(fmesh * K + j) * NCELL + fcell] = fj[j];
        }
        __syncthreads();
        // mode (a, b) != (0, 0) takes the factor of total degree min(a + b, K);
        // a thread keeps one damped cell and walks its entries
        constexpr int RD = NT / NDAMP, NID = (NE + RD - 1) / RD;
        static_assert(RD >= 1, "one pass covers every damped cell");
        if (tid < RD * NDAMP) {
            const int cs = tid % NDAMP, e0 = tid / NDAMP;
            const int mesh = cs / ND1, rr = cs % ND1;
            const int cell = (rr / (TX + 1) + mesh) * W + rr % (TX + 1) + mesh;
            double f[K];
#pragma unroll
            for (int j = 0; j < K; ++j) f[j] = fac[(mesh * K + j) * NCELL + cell];
#pragma unroll
            for (int i = 0; i < NID; ++i) {
                const int ent = e0 + i * RD;
                const int ab = ent % (K1 * K1), deg = ab / K1 + ab % K1;
                if (ent < NE && deg > 0) tile[(mesh * NE + ent) * NCELL + cell] *= f[(deg < K ? deg : K) - 1];
            }
        }
    }
    __syncthreads();

    // ---- owned cells: quad lanes per cell
    const int cs = tid >> 2;
    const int mesh = cs / (TX * TY), rr = cs % (TX * TY);
    const int lx = rr % TX + 1, ly = rr / TX + 1;
    const int cell = ly * W + lx;
    const int gx = i0 + lx - 1, gy = j0 + ly - 1;
    const bool valid = gx < a.nx && gy < a.ny;
    const long long gofs = (long long)gy * a.nx + gx;
    const double *town = tile + mesh * NE * NCELL;

    if (a.mode == M2_FINAL) {
        double *dst = mesh == 0 ? a.outC : a.outD;
        if (valid)
            for (int e = lane4; e < NE; e += 4) dst[e * a.plane + gofs] = town[e * NCELL + cell];
        return;
    }
    if (a.write_u && valid) {
        double *UM = mesh == 0 ? a.UC : a.UD;
        for (int e = lane4; e < NE; e += 4) UM[e * a.plane + gofs] = town[e * NCELL + cell];
    }
    const double *toth = tile + (1 - mesh) * NE * NCELL;
    const double tau = st->tau, itm = 1.0 / st->tau_max;
    const double hx = a.hx, hy = a.hy;
    const double *UM = mesh == 0 ? a.UC : a.UD;
    double *OM = mesh == 0 ? a.outC : a.outD;
    double *AM = mesh == 0 ? a.AC : a.AD;
    bool finite = true;
    if constexpr (NC == 4) {
        // lane q accumulates component q over all quadrants and edges; the
        // quad shares the point values of w so every lane can form its flux
        const int q = lane4;
        double Rq[K1][K1];
#pragma unroll
        for (int i = 0; i < K1; ++i)
#pragma unroll
            for (int j = 0; j < K1; ++j) Rq[i][j] = 0.0;
        const double gm1 = a.fp.gamma - 1.0;
        // coupling and volume, quadrant (sx, sy)
//
        // Quadrant (sx, sy) is evaluated in its mirror image on the upper
        // right quadrant: with P_n(-x) = (-1)^n P_n(x) and the symmetric Gauss
        // rule, mirroring a direction flips the sign of the odd modes of the
        // overlapping cell and of the odd test functions (the even ones for a
        // derivative, and the flux along that direction), so every quadrant
        // uses the same compile-time tables.
#pragma unroll 1
        for (int qd = 0; qd < 4; ++qd) {
            const int sx = qd & 1, sy = qd >> 1;
            const double sgx = sx ? 1.0 : -1.0, sgy = sy ? 1.0 : -1.0;
            const int oc = (ly + sy - mesh) * W + (lx + sx - mesh);
            double d[K1][K1];
#pragma unroll
            for (int c = 0; c < K1; ++c)
#pragma unroll
                for (int e = 0; e < K1; ++e) {
                    if (!kept<K, PK>(c, e)) {
                        d[c][e] = 0.0;
                        continue;
                    }
                    const double x = toth[((q * K1 + c) * K1 + e) * NCELL + oc];
                    const double xs = (c & 1) ? sgx * x : x;
                    d[c][e] = (e & 1) ? sgy * xs : xs;
                }
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                double cx[K1];
#pragma unroll
                for (int e = 0; e < K1; ++e) {
                    double t = 0.0;
#pragma unroll
                    for (int c = 0; c < K1; ++c)
                        if (kept<K, PK>(c, e)) t += d[c][e] * tb.nb[0][1][p][c];
                    cx[e] = t;
                }
                double A[K1], B[K1];
#pragma unroll
                for (int j = 0; j < K1; ++j) A[j] = B[j] = 0.0;
#pragma unroll
                for (int g = 0; g < Q; ++g) {
                    double wq = 0.0;
#pragma unroll
                    for (int e = 0; e < K1; ++e) wq += cx[e] * tb.nb[0][1][g][e];
                    const double w0 = dpp_all<0x00>(wq), w1 = dpp_all<0x55>(wq);
                    const double w2 = dpp_all<0xAA>(wq), w3 = dpp_all<0xFF>(wq);
                    const double ir = rcp_nr(w0), u = w1 * ir, v = w2 * ir;
                    const double pr = gm1 * (w3 - 0.5 * (w1 * u + w2 * v));
                    const double base = q == 3 ? w3 + pr : wq;
                    const double f1 = base * u + (q == 1 ? pr : 0.0);
                    const double f2 = sgy * (base * v + (q == 2 ? pr : 0.0));
#pragma unroll
                    for (int j = 0; j < K1; ++j) {
                        A[j] += tb.w[g] * (wq * itm * tb.own[0][1][g][j] + (2.0 / hy) * f2 * tb.own[1][1][g][j]);
                        B[j] += tb.w[g] * f1 * tb.own[0][1][g][j];
                    }
                }
                double Ax[K1], Bx[K1];
#pragma unroll
                for (int j = 0; j < K1; ++j) {
                    if (j & 1) A[j] *= sgy, B[j] *= sgy;
                    Ax[j] = sgx * A[j];
                    Bx[j] = sgx * B[j];
                }
                const double wp = hx * hy / 16.0 * tb.w[p];
#pragma unroll
                for (int i = 0; i < K1; ++i)
#pragma unroll
                    for (int j = 0; j < K1; ++j)
                        if (kept<K, PK>(i, j))
                            Rq[i][j] += wp * (tb.own[0][1][p][i] * ((i & 1) ? Ax[j] : A[j]) +
                                              (2.0 / hx) * tb.own[1][1][p][i] * ((i & 1) ? B[j] : Bx[j]));
            }
        }
        // edges: (dir, side) = W, E (f_1 on vertical centre lines), S, N (f_2)
#pragma unroll 1
        for (int ed = 0; ed < 4; ++ed) {
            const int dir = ed >> 1, side = ed & 1;
            const double ht = dir ? hx : hy, sgn = side ? 1.0 : -1.0;
            double Y[K1];
#pragma unroll
            for (int t = 0; t < K1; ++t) Y[t] = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ox = (dir ? lx + h : lx + side) - mesh, oy = (dir ? ly + side : ly + h) - mesh;
                const int oc = oy * W + ox;
                double r[K1];
#pragma unroll
                for (int t = 0; t < K1; ++t) {
                    double sum = 0.0;
#pragma unroll
                    for (int n = 0; n < K1; ++n) {
                        if (!kept<K, PK>(t, n)) continue;
                        const int ent = dir ? (q * K1 + t) * K1 + n : (q * K1 + n) * K1 + t;
                        sum += toth[ent * NCELL + oc] * tb.e0[0][n];
                    }
                    r[t] = sum;
                }
#pragma unroll
                for (int g = 0; g < Q; ++g) {
                    double wq = 0.0;
#pragma unroll
                    for (int t = 0; t < K1; ++t) wq += r[t] * tb.nb[0][h][g][t];
                    const double w0 = dpp_all<0x00>(wq), w1 = dpp_all<0x55>(wq);
                    const double w2 = dpp_all<0xAA>(wq), w3 = dpp_all<0xFF>(wq);
                    const double ir = rcp_nr(w0), un = (dir ? w2 : w1) * ir;
                    const double pr = gm1 * (w3 - 0.5 * (w1 * w1 + w2 * w2) * ir);
                    const double base = q == 3 ? w3 + pr : wq;
                    const double fn = base * un + (q == 1 + dir ? pr : 0.0);
#pragma unroll
                    for (int t = 0; t < K1; ++t) Y[t] += tb.w[g] * fn * tb.own[0][h][g][t];
                }
            }
#pragma unroll
            for (int n = 0; n < K1; ++n)
#pragma unroll
                for (int t = 0; t < K1; ++t) {
                    if (!kept<K, PK>(n, t)) continue;
                    const double x = sgn * 0.25 * ht * edge_val(1.0, n, 0, side) * Y[t];
                    if (dir) Rq[t][n] -= x;
                    else Rq[n][t] -= x;
                }
        }
        // own part of the coupling, mass inverse, RK combination
#pragma unroll
        for (int i = 0; i < K1; ++i)
#pragma unroll
            for (int j = 0; j < K1; ++j) {
                const int e = (q * K1 + i) * K1 + j;
                const double mass = hx * hy / ((2.0 * i + 1.0) * (2.0 * j + 1.0));
                const double s0 = town[e * NCELL + cell];
                const double Lv = (Rq[i][j] - mass * itm * s0) / mass;
                const double un = (a.l > 0 && valid) ? UM[e * a.plane + gofs] : 0.0;
                const double ac = (a.rs.acc_read && valid) ? AM[e * a.plane + gofs] : 0.0;
                double o = rk_out(a.rs, a.l, s0, Lv, tau, un, ac);
                if (!kept<K, PK>(i, j)) o = 0.0;
                finite = finite && isfinite(o);
                if (valid) {
                    OM[e * a.plane + gofs] = o;
                    if (a.rs.ca != 0.0) {     // classical RK4: this stage's damped input joins the sum
                        double *p = AM + e * a.plane + gofs;
                        *p = a.rs.acc_first ? a.rs.ca * s0 : fma(a.rs.ca, s0, *p);
                    }
                }
            }
    } else {
        // one component: lane t takes quadrant t and edge t, the quad sums
        double R[NC][K1][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int i = 0; i < K1; ++i)
#pragma unroll
                for (int j = 0; j < K1; ++j) R[q][i][j] = 0.0;
        {
            const int sx = lane4 & 1, sy = lane4 >> 1;
            const int oc = (ly + sy - mesh) * W + (lx + sx - mesh);
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                double cx[NC][K1];
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int d = 0; d < K1; ++d) {
                        double sum = 0.0;
#pragma unroll
                        for (int c = 0; c < K1; ++c)
                            if (kept<K, PK>(c, d))
                                sum += toth[((q * K1 + c) * K1 + d) * NCELL + oc] *
                                       (sx ? tb.nb[0][1][p][c] : tb.nb[0][0][p][c]);
                        cx[q][d] = sum;
                    }
                double A[NC][K1], B[NC][K1];
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int j = 0; j < K1; ++j) A[q][j] = B[q][j] = 0.0;
#pragma unroll
                for (int g = 0; g < Q; ++g) {
                    double w[NC], f1[NC], f2[NC];
#pragma unroll
                    for (int q = 0; q < NC; ++q) {
                        double sum = 0.0;
#pragma unroll
                        for (int d = 0; d < K1; ++d) sum += cx[q][d] * (sy ? tb.nb[0][1][g][d] : tb.nb[0][0][g][d]);
                        w[q] = sum;
                    }
                    F::f(0, w, f1, a.fp);
                    F::f(1, w, f2, a.fp);
#pragma unroll
                    for (int q = 0; q < NC; ++q)
#pragma unroll
                        for (int j = 0; j < K1; ++j) {
                            const double pb = sy ? tb.own[0][1][g][j] : tb.own[0][0][g][j];
                            const double dpb = sy ? tb.own[1][1][g][j] : tb.own[1][0][g][j];
                            A[q][j] += tb.w[g] * (w[q] * itm * pb + (2.0 / hy) * f2[q] * dpb);
                            B[q][j] += tb.w[g] * f1[q] * pb;
                        }
                }
                const double wp = hx * hy / 16.0 * tb.w[p];
#pragma unroll
                for (int i = 0; i < K1; ++i) {
                    const double pa = sx ? tb.own[0][1][p][i] : tb.own[0][0][p][i];
                    const double dpa = sx ? tb.own[1][1][p][i] : tb.own[1][0][p][i];
#pragma unroll
                    for (int q = 0; q < NC; ++q)
#pragma unroll
                        for (int j = 0; j < K1; ++j)
                            if (kept<K, PK>(i, j)) R[q][i][j] += wp * (pa * A[q][j] + (2.0 / hx) * dpa * B[q][j]);
                }
            }
        }
        {
            const int dir = lane4 >> 1, side = lane4 & 1;
            const double ht = dir ? hx : hy, sgn = side ? 1.0 : -1.0;
            double Y[NC][K1];
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int t = 0; t < K1; ++t) Y[q][t] = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ox = (dir ? lx + h : lx + side) - mesh, oy = (dir ? ly + side : ly + h) - mesh;
                const int oc = oy * W + ox;
                double r[NC][K1];
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int t = 0; t < K1; ++t) {
                        double sum = 0.0;
#pragma unroll
                        for (int n = 0; n < K1; ++n) {
                            if (!kept<K, PK>(t, n)) continue;
                            const int ent = dir ? (q * K1 + t) * K1 + n : (q * K1 + n) * K1 + t;
                            sum += toth[ent * NCELL + oc] * tb.e0[0][n];
                        }
                        r[q][t] = sum;
                    }
#pragma unroll
                for (int g = 0; g < Q; ++g) {
                    double w[NC], fn[NC];
#pragma unroll
                    for (int q = 0; q < NC; ++q) {
                        double sum = 0.0;
#pragma unroll
                        for (int t = 0; t < K1; ++t) sum += r[q][t] * tb.nb[0][h][g][t];
                        w[q] = sum;
                    }
                    F::f(dir, w, fn, a.fp);
#pragma unroll
                    for (int q = 0; q < NC; ++q)
#pragma unroll
                        for (int t = 0; t < K1; ++t) Y[q][t] += tb.w[g] * fn[q] * tb.own[0][h][g][t];
                }
            }
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int i = 0; i < K1; ++i)
#pragma unroll
                    for (int j = 0; j < K1; ++j) {
                        if (!kept<K, PK>(i, j)) continue;
                        const double x_ij = sgn * 0.25 * ht * edge_val(1.0, i, 0, side) * Y[q][j];
                        const double x_ji = sgn * 0.25 * ht * edge_val(1.0, j, 0, side) * Y[q][i];
                        R[q][i][j] -= dir ? x_ji : x_ij;
                    }
        }
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int i = 0; i < K1; ++i)
#pragma unroll
                for (int j = 0; j < K1; ++j) {
                    const int e = (q * K1 + i) * K1 + j;
                    if (!kept<K, PK>(i, j)) {
                        if ((e & 3) == lane4 && valid) OM[e * a.plane + gofs] = 0.0;
                        continue;
                    }
                    const double mass = hx * hy / ((2.0 * i + 1.0) * (2.0 * j + 1.0));
                    const double s0 = town[e * NCELL + cell];
                    const double Lv = (quad_sum(R[q][i][j]) - mass * itm * s0) / mass;
                    if ((e & 3) == lane4) {
                        const double un = (a.l > 0 && valid) ? UM[e * a.plane + gofs] : 0.0;
                        const double ac = (a.rs.acc_read && valid) ? AM[e * a.plane + gofs] : 0.0;
                        const double o = rk_out(a.rs, a.l, s0, Lv, tau, un, ac);
                        finite = finite && isfinite(o);
                        if (valid) {
                            OM[e * a.plane + gofs] = o;
                            if (a.rs.ca != 0.0) {
                                double *p = AM + e * a.plane + gofs;
                                *p = a.rs.acc_first ? a.rs.ca * s0 : fma(a.rs.ca, s0, *p);
                            }
                        }
                    }
                }
    }
    if (valid && !finite) a.err[0] = 1;
}

// Damping numerators and statistics of a state (the undamped output of a
// stage, or initial data): per owned cell and component q
//   N^m_q = sum_{e in {W,E,S,N}} beta_{e,K} (2m+1) h_e^(m-1) / ((2k-1) m!)
//           (1/|e|) int_e ( sum_{alpha1+alpha2=m} (d^alpha (u_K - w)_q)^2 )^(1/2) ds
// (delta^m_K = max_q N^m_q / sigma_q once sigma is known, Sec. 2.2), with one
// lane per edge; then the tile's partial statistics (sums of averages, sample
// max / min per component, largest wave speeds) with one lane per component.
template <int K, int FLUX, int TX, int TY, bool PK>
// Two workgroups per CU (4 waves per SIMD; the LDS tile allows no more): the
// register cap spills a few values to scratch, which costs less than running
// one workgroup per CU (6.86 -> 6.32 ms per step on the 1024^2 workload).  At
// k = 3 the LDS tile allows 2 waves per SIMD only, so no register cap.
__global__ __launch_bounds__(8 * TX * TY, K == 3 ? 2 : 4) void k_delta2d(Stage2Args a) {
    using F = Flux2D<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, Q = K + 1, NE = NC * K1 * K1, NSP = 2 * K + 4;
    constexpr int W = TX + 2, NCELL = W * (TY + 2), NT = 8 * TX * TY, NW = NT / WAVE;
    constexpr int NR = nrow2<NC>();
    constexpr Tab2<K> tb = make_tab2<K>();
    __shared__ double tile[2 * NE * NCELL];
    __shared__ double red[NW * NR];

    const int tid = threadIdx.x, lane4 = tid & 3;
    const int nt = a.ntx * a.nty, tileid = tile_of_block(nt);
    const int i0 = (tileid % a.ntx) * TX, j0 = (tileid / a.ntx) * TY;
    if (a.mode == M2_STAGE && a.st->done) return;
    stage_tile2d<NE, TX, TY, NT>(tile, a.inC, a.inD, i0, j0, a.nx, a.ny, a.plane);
    __syncthreads();

    const int cs = tid >> 2;
    const int mesh = cs / (TX * TY), rr = cs % (TX * TY);
    const int lx = rr % TX + 1, ly = rr / TX + 1;
    const int cell = ly * W + lx;
    const int gx = i0 + lx - 1, gy = j0 + ly - 1;
    const bool valid = gx < a.nx && gy < a.ny;
    const long long gofs = (long long)gy * a.nx + gx;
    const double *own = tile + mesh * NE * NCELL, *oth = tile + (1 - mesh) * NE * NCELL;
    double ubar[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) ubar[q] = own[(q * K1 * K1) * NCELL + cell];

    if (a.numC) {
        const int dir = lane4 >> 1, side = lane4 & 1;
        const double hn = dir ? a.hy : a.hx, ht = dir ? a.hx : a.hy;
        const double beta = F::speed(dir, ubar, a.fp);
        int oc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ox = (dir ? lx + h : lx + side) - mesh, oy = (dir ? ly + side : ly + h) - mesh;
            oc[h] = oy * W + ox;
        }
        double* N = mesh == 0 ? a.numC : a.numD;
#pragma unroll 1
        for (int q = 0; q < NC; ++q) {
            // traces restricted to the edge, by normal derivative order: own at
            // the edge (normal coordinate +-1); the other mesh at its centre
            // line (0), one half-edge at a time (each mean[m] still sums the
            // half-edges in order)
            double ro[K1][K1];
#pragma unroll
            for (int dn = 0; dn < K1; ++dn)
#pragma unroll
                for (int t = 0; t < K1; ++t) {
                    double so = 0.0;
#pragma unroll
                    for (int n = 0; n < K1; ++n) {
                        if (!kept<K, PK>(t, n)) continue;
                        const int ent = dir ? (q * K1 + t) * K1 + n : (q * K1 + n) * K1 + t;
                        so += own[ent * NCELL + cell] * edge_val(tb.e1[dn][n], n, dn, side);
                    }
                    ro[dn][t] = so;
                }
            double mean[K1];
#pragma unroll
            for (int m = 0; m < K1; ++m) mean[m] = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double rt[K1][K1];
#pragma unroll
                for (int dn = 0; dn < K1; ++dn)
#pragma unroll
                    for (int t = 0; t < K1; ++t) {
                        double sh = 0.0;
#pragma unroll
                        for (int n = 0; n < K1; ++n) {
                            if (!kept<K, PK>(t, n)) continue;
                            const int ent = dir ? (q * K1 + t) * K1 + n : (q * K1 + n) * K1 + t;
                            sh += oth[ent * NCELL + oc[h]] * tb.e0[dn][n];
                        }
                        rt[dn][t] = sh;
                    }
#pragma unroll
                for (int m = 0; m < K1; ++m)
#pragma unroll
                    for (int g = 0; g < Q; ++g) {
                        double ss = 0.0;
                        double scn = 1.0;
#pragma unroll
                        for (int dn = 0; dn <= m; ++dn) {
                            const int dt = m - dn;
                            double sct = scn;
#pragma unroll
                            for (int j = 0; j < dt; ++j) sct *= 2.0 / ht;
                            double vo = 0.0, vt = 0.0;
#pragma unroll
                            for (int t = 0; t < K1; ++t) {
                                vo += ro[dn][t] * tb.own[dt][h][g][t];
                                vt += rt[dn][t] * tb.nb[dt][h][g][t];
                            }
                            const double d = sct * (vo - vt);
                            ss = m == 0 ? fabs(d) : ss + d * d;
                            scn *= 2.0 / hn;
                        }
                        mean[m] += 0.25 * tb.w[g] * (m == 0 ? ss : sqrt(ss));   // |d| = (d^2)^(1/2) for m = 0
                    }
            }
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                double hm = 1.0;                          // h_e^(m-1)
                if (m == 0) hm = 1.0 / hn;
#pragma unroll
                for (int j = 1; j < m; ++j) hm *= hn;
                const double num = quad_sum(beta * tb.cdel[m] * hm * mean[m]);
                if (valid && lane4 == (m & 3)) N[(m * NC + q) * a.plane + gofs] = num;
            }
        }
    }

    // ---- partial statistics: component cq of this cell, all sample rows for
    // a component lane (Euler), rows i = lane (mod 4) for one component
    // (a wave holds cells of one mesh only, so a thread keeps the rows of its
    // own mesh, (sum, max, min) per component, and the two wave-speed rows)
    constexpr bool LANE_COMP = NC == 4;
    constexpr int NM = 3 * NC;
    const int cq = LANE_COMP ? lane4 : 0;
    double vals[NM + 2];
#pragma unroll
    for (int j = 0; j < NM + 2; ++j) vals[j] = j < NM ? stat_identity(j % 3) : -INFINITY;
    if (valid) {
        double cst[K1][K1];
#pragma unroll
        for (int i = 0; i < K1; ++i)
#pragma unroll
            for (int j = 0; j < K1; ++j) cst[i][j] = kept<K, PK>(i, j) ? own[((cq * K1 + i) * K1 + j) * NCELL + cell] : 0.0;
        double mx = -INFINITY, mn = INFINITY;
#pragma unroll
        for (int i = 0; i < NSP; ++i) {
            if (!LANE_COMP && (i & 3) != lane4) continue;
            double rb[K1];
#pragma unroll
            for (int j = 0; j < K1; ++j) {
                double sum = 0.0;
#pragma unroll
                for (int c = 0; c < K1; ++c)
                    if (kept<K, PK>(c, j)) sum += cst[c][j] * tb.sp[i][c];
                rb[j] = sum;
            }
#pragma unroll
            for (int jj = 0; jj < NSP; ++jj) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < K1; ++j) v += rb[j] * tb.sp[jj][j];
                mx = fmax(mx, v);
                mn = fmin(mn, v);
            }
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (q != cq) continue;
            vals[3 * q] = (LANE_COMP || lane4 == 0) ? cst[0][0] : 0.0;
            vals[3 * q + 1] = mx;
            vals[3 * q + 2] = mn;
        }
        if (lane4 == 0) {
            double ub[NC];                // the cell averages again from LDS: not kept live across the numerators
#pragma unroll
            for (int q = 0; q < NC; ++q) ub[q] = own[(q * K1 * K1) * NCELL + cell];
            vals[NM] = F::speed(0, ub, a.fp);
            vals[NM + 1] = F::speed(1, ub, a.fp);
            if (!F::physical(ub, a.fp)) a.err[1] = 1;
        }
    }
    {
        // the wave's own mesh rows and the wave speeds are reduced; the other
        // mesh's rows are the identity in this wave
        static_assert((4 * TX * TY) % WAVE == 0, "waves do not straddle the meshes");
        const int lane = tid % WAVE, wave = tid / WAVE, wmesh = wave / (4 * TX * TY / WAVE);
#pragma unroll
        for (int j = 0; j < NM + 2; ++j) {
            const int kind = j < NM ? j % 3 : 1;
            const double v = wave_reduce(kind, vals[j]);
            if (lane == WAVE - 1) red[wave * NR + (j < NM ? row2(NC, wmesh, j / 3, j % 3) : 2 * NM + (j - NM))] = v;
        }
        if (lane == WAVE - 1) {
#pragma unroll
            for (int j = 0; j < NM; ++j) red[wave * NR + row2(NC, 1 - wmesh, j / 3, j % 3)] = stat_identity(j % 3);
        }
        __syncthreads();
        if (tid < NR) {
            const int kind = tid < 2 * NC * 3 ? tid % 3 : 1;
            double v = red[tid];
            for (int w2 = 1; w2 < NW; ++w2) v = stat_op(kind, v, red[w2 * NR + tid]);
            a.part[(long long)tid * nt + tileid] = v;
        }
    }
}

// ------------------------------------------------------- reduce kernels ---
// Two levels, both in a fixed order: k_fold2d folds contiguous ranges of
// tiles into one partial per workgroup; k_reduce2d folds those in one
// workgroup and updates the step scalars.

constexpr int RED2_NT = 256;
constexpr int FOLD2_MAXB = 64;

template <int NC>
__global__ __launch_bounds__(RED2_NT) void k_fold2d(const double *part, int ntiles, int per, double *out, int nb) {
    constexpr int NR = nrow2<NC>(), NW = RED2_NT / WAVE;
    __shared__ double red[NW * NR];
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    const int t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = stat_identity(j < 2 * NC * 3 ? j % 3 : 1);
    for (int t = t0 + tid; t < t1; t += RED2_NT)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = stat_op(j < 2 * NC * 3 ? j % 3 : 1, acc[j], part[(long long)j * ntiles + t]);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const double v = wave_reduce(j < 2 * NC * 3 ? j % 3 : 1, acc[j]);
        if (lane == WAVE - 1) red[wave * NR + j] = v;
    }
    __syncthreads();
    if (tid < NR) {
        const int kind = tid < 2 * NC * 3 ? tid % 3 : 1;
        double v = red[tid];
        for (int w = 1; w < NW; ++w) v = stat_op(kind, v, red[w * NR + tid]);
        out[(long long)tid * nb + blockIdx.x] = v;
    }
}

template <int NC>
__global__ __launch_bounds__(RED2_NT) void k_reduce2d(Red2Args r) {
    constexpr int NR = nrow2<NC>(), NW = RED2_NT / WAVE;
    __shared__ double red[NW * NR];
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    Stats2 *st = r.st;
    if ((r.mode == R2_STAGE) && st->done) return;
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = stat_identity(j < 2 * NC * 3 ? j % 3 : 1);
    for (int t = tid; t < r.ntiles; t += RED2_NT)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = stat_op(j < 2 * NC * 3 ? j % 3 : 1, acc[j], r.part[(long long)j * r.ntiles + t]);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const double v = wave_reduce(j < 2 * NC * 3 ? j % 3 : 1, acc[j]);
        if (lane == WAVE - 1) red[wave * NR + j] = v;
    }
    __syncthreads();
    if (tid != 0) return;
    double tot[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kind = j < 2 * NC * 3 ? j % 3 : 1;
        double v = red[j];
        for (int w = 1; w < NW; ++w) v = stat_op(kind, v, red[w * NR + j]);
        tot[j] = v;
    }
    for (int mesh = 0; mesh < 2; ++mesh)
        for (int q = 0; q < NC; ++q) {
            const double avg = tot[row2(NC, mesh, q, 0)] / (double)r.ncell;
            st->avg[mesh][q] = avg;
            st->sig[mesh][q] = fmax(tot[row2(NC, mesh, q, 1)] - avg, avg - tot[row2(NC, mesh, q, 2)]);
        }
    st->bx = tot[2 * NC * 3];
    st->by = tot[2 * NC * 3 + 1];
    if (r.mode == R2_STEP || r.mode == R2_FINAL) {
        if (st->pending) {                       // complete the previous step
            st->t = st->last ? r.t_end : st->t + st->tau;
            st->nexec += 1;
            st->pending = 0;
        }
        st->tau_damp = st->tau;
    }
    if (r.mode == R2_STEP) {
        if (!(st->t < r.t_end)) {
            st->done = 1;
            return;
        }
        double tm = r.dt_fixed;
        if (!(tm > 0.0)) {
            const double rate = st->bx / r.hx + st->by / r.hy;
            if (!(rate > 0.0) || !isfinite(rate)) {
                st->done = 1;
                st->bad = 1;
                r.err[2] = 1;
                return;
            }
            tm = r.cfl / rate;
        }
        double tau = tm;
        int last = 0;
        if (st->t + tau >= r.t_end) {
            tau = r.t_end - st->t;
            last = 1;
        }
        st->tau = tau;
        st->tau_max = tm;
        st->last = last;
        st->done = 0;
        st->pending = 1;
    } else if (r.mode == R2_STAGE) {
        st->tau_damp = st->tau;
    } else if (r.mode == R2_SINGLE) {
        st->tau = r.tau_o;
        st->tau_max = r.taumax_o;
        st->tau_damp = r.tau_o;
        st->done = 0;
    }
}

// ------------------------------------------------------------ host side ---

namespace {

// Tiles of 8 x 8 primal cells for k = 1, 2; 4 x 4 for k = 3, whose 64
// coefficients per cell would make an 8 x 8 tile with its halo overflow LDS.
template <int K> struct Tile2 {
    static constexpr int TX = K == 3 ? 4 : 8, TY = K == 3 ? 4 : 8;
};
constexpr int tile2(int k) { return k == 3 ? 4 : 8; }

template <int K, int FLUX, bool PK>
void *stage2d_fn(bool delta) {
    constexpr int TX = Tile2<K>::TX, TY = Tile2<K>::TY;
    return delta ? (void *)k_delta2d<K, FLUX, TX, TY, PK> : (void *)k_stage2d<K, FLUX, TX, TY, PK>;
}

template <int K>
void *pick2_k(int flux, bool pk, bool delta) {
    if (flux == OECDG_FLUX_EULER) return pk ? stage2d_fn<K, OECDG_FLUX_EULER, true>(delta) : stage2d_fn<K, OECDG_FLUX_EULER, false>(delta);
    return pk ? stage2d_fn<K, OECDG_FLUX_ADVECTION, true>(delta) : stage2d_fn<K, OECDG_FLUX_ADVECTION, false>(delta);
}

void *pick2(int k, int flux, bool pk, bool delta) {
    switch (k) {
    case 1: return pick2_k<1>(flux, pk, delta);
    case 2: return pick2_k<2>(flux, pk, delta);
    default: return pick2_k<3>(flux, pk, delta);
    }
}

struct Ext2D {
    int k, nc, flux, oe;
    int pk;                      // total-degree space P^k
    int tx, ty;                  // primal cells per tile and direction
    int rk, ns;                  // RK method (rk_stage) and its stages per step
    int nx, ny, ntx, nty, ntiles;
    double hx, hy, cfl;
    FPar2 fp;
    long long S1;                // doubles of one mesh
    long long SN;                // damping numerators of one mesh: (k+1) nc nx ny
    double *B[2] = {nullptr, nullptr};      // stage states, both meshes each
    double *num[2] = {nullptr, nullptr};    // damping numerators of B[i], both meshes each
    double *U = nullptr;
    double *A = nullptr;         // classical RK4: accumulated damped inputs of stages 1 and 2 (both meshes)
    double *part[2] = {nullptr, nullptr};
    double *fold = nullptr;      // [row][nfold] first-level partials
    int nfold = 1, fold_per = 1;
    Stats2 *st = nullptr;
    Stats2 *st_h = nullptr;      // pinned
    int *err = nullptr, *err_h = nullptr;
};

Ext2D *ext(oecdg_handle *h) { return static_cast<Ext2D *>(handle_ext2d(h)); }

#define HIPCHK2(h, expr)                                                                                      \
    do {                                                                                                      \
        hipError_t e_ = (expr);                                                                               \
        if (e_ != hipSuccess) return handle_fail((h), OECDG_EHIP, hipGetErrorString(e_));                     \
    } while (0)

hipError_t launch_tile(void *fn, const Ext2D &x, const Stage2Args &a, hipStream_t s) {
    Stage2Args copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(x.ntiles), dim3(8 * x.tx * x.ty), args, 0, s);
}

hipError_t launch_stage2d(const Ext2D &x, const Stage2Args &a, hipStream_t s) {
    return launch_tile(pick2(x.k, x.flux, x.pk, false), x, a, s);
}

hipError_t launch_delta2d(const Ext2D &x, const Stage2Args &a, hipStream_t s) {
    return launch_tile(pick2(x.k, x.flux, x.pk, true), x, a, s);
}

// Fold r.part (per-tile partials) into the global scalars: first level into
// x.fold, then the single-workgroup finish.
hipError_t launch_reduce2d(const Ext2D &x, const Red2Args &r, hipStream_t s) {
    const double *part = r.part;
    int n = r.ntiles, per = x.fold_per, nb = x.nfold;
    double *out = x.fold;
    void *args1[] = {&part, &n, &per, &out, &nb};
    void *fold = x.nc == 4 ? (void *)k_fold2d<4> : (void *)k_fold2d<1>;
    hipError_t e = hipLaunchKernel(fold, dim3(nb), dim3(RED2_NT), args1, 0, s);
    if (e != hipSuccess) return e;
    void *fn = x.nc == 4 ? (void *)k_reduce2d<4> : (void *)k_reduce2d<1>;
    Red2Args copy = r;
    copy.part = x.fold;
    copy.ntiles = nb;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(1), dim3(RED2_NT), args, 0, s);
}

Stage2Args stage_args(const Ext2D &x) {
    Stage2Args a;
    memset(&a, 0, sizeof(a));
    a.nx = x.nx;
    a.ny = x.ny;
    a.ntx = x.ntx;
    a.nty = x.nty;
    a.plane = (long long)x.nx * x.ny;
    a.hx = x.hx;
    a.hy = x.hy;
    a.fp = x.fp;
    a.st = x.st;
    a.err = x.err;
    if (x.A) {
        a.AC = x.A;
        a.AD = x.A + x.S1;
    }
    a.rs = rk_stage(x.rk, 0);
    return a;
}

Red2Args red_args(const Ext2D &x, const double *part, int mode) {
    Red2Args r;
    memset(&r, 0, sizeof(r));
    r.part = part;
    r.ntiles = x.ntiles;
    r.mode = mode;
    r.ncell = (long long)x.nx * x.ny;
    r.t_end = INFINITY;
    r.cfl = x.cfl;
    r.hx = x.hx;
    r.hy = x.hy;
    r.st = x.st;
    r.err = x.err;
    return r;
}

// Damping numerators (when OE is on) and partial statistics of a state into
// num[i] / part[i]; mode M2_STAGE skips the work once the run is done.
hipError_t delta_of(const Ext2D &x, const double *uC, const double *uD, int i, int mode, hipStream_t s) {
    Stage2Args a = stage_args(x);
    a.mode = mode;
    a.inC = uC;
    a.inD = uD;
    a.part = x.part[i];
    if (x.oe && x.k > 0) {
        a.numC = x.num[i];
        a.numD = x.num[i] + x.SN;
    }
    return launch_delta2d(x, a, s);
}

int check2d(oecdg_handle *h, const Ext2D &x) {
    hipStream_t s = handle_stream(h);
    HIPCHK2(h, hipMemcpyAsync(x.err_h, x.err, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK2(h, hipStreamSynchronize(s));
    if (x.err_h[2]) return handle_fail(h, OECDG_ENONFINITE, "no admissible time step (wave speed zero or not finite)");
    if (x.err_h[0]) return handle_fail(h, OECDG_ENONFINITE, "non-finite coefficient produced");
    if (x.err_h[1]) return handle_fail(h, OECDG_ENONPHYSICAL, "non-positive density or pressure at a cell average");
    return OECDG_OK;
}

int reset2d(oecdg_handle *h, Ext2D &x) {
    hipStream_t s = handle_stream(h);
    memset(x.st_h, 0, sizeof(Stats2));
    HIPCHK2(h, hipMemcpyAsync(x.st, x.st_h, sizeof(Stats2), hipMemcpyHostToDevice, s));
    HIPCHK2(h, hipMemsetAsync(x.err, 0, 4 * sizeof(int), s));
    return OECDG_OK;
}

}  // namespace

int create_2d(oecdg_handle *h, const oecdg_desc *d) {
    Ext2D *x = new (std::nothrow) Ext2D();
    if (!x) return OECDG_ENOMEM;
    handle_ext2d(h) = x;
    x->k = d->k;
    x->flux = d->flux;
    x->nc = d->flux == OECDG_FLUX_EULER ? 4 : 1;
    x->oe = d->oe;
    x->pk = d->space == 1;
    x->nx = (int)d->nx;
    x->ny = (int)d->ny;
    x->tx = x->ty = tile2(x->k);
    x->rk = d->rk == 0 ? 3 : d->rk;
    x->ns = rk_stages(x->rk);
    x->ntx = (x->nx + x->tx - 1) / x->tx;
    x->nty = (x->ny + x->ty - 1) / x->ty;
    x->ntiles = x->ntx * x->nty;
    x->hx = (d->xhi - d->xlo) / d->nx;
    x->hy = (d->yhi - d->ylo) / d->ny;
    x->cfl = d->cfl;
    x->fp.a = d->flux_param[0];
    x->fp.b = d->flux_param[1];
    x->fp.gamma = d->flux_param[0];
    x->S1 = (long long)x->nc * (x->k + 1) * (x->k + 1) * x->nx * x->ny;
    x->SN = (long long)x->nc * (x->k + 1) * x->nx * x->ny;
    const size_t nrow = x->nc == 4 ? nrow2<4>() : nrow2<1>();
    for (int i = 0; i < 2; ++i) {
        HIPCHK2(h, hipMalloc(&x->B[i], sizeof(double) * 2 * x->S1));
        HIPCHK2(h, hipMalloc(&x->num[i], sizeof(double) * 2 * x->SN));
        HIPCHK2(h, hipMalloc(&x->part[i], sizeof(double) * nrow * x->ntiles));
    }
    HIPCHK2(h, hipMalloc(&x->U, sizeof(double) * 2 * x->S1));
    if (x->rk == 4) HIPCHK2(h, hipMalloc(&x->A, sizeof(double) * 2 * x->S1));
    x->nfold = x->ntiles < FOLD2_MAXB ? x->ntiles : FOLD2_MAXB;
    x->fold_per = (x->ntiles + x->nfold - 1) / x->nfold;
    HIPCHK2(h, hipMalloc(&x->fold, sizeof(double) * nrow * x->nfold));
    HIPCHK2(h, hipMalloc(&x->st, sizeof(Stats2)));
    HIPCHK2(h, hipHostMalloc((void **)&x->st_h, sizeof(Stats2), hipHostMallocDefault));
    HIPCHK2(h, hipMalloc(&x->err, 4 * sizeof(int)));
    HIPCHK2(h, hipHostMalloc((void **)&x->err_h, 4 * sizeof(int), hipHostMallocDefault));
    return OECDG_OK;
}

void destroy_2d(oecdg_handle *h) {
    Ext2D *x = ext(h);
    if (!x) return;
    for (int i = 0; i < 2; ++i) {
        if (x->B[i]) (void)hipFree(x->B[i]);
        if (x->num[i]) (void)hipFree(x->num[i]);
        if (x->part[i]) (void)hipFree(x->part[i]);
    }
    if (x->U) (void)hipFree(x->U);
    if (x->A) (void)hipFree(x->A);
    if (x->fold) (void)hipFree(x->fold);
    if (x->st) (void)hipFree(x->st);
    if (x->st_h) (void)hipHostFree(x->st_h);
    if (x->err) (void)hipFree(x->err);
    if (x->err_h) (void)hipHostFree(x->err_h);
    delete x;
    handle_ext2d(h) = nullptr;
}

int dt_2d(oecdg_handle *h, const double *uC, const double *uD, double *dt_out) {
    Ext2D &x = *ext(h);
    hipStream_t s = handle_stream(h);
    int rc = reset2d(h, x);
    if (rc != OECDG_OK) return rc;
    HIPCHK2(h, delta_of(x, uC, uD, 0, M2_FINAL, s));
    HIPCHK2(h, launch_reduce2d(x, red_args(x, x.part[0], R2_STATS), s));
    HIPCHK2(h, hipMemcpyAsync(x.st_h, x.st, sizeof(Stats2), hipMemcpyDeviceToHost, s));
    HIPCHK2(h, hipStreamSynchronize(s));
    const double rate = x.st_h->bx / x.hx + x.st_h->by / x.hy;
    if (!(rate > 0.0) || !std::isfinite(rate)) return handle_fail(h, OECDG_ENONFINITE, "wave speed is zero or not finite");
    *dt_out = x.cfl / rate;
    return OECDG_OK;
}

int stage_2d(oecdg_handle *h, int stage, double dt, double tau_max, const double *uCn, const double *uDn,
             const double *uCl, const double *uDl, double *uCo, double *uDo) {
    Ext2D &x = *ext(h);
    hipStream_t s = handle_stream(h);
    int rc = reset2d(h, x);
    if (rc != OECDG_OK) return rc;
    // the step scalars only (the partials read here are discarded by mode)
    Red2Args r = red_args(x, x.part[1], R2_SINGLE);
    r.tau_o = dt;
    r.taumax_o = tau_max;
    HIPCHK2(h, hipMemsetAsync(x.part[1], 0, sizeof(double) * (x.nc == 4 ? nrow2<4>() : nrow2<1>()) * x.ntiles, s));
    HIPCHK2(h, launch_reduce2d(x, r, s));
    Stage2Args a = stage_args(x);
    a.mode = M2_STAGE;
    a.l = stage;
    a.rs = rk_stage(x.rk, stage);
    a.damp = 0;
    a.write_u = 0;
    a.inC = stage == 0 ? uCn : uCl;
    a.inD = stage == 0 ? uDn : uDl;
    a.UC = const_cast<double *>(uCn);
    a.UD = const_cast<double *>(uDn);
    a.outC = x.B[0];
    a.outD = x.B[0] + x.S1;
    HIPCHK2(h, launch_stage2d(x, a, s));
    HIPCHK2(h, delta_of(x, x.B[0], x.B[0] + x.S1, 0, M2_FINAL, s));
    HIPCHK2(h, launch_reduce2d(x, red_args(x, x.part[0], R2_STAGE), s));
    Stage2Args f = stage_args(x);
    f.mode = M2_FINAL;
    f.damp = x.oe && x.k > 0;
    f.inC = x.B[0];
    f.inD = x.B[0] + x.S1;
    f.numC = x.num[0];
    f.numD = x.num[0] + x.SN;
    f.outC = uCo;
    f.outD = uDo;
    HIPCHK2(h, launch_stage2d(x, f, s));
    return check2d(h, x);
}

int run_2d(oecdg_handle *h, double *uC, double *uD, double t_end, int64_t nsteps, double dt_fixed, double *t_out,
           int64_t *steps_out) {
    Ext2D &x = *ext(h);
    hipStream_t s = handle_stream(h);
    if (nsteps < 0 && !std::isfinite(t_end)) return handle_fail(h, OECDG_EINVAL, "give a finite t_end or nsteps >= 0");
    int rc = reset2d(h, x);
    if (rc != OECDG_OK) return rc;
    HIPCHK2(h, hipMemcpyAsync(x.B[0], uC, sizeof(double) * x.S1, hipMemcpyDeviceToDevice, s));
    HIPCHK2(h, hipMemcpyAsync(x.B[0] + x.S1, uD, sizeof(double) * x.S1, hipMemcpyDeviceToDevice, s));
    if (x.pk) {   // P^k: the modes of total degree above k are not part of the state
        const long long plane = (long long)x.nx * x.ny;
        for (int mesh = 0; mesh < 2; ++mesh)
            for (int q = 0; q < x.nc; ++q)
                for (int i = 0; i <= x.k; ++i)
                    for (int j = 0; j <= x.k; ++j)
                        if (i + j > x.k)
                            HIPCHK2(h, hipMemsetAsync(x.B[0] + mesh * x.S1 + ((q * (x.k + 1) + i) * (x.k + 1) + j) * plane,
                                                      0, sizeof(double) * plane, s));
    }
    // statistics of the initial data (wave speeds for the first step) into part[0]
    HIPCHK2(h, delta_of(x, x.B[0], x.B[0] + x.S1, 0, M2_FINAL, s));
    const int chunk = 16;
    long long n = 0;
    while (nsteps < 0 || n < nsteps) {
        const long long m = nsteps < 0 ? chunk : std::min<long long>(chunk, nsteps - n);
        for (long long j = 0; j < m; ++j)
            for (int l = 0; l < x.ns; ++l) {
                const long long g = (long long)x.ns * (n + j) + l;
                const int ib = (int)(g & 1), ob = (int)((g + 1) & 1);
                Red2Args r = red_args(x, x.part[ib], l == 0 ? R2_STEP : R2_STAGE);
                r.t_end = t_end;
                r.dt_fixed = dt_fixed;
                HIPCHK2(h, launch_reduce2d(x, r, s));
                Stage2Args a = stage_args(x);
                a.mode = M2_STAGE;
                a.l = l;
                a.rs = rk_stage(x.rk, l);
                a.damp = x.oe && x.k > 0 && !(n + j == 0 && l == 0);
                a.write_u = l == 0;
                a.inC = x.B[ib];
                a.inD = x.B[ib] + x.S1;
                a.numC = x.num[ib];
                a.numD = x.num[ib] + x.SN;
                a.outC = x.B[ob];
                a.outD = x.B[ob] + x.S1;
                a.UC = x.U;
                a.UD = x.U + x.S1;
                HIPCHK2(h, launch_stage2d(x, a, s));
                HIPCHK2(h, delta_of(x, x.B[ob], x.B[ob] + x.S1, ob, M2_STAGE, s));
            }
        n += m;
        HIPCHK2(h, hipMemcpyAsync(x.st_h, x.st, sizeof(Stats2), hipMemcpyDeviceToHost, s));
        HIPCHK2(h, hipStreamSynchronize(s));
        if (x.st_h->done) break;
    }
    const long long N = x.st_h->nexec + x.st_h->pending;   // executed steps
    const int fb = (int)((x.ns * N) & 1);                  // buffer of the last stage's output
    Red2Args r = red_args(x, x.part[fb], R2_FINAL);
    r.t_end = t_end;
    HIPCHK2(h, launch_reduce2d(x, r, s));
    Stage2Args f = stage_args(x);
    f.mode = M2_FINAL;
    f.damp = x.oe && x.k > 0 && N > 0;
    f.inC = x.B[fb];
    f.inD = x.B[fb] + x.S1;
    f.numC = x.num[fb];
    f.numD = x.num[fb] + x.SN;
    f.outC = uC;
    f.outD = uD;
    HIPCHK2(h, launch_stage2d(x, f, s));
    HIPCHK2(h, hipMemcpyAsync(x.st_h, x.st, sizeof(Stats2), hipMemcpyDeviceToHost, s));
    rc = check2d(h, x);
    if (t_out) *t_out = x.st_h->t;
    if (steps_out) *steps_out = N;
    return rc;
}

}  // namespace oecdg
