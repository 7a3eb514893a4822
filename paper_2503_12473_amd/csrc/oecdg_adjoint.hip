// oecdg_adjoint.hip -- discrete adjoint of the 1D scalar RK-OECDG step
// (periodic mesh, fixed tau), the transpose of the forward kernels' map.
//
// Forward stage l of a step (eq:RKCDG with SSP-RK3, then the OE step):
//   h_{l+1} = a_l s_0 + b_l (s_l + tau L(s_l)),   s_{l+1} = F_tau(h_{l+1}),
//   (a_l, b_l) = (0, 1), (3/4, 1/4), (1/3, 2/3); u^{n+1} = s_3.
// F_tau(h)_j = h_j exp(-tau sum_{m<=j} delta^m(h)) for j >= 1 (the exact
// solution of the damping ODE), delta^m_K = C_m / h * beta_K (|dR_m| + |dL_m|)
// / sigma (Sec. 2.2).  Given lambda = dJ/ds_{l+1}, the reverse of stage l is
//   mu = F'(h_{l+1})^T lambda,
//   dJ/ds_l = b_l (mu + tau L'(s_l)^T mu),   dJ/ds_0 += a_l mu.
//
// One launch per reverse stage.  F'(h)^T lambda splits into a part local to
// each cell (diagonal, the cell's own traces in delta, beta), coefficients
// scattered to the two overlapping cells of the other mesh, and two global
// terms (sigma and the mesh average).  The local part for stage l-1 needs
// lambda = dJ/ds_l only at the cell itself, so the launch that finishes
// dJ/ds_l also "prepares" stage l-1: it writes that local part, the scattered
// coefficients and per-workgroup partials of the global terms, which the next
// launch gathers.  A prepare-only launch starts each chain.
//
// Non-smooth points follow fixed conventions: d|x|/dx = 0 at x = 0, the
// L-infinity norm in sigma is attributed to the first maximiser in (cell,
// sample point) order, and a vanishing sigma contributes nothing.
#include "oecdg_device.h"
#include "oecdg_internal.h"
#include "oecdg_tables.h"

namespace oecdg {

constexpr int ADJ_NT = 128;          // threads (= cells) per workgroup
constexpr int ADJ_NW = ADJ_NT / WAVE;
constexpr int ADJ_PRE = 4;           // partial entries per thread issued before the first wait
// per-workgroup partials: sigma adjoint, sample max, its first index, sample
// min, its first index, and the forward average / max / min of the mesh
constexpr int ADJ_BP = 8;

// Cells of the other mesh that overlap cell c (periodic, n cells per mesh):
// primal i: left dual i, right dual i+1; dual j: left primal j-1, right primal j.
__device__ inline int nb_left(int mesh, int c, int n) { return mesh == 0 ? c : (c == 0 ? n - 1 : c - 1); }
__device__ inline int nb_right(int mesh, int c, int n) { return mesh == 0 ? (c + 1 == n ? 0 : c + 1) : c; }
// Cells of the other mesh whose left (right) overlapping neighbour is cell c.
__device__ inline int user_left(int mesh, int c, int n) { return mesh == 0 ? (c + 1 == n ? 0 : c + 1) : c; }
__device__ inline int user_right(int mesh, int c, int n) { return mesh == 0 ? c : (c == 0 ? n - 1 : c - 1); }

template <int K>
__device__ inline void load_cell(const double *u, int n, int c, double (&v)[K + 1]) {
#pragma unroll
    for (int m = 0; m <= K; ++m) v[m] = u[(long long)m * n + c];
}

// Broadcast lane 63 (where wave_reduce leaves its result) to the wave.
__device__ inline double bcast_last(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffLL), WAVE - 1);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), WAVE - 1);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave part of a block reduction: plain values (sum/max/min) and extremum
// pairs (value, first index); lane 63 stores them into this wave's row of
// `scratch`.  After one barrier, combine_* fold the rows of all waves.
template <int NV, int NP>
__device__ inline void wave_stage(const int (&kind)[NV], double (&v)[NV], const int (&pkind)[NP], double (&pv)[NP],
                                  double (&pi)[NP], double *scratch) {
    constexpr int ROW = NV + 2 * NP;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_reduce(kind[i], v[i]);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double m = bcast_last(wave_reduce(pkind[i], pv[i]));
        pi[i] = wave_reduce(2, pv[i] == m ? pi[i] : INFINITY);
        pv[i] = m;
    }
    if (lane == WAVE - 1) {
        double *row = scratch + wave * ROW;
#pragma unroll
        for (int i = 0; i < NV; ++i) row[i] = v[i];
#pragma unroll
        for (int i = 0; i < NP; ++i) row[NV + 2 * i] = pv[i], row[NV + 2 * i + 1] = pi[i];
    }
}

template <int NV, int NP>
__device__ inline void combine_rows(const int (&kind)[NV], double (&v)[NV], const int (&pkind)[NP], double (&pv)[NP],
                                    double (&pi)[NP], const double *scratch) {
    constexpr int ROW = NV + 2 * NP;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double r = scratch[i];
        for (int w = 1; w < ADJ_NW; ++w) r = stat_op(kind[i], r, scratch[w * ROW + i]);
        v[i] = r;
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double m = scratch[NV + 2 * i], id = scratch[NV + 2 * i + 1];
        for (int w = 1; w < ADJ_NW; ++w) {
            const double mw = scratch[w * ROW + NV + 2 * i], iw = scratch[w * ROW + NV + 2 * i + 1];
            const bool better = pkind[i] == 1 ? mw > m : mw < m;
            if (better || (mw == m && iw < id)) m = mw, id = iw;
        }
        pv[i] = m;
        pi[i] = id;
    }
}

// The global terms of F'(h)^T lambda on each mesh: sign x sigma adjoint (0 if
// sigma vanished) and the sample point the L-infinity norm is attributed to.
struct SigmaTerm {
    double w[2];
    long long cell[2];
    int sidx[2];
};

// Operands of mu = F'(h)^T lambda at cell c of mesh X: its local part (or
// lambda itself when OE is off) and the coefficients scattered to it by the
// two overlapping cells of the other mesh.
template <int K>
struct MuIn {
    double lp[K + 1], cr[K + 1], cl[K + 1];
};

template <int K, bool OE>
__device__ inline void load_mu(const AdjArgs &a, int X, int c, MuIn<K> &in) {
    const int n = a.n;
    if constexpr (!OE) {
        load_cell<K>(a.lam + X * a.S, n, c, in.lp);
    } else {
        load_cell<K>(a.lp_in + X * a.S, n, c, in.lp);
        load_cell<K>(a.cr_in + (1 - X) * a.S, n, user_right(X, c, n), in.cr);
        load_cell<K>(a.cl_in + (1 - X) * a.S, n, user_left(X, c, n), in.cl);
    }
}

// mu from its operands and the global terms (sigma, mesh average).
template <int K, bool OE>
__device__ inline void finish_mu(const AdjArgs &a, const SigmaTerm &t, int X, int c, const MuIn<K> &in,
                                 double (&mu)[K + 1]) {
    constexpr Tab<K> tb = make_tab<K>();
#pragma unroll
    for (int q = 0; q <= K; ++q) mu[q] = in.lp[q];
    if constexpr (!OE) return;
#pragma unroll
    for (int q = 0; q <= K; ++q) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m <= q; ++m) s += (in.cr[m] + in.cl[m]) * tb.D0[m][q];
        mu[q] -= s;
    }
    if (t.w[X] != 0.0) {
        if ((long long)c == t.cell[X]) {
#pragma unroll
            for (int q = 0; q <= K; ++q) mu[q] += t.w[X] * tb.SP[t.sidx[X]][q];
        }
        mu[0] -= t.w[X] * a.inv_n;
    }
}

// Transpose of the CDG operator's dependence on an overlapping cell J of the
// other mesh (coefficients sJ) for the half hf of cell K that J overlaps:
// the 1/tau_max coupling, the volume quadrature of f and the edge flux.
template <int K, int FLUX>
__device__ inline void neighbour_transpose(const AdjArgs &a, const double (&sJ)[K + 1], const double (&muK)[K + 1],
                                           int hf, double (&acc)[K + 1]) {
    constexpr Tab<K> tb = make_tab<K>();
#pragma unroll
    for (int g = 0; g <= K; ++g) {
        double w = 0.0;
#pragma unroll
        for (int q = 0; q <= K; ++q) w += sJ[q] * tb.E[hf][g][q];
        const double fp = FLUX == 0 ? a.p0 : w;            // f'(w)
        double coef = 0.0;
#pragma unroll
        for (int m = 0; m <= K; ++m)
            coef += muK[m] * ((m + 0.5) * a.inv_tm * tb.WP[hf][g][m] + (2.0 * m + 1.0) * a.hinv * tb.WD[hf][g][m] * fp);
#pragma unroll
        for (int q = 0; q <= K; ++q) acc[q] += coef * tb.E[hf][g][q];
    }
    double w0 = 0.0;
#pragma unroll
    for (int q = 0; q <= K; ++q) w0 += sJ[q] * tb.D0[0][q];
    const double fp0 = FLUX == 0 ? a.p0 : w0;
    double e = 0.0;
#pragma unroll
    for (int m = 0; m <= K; ++m) e += muK[m] * (2.0 * m + 1.0) * a.hinv * (hf == 1 ? -1.0 : ((m & 1) ? -1.0 : 1.0));
#pragma unroll
    for (int q = 0; q <= K; ++q) acc[q] += e * fp0 * tb.D0[0][q];
}

// Launch modes: the reverse of a stage without OE (lambda gathered directly),
// with OE (gathering the preparation of the stage above), prepare-only, and
// reverse with OE plus preparation of the stage below.
enum { ADJ_RK_PLAIN = 0, ADJ_RK = 1, ADJ_PREP = 2, ADJ_RK_PREP = 3 };

template <int K, int FLUX, int MODE>
__global__ __launch_bounds__(ADJ_NT) void k_adj(AdjArgs a) {
    using F = FluxT<FLUX>;
    constexpr Tab<K> tb = make_tab<K>();
    constexpr int NSP = 2 * K + 4;
    constexpr bool RK = MODE != ADJ_PREP, OE = MODE != ADJ_RK_PLAIN;
    constexpr bool PREP = MODE == ADJ_PREP || MODE == ADJ_RK_PREP, GSIG = MODE == ADJ_RK || MODE == ADJ_RK_PREP;
    constexpr int ROW1 = 5 + 2 * 4, ROW2 = 1 + 2 * 2;
    static_assert(ADJ_NW * (ROW1 + ROW2) <= 64, "scratch holds one row per wave and pass");
    __shared__ double scratch[64];
    const int n = a.n, tid = threadIdx.x;
    const int mesh = blockIdx.x >= (unsigned)a.nb;
    const int blk = blockIdx.x - mesh * a.nb;
    const int c = blk * ADJ_NT + tid;
    const bool valid = c < n;
    const int cc = valid ? c : 0;
    const int other = 1 - mesh;

    // ---- every load that does not depend on another, issued before any wait
    // (no loads under divergent branches: clamped indices, then selects); one
    // entry per thread of the workgroup and tile partials, larger grids loop below
    MuIn<K> inJ, inL, inR;
    double sJ[K + 1], accv[K + 1], own[K + 1], nl[K + 1], nr[K + 1], lam[K + 1];
    if constexpr (RK) {
        load_mu<K, OE>(a, mesh, cc, inJ);
        load_mu<K, OE>(a, other, user_left(mesh, cc, n), inL);     // cc overlaps its left half
        load_mu<K, OE>(a, other, user_right(mesh, cc, n), inR);    // cc overlaps its right half
        // s_l: for l = 0 the damped u^n the forward stage stored (also at a
        // segment start, where h of the step before is not at hand); for
        // l > 0 with preparation it is formed below as F_tau(h_l)
        load_cell<K>(a.s + mesh * a.S, n, cc, sJ);
        load_cell<K>(a.acc + mesh * a.S, n, cc, accv);            // unused when acc_init
    } else {
        load_cell<K>(a.lam + mesh * a.S, n, cc, lam);
    }
    if constexpr (PREP) {
        load_cell<K>(a.h + mesh * a.S, n, cc, own);
        load_cell<K>(a.h + other * a.S, n, nb_left(mesh, cc, n), nl);
        load_cell<K>(a.h + other * a.S, n, nb_right(mesh, cc, n), nr);
    }
    // up to ADJ_PRE entries per thread of the per-wave partials of the stage
    // above and of the forward tile partials, loaded unconditionally (clamped
    // indices) before any wait and folded afterwards; larger grids loop
    double bsum[2], bmx[2], bmn[2], bimx[2], bimn[2], fav[2], fmx[2], fmn[2];
    double ebp[2][ADJ_PRE][5], efs[3][ADJ_PRE];
    if constexpr (GSIG) {
#pragma unroll
        for (int Y = 0; Y < 2; ++Y) {
            const double *f0 = a.bp_in + (long long)(Y * a.nbp) * ADJ_BP;
            fav[Y] = f0[5];
            fmx[Y] = f0[6];
            fmn[Y] = f0[7];
#pragma unroll
            for (int r = 0; r < ADJ_PRE; ++r) {
                const int bb = tid + r * ADJ_NT;
                const double *bp = a.bp_in + (long long)(Y * a.nbp + (bb < a.nbp ? bb : 0)) * ADJ_BP;
#pragma unroll
                for (int c = 0; c < 5; ++c) ebp[Y][r][c] = bp[c];
            }
        }
    }
    if constexpr (PREP) {
#pragma unroll
        for (int kd = 0; kd < 3; ++kd) {
            const double *col = a.fpart + (long long)a.ftile0 * NSTAT + stat_index(mesh, 0, kd);   // [tile][row]
#pragma unroll
            for (int r = 0; r < ADJ_PRE; ++r) {
                const int tt = tid + r * ADJ_NT;
                efs[kd][r] = col[(long long)(tt < a.fntiles ? tt : 0) * NSTAT];
            }
        }
    }
#pragma unroll
    for (int Y = 0; Y < 2; ++Y) {
        bsum[Y] = 0.0;
        bmx[Y] = -INFINITY;
        bmn[Y] = bimx[Y] = bimn[Y] = INFINITY;
    }
    if constexpr (GSIG) {
#pragma unroll
        for (int Y = 0; Y < 2; ++Y) {
#pragma unroll
            for (int r = 0; r < ADJ_PRE; ++r) {
                if (tid + r * ADJ_NT >= a.nbp) continue;
                const double *v = ebp[Y][r];
                bsum[Y] += v[0];
                if (v[1] > bmx[Y] || (v[1] == bmx[Y] && v[2] < bimx[Y])) bmx[Y] = v[1], bimx[Y] = v[2];
                if (v[3] < bmn[Y] || (v[3] == bmn[Y] && v[4] < bimn[Y])) bmn[Y] = v[3], bimn[Y] = v[4];
            }
            for (int bb = tid + ADJ_PRE * ADJ_NT; bb < a.nbp; bb += ADJ_NT) {
                const double *bp = a.bp_in + (long long)(Y * a.nbp + bb) * ADJ_BP;
                bsum[Y] += bp[0];
                if (bp[1] > bmx[Y] || (bp[1] == bmx[Y] && bp[2] < bimx[Y])) bmx[Y] = bp[1], bimx[Y] = bp[2];
                if (bp[3] < bmn[Y] || (bp[3] == bmn[Y] && bp[4] < bimn[Y])) bmn[Y] = bp[3], bimn[Y] = bp[4];
            }
        }
    } else {
#pragma unroll
        for (int Y = 0; Y < 2; ++Y) fav[Y] = fmx[Y] = fmn[Y] = 0.0;
    }
    // forward statistics of h on this workgroup's mesh: sum, max, min over its tiles
    double fs[3] = {0.0, -INFINITY, INFINITY};
    if constexpr (PREP) {
#pragma unroll
        for (int kd = 0; kd < 3; ++kd) {
#pragma unroll
            for (int r = 0; r < ADJ_PRE; ++r)
                if (tid + r * ADJ_NT < a.fntiles) fs[kd] = stat_op(kd, fs[kd], efs[kd][r]);
            const double *col = a.fpart + (long long)a.ftile0 * NSTAT + stat_index(mesh, 0, kd);
            for (int tt = tid + ADJ_PRE * ADJ_NT; tt < a.fntiles; tt += ADJ_NT)
                fs[kd] = stat_op(kd, fs[kd], col[(long long)tt * NSTAT]);
        }
    }

    // ---- first reduction pass: global terms of the stage above and the forward statistics of h
    SigmaTerm t;
    t.w[0] = t.w[1] = 0.0;
    t.cell[0] = t.cell[1] = -1;
    t.sidx[0] = t.sidx[1] = 0;
    double sig = 0.0, avg = 0.0;
    if constexpr (GSIG || PREP) {
        const int k1[5] = {0, 0, 0, 1, 2};
        double v1[5] = {bsum[0], bsum[1], fs[0], fs[1], fs[2]};
        const int pk1[4] = {1, 1, 2, 2};
        double pv1[4] = {bmx[0], bmx[1], bmn[0], bmn[1]};
        double pi1[4] = {bimx[0], bimx[1], bimn[0], bimn[1]};
        wave_stage<5, 4>(k1, v1, pk1, pv1, pi1, scratch);
        __syncthreads();
        combine_rows<5, 4>(k1, v1, pk1, pv1, pi1, scratch);
        if constexpr (GSIG) {
#pragma unroll
            for (int Y = 0; Y < 2; ++Y) {
                // sigma = max(max - avg, avg - min): the branch of the first maximiser
                const double up = fmx[Y] - fav[Y], dn = fav[Y] - fmn[Y];
                const bool use_max = up > dn || (up == dn && pi1[Y] <= pi1[2 + Y]);
                const double idx = use_max ? pi1[Y] : pi1[2 + Y];
                const bool live = fmax(up, dn) != 0.0 && idx < INFINITY;
                t.w[Y] = live ? (use_max ? v1[Y] : -v1[Y]) : 0.0;
                const long long li = live ? (long long)idx : 0;     // an exact integer below 2^53
                t.cell[Y] = live ? li / NSP : -1;
                t.sidx[Y] = (int)(li % NSP);
            }
        }
        avg = v1[2] / (double)n;                     // the forward kernels' average, same division
        fs[1] = v1[3];
        fs[2] = v1[4];
        sig = fmax(fs[1] - avg, avg - fs[2]);
    }

    // ---- the damping of h_l at this cell (the lambda-independent part of the
    // preparation); the reverse stage then uses s_l = F_tau(h_l) at the cell
    double beta = 0.0, isig = 0.0, dR[K + 1], dL[K + 1], del[K + 1], facj[K + 1];
    if constexpr (PREP) {
        beta = F::speed(own, a.p0);
        isig = sig != 0.0 ? 1.0 / sig : 0.0;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            double ur = 0.0, ul = 0.0, vr = 0.0, vl = 0.0;
#pragma unroll
            for (int q = m; q <= K; ++q) {
                const double d1 = tb.D1[m][q];
                ur += own[q] * d1;
                ul += own[q] * (((q + m) & 1) ? -d1 : d1);
                vr += nr[q] * tb.D0[m][q];
                vl += nl[q] * tb.D0[m][q];
            }
            dR[m] = ur - vr;
            dL[m] = ul - vl;
            del[m] = tb.C[m] * a.hinv * (beta * (fabs(dR[m]) + fabs(dL[m])) * isig);
        }
        double S = 0.0;
        facj[0] = 1.0;
#pragma unroll
        for (int j = 1; j <= K; ++j) {
            S = (j == 1 ? del[0] : S) + del[j];
            facj[j] = exp(-a.tau * S);
        }
        if constexpr (RK) {
            if (!a.stage0) {
#pragma unroll
                for (int q = 0; q <= K; ++q) sJ[q] = own[q] * facj[q];
            }
        }
    }

    // ---- reverse of stage l: dJ/ds_l and the a_l share of dJ/ds_0
    if constexpr (RK) {
        double muJ[K + 1], muL[K + 1], muR[K + 1];
        finish_mu<K, OE>(a, t, mesh, cc, inJ, muJ);
        finish_mu<K, OE>(a, t, other, user_left(mesh, cc, n), inL, muL);
        finish_mu<K, OE>(a, t, other, user_right(mesh, cc, n), inR, muR);
        double lt[K + 1];
#pragma unroll
        for (int q = 0; q <= K; ++q) lt[q] = -a.inv_tm * muJ[q];
        neighbour_transpose<K, FLUX>(a, sJ, muL, 0, lt);
        neighbour_transpose<K, FLUX>(a, sJ, muR, 1, lt);
#pragma unroll
        for (int q = 0; q <= K; ++q) {
            const double v = a.bl * (muJ[q] + a.tau * lt[q]);
            if (a.stage0) {
                lam[q] = accv[q] + v;
            } else {
                lam[q] = v;
                accv[q] = a.acc_init ? a.al * muJ[q] : accv[q] + a.al * muJ[q];
            }
        }
        if (valid) {
            double *out = a.out + mesh * a.S, *acc = a.acc + mesh * a.S;
#pragma unroll
            for (int q = 0; q <= K; ++q) {
                out[(long long)q * n + c] = lam[q];
                if (!a.stage0) acc[(long long)q * n + c] = accv[q];
            }
        }
    }
    if constexpr (!PREP) return;

    // ---- preparation of the stage below: the local part of F'(h)^T lambda
    double lp[K + 1], fo[K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j) {
        fo[j] = own[j] * facj[j];
        lp[j] = lam[j] * facj[j];
    }
    double cR[K + 1], cL[K + 1], sbar = 0.0;
#pragma unroll
    for (int m = 0; m <= K; ++m) cR[m] = cL[m] = 0.0;
    if (sig != 0.0) {
        double dbeta = 0.0;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            double g = 0.0;
#pragma unroll
            for (int j = (m > 1 ? m : 1); j <= K; ++j) g += lam[j] * fo[j];
            g *= -a.tau;                                    // dJ/d delta^m
            const double w = g * tb.C[m] * a.hinv * isig;
            const double sR = (dR[m] > 0.0) - (dR[m] < 0.0), sL = (dL[m] > 0.0) - (dL[m] < 0.0);
            cR[m] = w * beta * sR;
            cL[m] = w * beta * sL;
            dbeta += w * (fabs(dR[m]) + fabs(dL[m]));
            sbar -= g * del[m] * isig;
        }
#pragma unroll
        for (int q = 0; q <= K; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m <= q; ++m) {
                const double d1 = tb.D1[m][q];
                acc += cR[m] * d1 + cL[m] * (((q + m) & 1) ? -d1 : d1);
            }
            lp[q] += acc;
        }
        if constexpr (FLUX == 1) lp[0] += dbeta * ((own[0] > 0.0) - (own[0] < 0.0));   // beta = |u_bar|
    }
    // sample values of h (edges and half-cell nodes, natural order)
    double vmax = -INFINITY, vmin = INFINITY, imax = INFINITY, imin = INFINITY;
    if (valid) {
        double *LP = a.lp + mesh * a.S, *CR = a.cr + mesh * a.S, *CL = a.cl + mesh * a.S;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            LP[(long long)m * n + c] = lp[m];
            CR[(long long)m * n + c] = cR[m];
            CL[(long long)m * n + c] = cL[m];
        }
#pragma unroll
        for (int sidx = 0; sidx < NSP; ++sidx) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q <= K; ++q) v += own[q] * tb.SP[sidx][q];
            const double idx = (double)c * NSP + sidx;
            if (v > vmax) vmax = v, imax = idx;
            if (v < vmin) vmin = v, imin = idx;
        }
    }
    // ---- this wave's partials of the prepared stage (no barrier: one entry
    // per wave, entry (mesh, workgroup, wave) in that order)
    double *sc2 = scratch + ADJ_NW * ROW1;
    const int k2[1] = {0};
    double v2[1] = {valid ? sbar : 0.0};
    const int pk2[2] = {1, 2};
    double pv2[2] = {vmax, vmin}, pi2[2] = {imax, imin};
    wave_stage<1, 2>(k2, v2, pk2, pv2, pi2, sc2);
    if (tid % WAVE == WAVE - 1) {
        double *bp = a.bp + ((long long)blockIdx.x * ADJ_NW + tid / WAVE) * ADJ_BP;
        bp[0] = v2[0];
        bp[1] = pv2[0];
        bp[2] = pi2[0];
        bp[3] = pv2[1];
        bp[4] = pi2[1];
        bp[5] = avg;
        bp[6] = fs[1];
        bp[7] = fs[2];
    }
}

// ------------------------------------------------------------ host side ---

template <int K, int FLUX>
static void *adj_kernel(int mode) {
    switch (mode) {
    case ADJ_RK_PLAIN: return (void *)k_adj<K, FLUX, ADJ_RK_PLAIN>;
    case ADJ_RK: return (void *)k_adj<K, FLUX, ADJ_RK>;
    case ADJ_PREP: return (void *)k_adj<K, FLUX, ADJ_PREP>;
    default: return (void *)k_adj<K, FLUX, ADJ_RK_PREP>;
    }
}

static void *adj_pick(int k, int flux, int mode) {
    switch (k * 2 + (flux == 1)) {
    case 0: return adj_kernel<0, 0>(ADJ_RK_PLAIN);
    case 1: return adj_kernel<0, 1>(ADJ_RK_PLAIN);
    case 2: return adj_kernel<1, 0>(mode);
    case 3: return adj_kernel<1, 1>(mode);
    case 4: return adj_kernel<2, 0>(mode);
    case 5: return adj_kernel<2, 1>(mode);
    case 6: return adj_kernel<3, 0>(mode);
    default: return adj_kernel<3, 1>(mode);
    }
}

hipError_t launch_adj(const AdjArgs &a, hipStream_t s) {
    AdjArgs copy = a;
    void *args[] = {&copy};
    const bool oe = a.oe && a.k > 0;
    const int mode = !oe ? ADJ_RK_PLAIN : (!a.do_rk ? ADJ_PREP : (a.do_prep ? ADJ_RK_PREP : ADJ_RK));
    if (!oe && !a.do_rk) return hipSuccess;          // nothing to prepare without OE
    return hipLaunchKernel(adj_pick(a.k, a.flux, mode), dim3(2 * a.nb), dim3(ADJ_NT), args, 0, s);
}
int adj_block_size() { return ADJ_NT; }
int adj_block_partials() { return ADJ_BP * ADJ_NW; }
int adj_waves() { return ADJ_NW; }

}  // namespace oecdg
