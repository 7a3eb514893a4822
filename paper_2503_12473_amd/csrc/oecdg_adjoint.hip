// oecdg_adjoint.hip -- discrete adjoint of the 1D scalar RK-OECDG step
// (periodic mesh, fixed tau), the transpose of the forward kernels' map.
//
// Forward stage l of a step (eq:RKCDG with SSP-RK3, then OEstep1):
//   h_{l+1} = a_l s_0 + b_l (s_l + tau L(s_l)),   s_{l+1} = F_tau(h_{l+1}),
//   (a_l, b_l) = (0, 1), (3/4, 1/4), (1/3, 2/3); u^{n+1} = s_3.
// F_tau(h)_j = h_j exp(-tau sum_{m<=j} delta^m(h)) for j >= 1 (OEstep2D),
// delta^m_K = C_m / h * beta_K (|dR_m| + |dL_m|) / sigma (Sec. 2.2).
// Given lambda = dJ/ds_{l+1} the reverse stage computes
//   mu = F'(h)^T lambda                                   (k_adj_oe + gather),
//   dJ/ds_l = b_l (mu + tau L'(s_l)^T mu),  dJ/ds_0 += a_l mu  (k_adj_rk).
// Both transposes are evaluated in gather form: a cell collects what its two
// overlapping neighbours on the other mesh scattered to it.  Non-smooth points
// follow fixed conventions: d|x|/dx = 0 at x = 0, the L-infinity norm in sigma
// is attributed to the first maximiser in (cell, sample point) order, and a
// vanishing sigma contributes nothing.
#include "oecdg_device.h"
#include "oecdg_internal.h"
#include "oecdg_tables.h"

namespace oecdg {

constexpr int ADJ_NT = 256;          // threads (= cells) per workgroup
constexpr int ADJ_BP = 5;            // block partials: sigma-bar, max, first argmax, min, first argmin

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

// Forward statistics of the stage output (avg, sigma, max, min per mesh) from
// the forward kernels' per-tile partials, reduced in their fixed order.
struct MeshStats {
    double avg[2], sig[2], mx[2], mn[2];
};

template <int NT>
__device__ inline MeshStats forward_stats(const AdjArgs &a, double *red, double *scratch) {
    static_assert(((NT + WAVE - 1) / WAVE) * Partials<1>::NS <= 64, "scratch holds one row per wave");
    Partials<1> p;
    const int ns = Partials<1>::NS - 2;
    load_partials<NT, 1>(a.fpart, a.fntot, a.ftile0, a.fntiles, ns, p);
    finish_partials<NT, 1>(p, a.fpart, a.fntot, a.ftile0, a.fntiles, ns, red, scratch);
    MeshStats s;
#pragma unroll
    for (int mesh = 0; mesh < 2; ++mesh) {
        s.avg[mesh] = red[stat_index(mesh, 0, 0)] / (double)a.n;
        s.mx[mesh] = red[stat_index(mesh, 0, 1)];
        s.mn[mesh] = red[stat_index(mesh, 0, 2)];
        s.sig[mesh] = fmax(s.mx[mesh] - s.avg[mesh], s.avg[mesh] - s.mn[mesh]);
    }
    return s;
}

// Block-wide reduction (256 threads, 4 waves, fixed order); result broadcast.
__device__ inline double block_reduce(int kind, double v, double *scratch) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    v = wave_reduce(kind, v);
    __syncthreads();
    if (lane == WAVE - 1) scratch[wave] = v;
    __syncthreads();
    double r = scratch[0];
    for (int w = 1; w < ADJ_NT / WAVE; ++w) r = stat_op(kind, r, scratch[w]);
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- OE pass ---
// Per cell K of the damped mesh: recompute delta, the damping factors and
// F(h); write the local part of F'(h)^T lambda (diagonal, own traces, beta),
// the coefficients scattered to the right/left neighbours through dR/dL, and
// the block partials of the sigma adjoint and of the first maximiser/minimiser.
template <int K, int FLUX>
__global__ __launch_bounds__(ADJ_NT) void k_adj_oe(AdjArgs a) {
    using F = FluxT<FLUX>;
    constexpr Tab<K> tb = make_tab<K>();
    constexpr int NSP = 2 * K + 4;
    __shared__ double red[NSTAT], scratch[64];
    const MeshStats st = forward_stats<ADJ_NT>(a, red, scratch);
    const int mesh = blockIdx.x >= (unsigned)a.nb;
    const int c = (blockIdx.x - mesh * a.nb) * ADJ_NT + threadIdx.x;
    const bool valid = c < a.n;
    const int cc = valid ? c : 0;
    const double *hM = mesh == 0 ? a.hC : a.hD, *hO = mesh == 0 ? a.hD : a.hC;
    const double *lam = mesh == 0 ? a.lamC : a.lamD;
    double own[K + 1], nl[K + 1], nr[K + 1], lm[K + 1];
    load_cell<K>(hM, a.n, cc, own);
    load_cell<K>(hO, a.n, nb_left(mesh, cc, a.n), nl);
    load_cell<K>(hO, a.n, nb_right(mesh, cc, a.n), nr);
    load_cell<K>(lam, a.n, cc, lm);
    const double sig = st.sig[mesh];
    const double beta = F::speed(own, a.p0);
    double dR[K + 1], dL[K + 1], del[K + 1];
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
        del[m] = sig != 0.0 ? tb.C[m] * a.hinv * (beta * (fabs(dR[m]) + fabs(dL[m])) / sig) : 0.0;
    }
    double lp[K + 1], out[K + 1];
    double S = 0.0;
    lp[0] = lm[0];
    out[0] = own[0];
#pragma unroll
    for (int j = 1; j <= K; ++j) {
        S = (j == 1 ? del[0] : S) + del[j];
        const double fac = exp(-a.tau * S);
        out[j] = own[j] * fac;
        lp[j] = lm[j] * fac;
    }
    double cR[K + 1], cL[K + 1], sbar = 0.0;
#pragma unroll
    for (int m = 0; m <= K; ++m) cR[m] = cL[m] = 0.0;
    if (sig != 0.0 && K > 0) {
        double dbeta = 0.0;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            double g = 0.0;
#pragma unroll
            for (int j = (m > 1 ? m : 1); j <= K; ++j) g += lm[j] * out[j];
            g *= -a.tau;                                    // dJ/d delta^m
            const double w = g * tb.C[m] * a.hinv / sig;
            const double sR = (dR[m] > 0.0) - (dR[m] < 0.0), sL = (dL[m] > 0.0) - (dL[m] < 0.0);
            cR[m] = w * beta * sR;
            cL[m] = w * beta * sL;
            dbeta += w * (fabs(dR[m]) + fabs(dL[m]));
            sbar -= g * del[m] / sig;
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
    if (valid) {
        double *LP = mesh == 0 ? a.lpC : a.lpD, *CR = mesh == 0 ? a.cRC : a.cRD, *CL = mesh == 0 ? a.cLC : a.cLD;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
            LP[(long long)m * a.n + c] = lp[m];
            CR[(long long)m * a.n + c] = cR[m];
            CL[(long long)m * a.n + c] = cL[m];
        }
    }
    // sample values of h (edges and half-cell nodes, natural order)
    double vmax = -INFINITY, vmin = INFINITY, imax = INFINITY, imin = INFINITY;
    if (valid) {
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
    const double bsum = block_reduce(0, valid ? sbar : 0.0, scratch);
    const double bmax = block_reduce(1, vmax, scratch);
    const double bimax = block_reduce(2, vmax == bmax ? imax : INFINITY, scratch);
    const double bmin = block_reduce(2, vmin, scratch);
    const double bimin = block_reduce(2, vmin == bmin ? imin : INFINITY, scratch);
    if (threadIdx.x == 0) {
        double *bp = a.bp + (long long)blockIdx.x * ADJ_BP;
        bp[0] = bsum;
        bp[1] = bmax;
        bp[2] = bimax;
        bp[3] = bmin;
        bp[4] = bimin;
    }
}

// ------------------------------------------------------------ fused pass ---

// The sigma adjoint of each mesh and the sample point it acts on.
struct SigmaTerm {
    double sbar[2], sgn[2];
    long long cell[2];
    int sidx[2];
};

template <int K>
__device__ inline SigmaTerm sigma_terms(const AdjArgs &a, const MeshStats &st, double *scratch) {
    constexpr int NSP = 2 * K + 4;
    SigmaTerm t;
    for (int mesh = 0; mesh < 2; ++mesh) {
        double s = 0.0, mx = -INFINITY, mn = INFINITY;
        for (int b = threadIdx.x; b < a.nb; b += ADJ_NT) {
            const double *bp = a.bp + (long long)(mesh * a.nb + b) * ADJ_BP;
            s += bp[0];
            mx = fmax(mx, bp[1]);
            mn = fmin(mn, bp[3]);
        }
        const double ssum = block_reduce(0, s, scratch);
        const double gmx = block_reduce(1, mx, scratch);
        const double gmn = block_reduce(2, mn, scratch);
        double imx = INFINITY, imn = INFINITY;
        for (int b = threadIdx.x; b < a.nb; b += ADJ_NT) {
            const double *bp = a.bp + (long long)(mesh * a.nb + b) * ADJ_BP;
            if (bp[1] == gmx) imx = fmin(imx, bp[2]);
            if (bp[3] == gmn) imn = fmin(imn, bp[4]);
        }
        imx = block_reduce(2, imx, scratch);
        imn = block_reduce(2, imn, scratch);
        // sigma = max(max - avg, avg - min): the branch of the first maximiser
        const double up = st.mx[mesh] - st.avg[mesh], dn = st.avg[mesh] - st.mn[mesh];
        const bool use_max = up > dn || (up == dn && imx <= imn);
        const double idx = use_max ? imx : imn;
        t.sbar[mesh] = st.sig[mesh] != 0.0 ? ssum : 0.0;
        t.sgn[mesh] = use_max ? 1.0 : -1.0;
        t.cell[mesh] = (long long)(idx / NSP);
        t.sidx[mesh] = (int)(idx - (double)t.cell[mesh] * NSP);
    }
    return t;
}

// mu = F'(h)^T lambda at cell c of mesh X: local part, the coefficients its
// overlapping neighbours scattered to it, and the sigma terms.
template <int K>
__device__ inline void oe_adjoint_at(const AdjArgs &a, const SigmaTerm &t, int X, int c, double (&mu)[K + 1]) {
    constexpr Tab<K> tb = make_tab<K>();
    const int n = a.n;
    if (!a.oe || K == 0) {
        load_cell<K>(X == 0 ? a.lamC : a.lamD, n, c, mu);
        return;
    }
    double cr[K + 1], cl[K + 1];
    load_cell<K>(X == 0 ? a.lpC : a.lpD, n, c, mu);
    // the other-mesh cell with c as right neighbour scattered -cR D0; the one with c as left neighbour -cL D0
    load_cell<K>(X == 0 ? a.cRD : a.cRC, n, user_right(X, c, n), cr);
    load_cell<K>(X == 0 ? a.cLD : a.cLC, n, user_left(X, c, n), cl);
#pragma unroll
    for (int q = 0; q <= K; ++q) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m <= q; ++m) s += (cr[m] + cl[m]) * tb.D0[m][q];
        mu[q] -= s;
    }
    if (t.sbar[X] != 0.0) {
        const double w = t.sgn[X] * t.sbar[X];
        if ((long long)c == t.cell[X]) {
#pragma unroll
            for (int q = 0; q <= K; ++q) mu[q] += w * tb.SP[t.sidx[X]][q];
        }
        mu[0] -= w / (double)n;
    }
}

// Transpose of the CDG operator's dependence on an overlapping neighbour:
// the part of (L'(s)^T mu_K) that lands on cell J (coefficients sJ), for the
// half hf of K that J overlaps.
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

template <int K, int FLUX>
__global__ __launch_bounds__(ADJ_NT) void k_adj_rk(AdjArgs a) {
    __shared__ double red[NSTAT], scratch[64];
    MeshStats st;
    SigmaTerm t;
    if (a.oe && K > 0) {
        st = forward_stats<ADJ_NT>(a, red, scratch);
        t = sigma_terms<K>(a, st, scratch);
    }
    const int mesh = blockIdx.x >= (unsigned)a.nb;
    const int c = (blockIdx.x - mesh * a.nb) * ADJ_NT + threadIdx.x;
    if (c >= a.n) return;
    const int n = a.n, other = 1 - mesh;
    double muJ[K + 1], muL[K + 1], muR[K + 1], sJ[K + 1];
    oe_adjoint_at<K>(a, t, mesh, c, muJ);
    oe_adjoint_at<K>(a, t, other, user_left(mesh, c, n), muL);    // J overlaps its left half
    oe_adjoint_at<K>(a, t, other, user_right(mesh, c, n), muR);   // J overlaps its right half
    load_cell<K>(mesh == 0 ? a.sC : a.sD, n, c, sJ);
    double lt[K + 1];
#pragma unroll
    for (int q = 0; q <= K; ++q) lt[q] = -a.inv_tm * muJ[q];
    neighbour_transpose<K, FLUX>(a, sJ, muL, 0, lt);
    neighbour_transpose<K, FLUX>(a, sJ, muR, 1, lt);
    double *out = mesh == 0 ? a.outC : a.outD, *acc = mesh == 0 ? a.accC : a.accD;
#pragma unroll
    for (int q = 0; q <= K; ++q) {
        const long long e = (long long)q * n + c;
        const double v = a.bl * (muJ[q] + a.tau * lt[q]);
        if (a.stage0) {
            out[e] = acc[e] + v;
        } else {
            out[e] = v;
            acc[e] = a.acc_init ? a.al * muJ[q] : acc[e] + a.al * muJ[q];
        }
    }
}

// ------------------------------------------------------------ host side ---

template <template <int, int> class Kern>
static void *adj_pick(int k, int flux) {
    switch (k * 2 + (flux == 1)) {
    case 0: return Kern<0, 0>::ptr();
    case 1: return Kern<0, 1>::ptr();
    case 2: return Kern<1, 0>::ptr();
    case 3: return Kern<1, 1>::ptr();
    case 4: return Kern<2, 0>::ptr();
    case 5: return Kern<2, 1>::ptr();
    case 6: return Kern<3, 0>::ptr();
    default: return Kern<3, 1>::ptr();
    }
}

template <int K, int FLUX> struct OeK {
    static void *ptr() { return (void *)k_adj_oe<K, FLUX>; }
};
template <int K, int FLUX> struct RkK {
    static void *ptr() { return (void *)k_adj_rk<K, FLUX>; }
};

static hipError_t adj_launch(void *fn, const AdjArgs &a, hipStream_t s) {
    AdjArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(2 * a.nb), dim3(ADJ_NT), args, 0, s);
}

hipError_t launch_adj_oe(const AdjArgs &a, hipStream_t s) { return adj_launch(adj_pick<OeK>(a.k, a.flux), a, s); }
hipError_t launch_adj_rk(const AdjArgs &a, hipStream_t s) { return adj_launch(adj_pick<RkK>(a.k, a.flux), a, s); }
int adj_block_size() { return ADJ_NT; }
int adj_block_partials() { return ADJ_BP; }

}  // namespace oecdg
