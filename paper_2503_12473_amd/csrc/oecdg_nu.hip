// oecdg_nu.hip -- 1D OECDG on a non-uniform periodic mesh.
//
// Meshes of the 1D setting of Sec. 2.1: primal cells [x_{i-1/2}, x_{i+1/2}] of
// width h_i, dual cells [x_{i-1}, x_i] between neighbouring primal centres, so a
// dual cell holds the primal edge x_{i-1/2} off its centre.  Every cell carries
// its own geometry (centre, width, and the point where the other mesh has its
// edge); the Legendre values at the mapped quadrature nodes are evaluated at run
// time.  One thread per cell of either mesh (a 2D grid, y = mesh); per step:
//   k_nu_dt                  beta over the cell averages -> tau (device-side slot);
//                            the wave-speed partials come from k_nu_wave before the
//                            first step and from the last stage's k_nu_oe after it
//   per stage:
//     k_nu_stage             operator of eq:1D_H + the c/d combination of eq:RKCDG,
//                            and per-block statistics of the undamped result
//     k_nu_oe                every workgroup first reduces the block statistics
//                            (the same fixed order everywhere: avg = domain mean,
//                            width-weighted, and sigma per mesh), then delta_K^m
//                            (Sec. 2.2, h_{e,K} = the width of K) and the exact
//                            damping F_tau into the stage's output
//   (the step ends in the next step's k_nu_dt; k_nu_advance ends the last one)
// No host synchronisation inside a step; the host polls the slot every few
// steps when it marches to a final time.
#include "oecdg_device.h"
#include "oecdg_tables.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace oecdg {
namespace {

constexpr int NB = 128;                 // threads per workgroup (2 waves: 256 workgroups at N = 16384)
constexpr int POLL = 16;                // steps between host checks of the slot when marching to t_end

// Run-time Legendre values: d-th derivative of P_m at x, m <= 3.
__device__ inline double legr(int m, int d, double x) {
    if (d == 0) return m == 0 ? 1.0 : m == 1 ? x : m == 2 ? 1.5 * x * x - 0.5 : (2.5 * x * x - 1.5) * x;
    if (d == 1) return m == 0 ? 0.0 : m == 1 ? 1.0 : m == 2 ? 3.0 * x : 7.5 * x * x - 1.5;
    if (d == 2) return m < 2 ? 0.0 : m == 2 ? 3.0 : 15.0 * x;
    return m == 3 ? 15.0 : 0.0;
}

struct NuArgs {
    int n, k, flux, oe;
    double L, hmax, cfl, p0, t_end, dt_fixed;
    const double *edges;                 // [n+1]
    const double *cC, *wC;               // primal centres and widths [n]
    const double *cD, *wD;               // dual centres and widths [n] (dual 0 starts below xlo)
    // stage
    const double *unC, *unD, *ulC, *ulD; // u^n and the stage input u^{n,l}
    double *tC, *tD;                     // undamped stage output
    double *oC, *oD;                     // damped stage output
    double cn, cw, dd;                   // c_{l0}, c_{ll}, d_{ll} (l = 0: cn = 0)
    double *part;                        // [mesh][3 NC][nblk]
    double *wpart;                       // wave-speed partials [2 nblk]
    Slot *slot;
    long long *nexec;                    // steps executed
    int wave_out;                        // last stage: also write the wave-speed partials of its output
    int pending;                         // k_nu_dt first ends the previous step
    int *err;                            // [0] non-finite, [1] non-physical, [2] bad wave speed
    int nblk;
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

// In-block reduction of NV values per thread in a fixed tree order (kind per value).
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], const int (&kind)[NV], double *sh) {
    const int t = threadIdx.x;
    for (int s = NB / 2; s > 0; s >>= 1) {
#pragma unroll
        for (int r = 0; r < NV; ++r) sh[r * NB + t] = v[r];
        __syncthreads();
        if (t < s) {
#pragma unroll
            for (int r = 0; r < NV; ++r) v[r] = stat_op(kind[r], v[r], sh[r * NB + t + s]);
        }
        __syncthreads();
    }
}

template <int FLUX>
__global__ void __launch_bounds__(NB) k_nu_wave(NuArgs a) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC;
    __shared__ double sh[NB];
    const int M = blockIdx.y, i = blockIdx.x * NB + threadIdx.x;
    double b = 0.0;
    if (i < a.n && !a.slot->done) {
        const double *u = M == 0 ? a.unC : a.unD;
        double ub[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) ub[q] = u[(long long)(q * (a.k + 1)) * a.n + i];
        b = F::speed(ub, a.p0);
        if (!(b >= 0.0)) b = INFINITY;               // NaN: reported by k_nu_dt
    }
    double v[1] = {b};
    const int kind[1] = {1};
    block_reduce<1>(v, kind, sh);
    if (threadIdx.x == 0) a.wpart[M * a.nblk + blockIdx.x] = v[0];
}

// One wave: first the previous step's end (t += tau, the step count, the stop
// at t_end or on an error) when a.pending, then beta (max over the wave-speed
// partials) and tau_max and tau of this step.  Every lane reads the slot and
// computes the same values; the last lane writes them.
__global__ void __launch_bounds__(WAVE) k_nu_dt(NuArgs a) {
    Slot *s = a.slot;
    Slot v = *s;
    long long inc = 0;
    if (a.pending && !v.done) {
        inc = 1;
        v.t = v.last ? a.t_end : v.t + v.tau;
        if (v.last) v.done = 1;
        v.done |= 2 * (a.err[0] | a.err[1] | a.err[2]);
    }
    double b = 0.0;
    for (int j = threadIdx.x; j < 2 * a.nblk; j += WAVE) b = fmax(b, a.wpart[j]);
    b = wave_reduce(1, b);
    if (threadIdx.x != WAVE - 1) return;
    *a.nexec += inc;
    if (!v.done && v.t >= a.t_end) v.done = 1;
    if (!v.done) {
        double tau_max = a.dt_fixed;
        if (!(a.dt_fixed > 0.0)) {
            if (!(b > 0.0) || !isfinite(b)) {
                a.err[2] = 1;
                v.done = 1;
            }
            tau_max = a.cfl * a.hmax / b;
        }
        if (!v.done) {
            double tau = tau_max;
            v.last = 0;
            if (v.t + tau >= a.t_end) { tau = a.t_end - v.t; v.last = 1; }
            v.tau = tau;
            v.tau_max = tau_max;
        }
    }
    *s = v;
}

// The end of the last step of a call (the others end in the next k_nu_dt).
__global__ void k_nu_advance(NuArgs a) {
    Slot *s = a.slot;
    if (s->done) return;
    *a.nexec += 1;
    s->t = s->last ? a.t_end : s->t + s->tau;
    if (s->last) s->done = 1;
    s->done |= 2 * (a.err[0] | a.err[1] | a.err[2]);
}

// Operator of eq:1D_H on cell i of mesh M, combined with u^n, and the block's
// statistics of the undamped result.
template <int K, int FLUX>
__global__ void __launch_bounds__(NB) k_nu_stage(NuArgs a) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1, Q = K + 1, NV = 3 * NC;
    constexpr ct::Gauss<Q> G = ct::gauss<Q>();
    __shared__ double sh[NV * NB];
    const int M = blockIdx.y, i = blockIdx.x * NB + threadIdx.x;
    const bool live = i < a.n && !a.slot->done;
    double st[NV];
    int kind[NV];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        kind[3 * q] = 0, kind[3 * q + 1] = 1, kind[3 * q + 2] = 2;
        st[3 * q] = 0.0, st[3 * q + 1] = -INFINITY, st[3 * q + 2] = INFINITY;
    }
    if (live) {
        const double tau = a.slot->tau, itm = 1.0 / a.slot->tau_max;
        const double *own = M == 0 ? a.ulC : a.ulD, *oth = M == 0 ? a.ulD : a.ulC;
        const double c = M == 0 ? a.cC[i] : a.cD[i], w = M == 0 ? a.wC[i] : a.wD[i];
        double lo, split, hi;
        pieces(a, M, i, lo, split, hi);
        double u[NC][K1], nb[2][NC][K1], cnb[2], wnb[2];
        load_cell<K, NC>(own, a.n, i, u);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int j;
            neighbour(a, M, i, p, j, cnb[p], wnb[p]);
            load_cell<K, NC>(oth, a.n, j, nb[p]);
        }
        double R[NC][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) R[q][m] = 0.0;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const double x0 = p == 0 ? lo : split, x1 = p == 0 ? split : hi;
#pragma unroll
            for (int g = 0; g < Q; ++g) {
                const double x = 0.5 * (x0 + x1) + 0.5 * (x1 - x0) * G.s[g], jac = 0.5 * (x1 - x0) * G.w[g];
                const double xi = 2.0 * (x - c) / w, xn = 2.0 * (x - cnb[p]) / wnb[p];
                double v[NC], uk[NC], fv[NC];
                eval<K, NC>(nb[p], 0, xn, 1.0, v);
                eval<K, NC>(u, 0, xi, 1.0, uk);
                F::f(v, fv, a.p0);
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int m = 0; m < K1; ++m)
                        R[q][m] += jac * ((v[q] - uk[q]) * itm * legr(m, 0, xi) + fv[q] * (2.0 / w) * legr(m, 1, xi));
            }
        }
        double vl[NC], vr[NC], fl[NC], fr[NC];
        eval<K, NC>(nb[0], 0, 2.0 * (lo - cnb[0]) / wnb[0], 1.0, vl);
        eval<K, NC>(nb[1], 0, 2.0 * (hi - cnb[1]) / wnb[1], 1.0, vr);
        F::f(vl, fl, a.p0);
        F::f(vr, fr, a.p0);
        const double *un = M == 0 ? a.unC : a.unD;
        double *out = M == 0 ? a.tC : a.tD;
        double o[NC][K1];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                const double sgn = (m % 2 == 0) ? 1.0 : -1.0;
                const double Lm = (2.0 * m + 1.0) / w * (R[q][m] - (fr[q] - fl[q] * sgn));
                const long long e = (long long)(q * K1 + m) * a.n + i;
                const double base = a.cn != 0.0 ? a.cn * un[e] : 0.0;
                o[q][m] = base + (a.cw * u[q][m] + tau * a.dd * Lm);
                out[e] = o[q][m];
            }
        // statistics of the undamped result: width-weighted sum of the averages,
        // max and min at the ends and the quadrature nodes of both pieces
#pragma unroll
        for (int q = 0; q < NC; ++q) st[3 * q] = w * o[q][0];
        double xs[2 * Q + 2];
        xs[0] = lo;
        xs[2 * Q + 1] = hi;
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            xs[1 + g] = 0.5 * (lo + split) + 0.5 * (split - lo) * G.s[g];
            xs[1 + Q + g] = 0.5 * (split + hi) + 0.5 * (hi - split) * G.s[g];
        }
#pragma unroll
        for (int j = 0; j < 2 * Q + 2; ++j) {
            double v[NC];
            eval<K, NC>(o, 0, 2.0 * (xs[j] - c) / w, 1.0, v);
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                st[3 * q + 1] = fmax(st[3 * q + 1], v[q]);
                st[3 * q + 2] = fmin(st[3 * q + 2], v[q]);
            }
        }
    }
    block_reduce<NV>(st, kind, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < NV; ++r) a.part[((long long)M * NV + r) * a.nblk + blockIdx.x] = st[r];
    }
}

// avg and sigma of both meshes ([mesh][q] in avg, sig) from the block
// partials: strided accumulation, a DPP tree per wave, then the waves in
// order; every workgroup gets the same bits.  All threads must take part.
template <int NC>
__device__ inline void nu_statistics(const NuArgs &a, double *sh, double (&avg)[2][NC], double (&sig)[2][NC]) {
    constexpr int NV = 3 * NC, NW = NB / WAVE;
    const int t = threadIdx.x, lane = t % WAVE, wave = t / WAVE;
    // first partial of every row per thread: unconditional loads of valid
    // elements and a select, so that all 2 NV loads are in flight together
    double v[2 * NV];
    const int b0 = min(t, a.nblk - 1);
#pragma unroll
    for (int j = 0; j < 2 * NV; ++j) {
        const double x = a.part[(long long)j * a.nblk + b0];
        v[j] = t < a.nblk ? x : stat_identity(j % 3);
    }
    for (int b = t + NB; b < a.nblk; b += NB) {     // meshes of more than NB * NB cells
#pragma unroll
        for (int j = 0; j < 2 * NV; ++j) v[j] = stat_op(j % 3, v[j], a.part[(long long)j * a.nblk + b]);
    }
#pragma unroll
    for (int j = 0; j < 2 * NV; ++j) {
        v[j] = wave_reduce(j % 3, v[j]);
        if (lane == WAVE - 1) sh[j * NW + wave] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int M = 0; M < 2; ++M)
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            double v[3];
#pragma unroll
            for (int kd = 0; kd < 3; ++kd) {
                const int r = 3 * q + kd;
                v[kd] = sh[(M * NV + r) * NW];
                for (int w = 1; w < NW; ++w) v[kd] = stat_op(kd, v[kd], sh[(M * NV + r) * NW + w]);
            }
            avg[M][q] = v[0] / a.L;
            sig[M][q] = fmax(v[1] - avg[M][q], avg[M][q] - v[2]);
        }
}

// delta_K^m from the undamped stage output, then F_tau into the stage output.
template <int K, int FLUX>
__global__ void __launch_bounds__(NB) k_nu_oe(NuArgs a) {
    using F = FluxT<FLUX>;
    constexpr int NC = F::NC, K1 = K + 1;
    __shared__ double sh[2 * 3 * NC * (NB / WAVE)];
    const int M = blockIdx.y, i = blockIdx.x * NB + threadIdx.x;
    if (a.slot->done) return;            // uniform over the grid
    double avg[2][NC], sigall[2][NC];
    if (a.oe && K > 0) nu_statistics<NC>(a, sh, avg, sigall);
    double bw = 0.0;                     // wave speed at the damped cell average (last stage)
    if (i < a.n) {
        const double *own = M == 0 ? a.tC : a.tD, *oth = M == 0 ? a.tD : a.tC;
        double *dst = M == 0 ? a.oC : a.oD;
        double u[NC][K1];
        load_cell<K, NC>(own, a.n, i, u);
        if (a.oe && K > 0) {
            const double tau = a.slot->tau;
            const double c = M == 0 ? a.cC[i] : a.cD[i], w = M == 0 ? a.wC[i] : a.wD[i];
            double lo, split, hi;
            pieces(a, M, i, lo, split, hi);
            double nb[2][NC][K1], cnb[2], wnb[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                int j;
                neighbour(a, M, i, p, j, cnb[p], wnb[p]);
                load_cell<K, NC>(oth, a.n, j, nb[p]);
            }
            double ub[NC], sig[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) ub[q] = u[q][0], sig[q] = sigall[M][q];
            const double beta = F::speed(ub, a.p0);
            double S = 0.0, fact = 1.0, wp = 1.0 / w;         // w^{m-1}
#pragma unroll
            for (int m = 0; m <= K; ++m) {
                if (m > 1) fact *= m;
                const double so = pow(2.0 / w, m), sl = pow(2.0 / wnb[0], m), sr = pow(2.0 / wnb[1], m);
                double oL[NC], oR[NC], vL[NC], vR[NC];
                eval<K, NC>(u, m, 2.0 * (lo - c) / w, so, oL);
                eval<K, NC>(u, m, 2.0 * (hi - c) / w, so, oR);
                eval<K, NC>(nb[0], m, 2.0 * (lo - cnb[0]) / wnb[0], sl, vL);
                eval<K, NC>(nb[1], m, 2.0 * (hi - cnb[1]) / wnb[1], sr, vR);
                const double cm = (2.0 * m + 1.0) * wp / ((2.0 * K - 1.0) * fact);
                double dm = 0.0;
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    if (sig[q] == 0.0) continue;
                    const double val = cm * beta * (fabs(oL[q] - vL[q]) + fabs(oR[q] - vR[q])) / sig[q];
                    dm = fmax(dm, val);
                }
                S += dm;
                wp *= w;
                if (m >= 1) {
                    const double fac = exp(-tau * S);
#pragma unroll
                    for (int q = 0; q < NC; ++q) u[q][m] *= fac;
                }
            }
        }
        bool finite = true;
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int m = 0; m < K1; ++m) {
                finite = finite && isfinite(u[q][m]);
                dst[(long long)(q * K1 + m) * a.n + i] = u[q][m];
            }
        double ub[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) ub[q] = u[q][0];
        if (!finite) __hip_atomic_store(&a.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!F::physical(ub, a.p0)) __hip_atomic_store(&a.err[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a.wave_out) {
            bw = F::speed(ub, a.p0);
            if (!(bw >= 0.0)) bw = INFINITY;             // NaN: reported by k_nu_dt
        }
    }
    // the next step's beta: per-workgroup maxima of the damped averages (every
    // thread of the workgroup reaches this point)
    if (a.wave_out) {
        __shared__ double shw[NB / WAVE];
        bw = wave_reduce(1, bw);
        if (threadIdx.x % WAVE == WAVE - 1) shw[threadIdx.x / WAVE] = bw;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = shw[0];
            for (int w = 1; w < NB / WAVE; ++w) b = fmax(b, shw[w]);
            a.wpart[M * a.nblk + blockIdx.x] = b;
        }
    }
}

struct NuState {
    int n = 0, nc = 0, k = 0;
    double *geo = nullptr;          // edges [n+1] | cC | wC | cD | wD
    double *buf = nullptr;          // S1 (C|D) | S2 (C|D) | T (C|D)
    double *part = nullptr, *wpart = nullptr;
    Slot *slot = nullptr;
    long long *nexec = nullptr;
    int *err = nullptr;
    long long *nexec_h = nullptr;
    Slot *slot_h = nullptr;
    int *err_h = nullptr;
    // POLL steps after the first, captured once per (state arrays, t_end, fixed step, h_max)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *g_uC = nullptr, *g_uD = nullptr;
    double g_tend = 0.0, g_dt = 0.0, g_hmax = 0.0;
};

void free_state(NuState *s) {
    if (!s) return;
    (void)hipFree(s->geo);
    (void)hipFree(s->buf);
    (void)hipFree(s->part);
    (void)hipFree(s->wpart);
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

template <int K, int FLUX>
void launch_stage(const NuArgs &a, dim3 grid, hipStream_t st) {
    hipLaunchKernelGGL((k_nu_stage<K, FLUX>), grid, dim3(NB), 0, st, a);
}
template <int K, int FLUX>
void launch_oe(const NuArgs &a, dim3 grid, hipStream_t st) {
    hipLaunchKernelGGL((k_nu_oe<K, FLUX>), grid, dim3(NB), 0, st, a);
}

template <int FLUX>
void launch_step_kernels(int which, const NuArgs &a, dim3 grid, hipStream_t st) {
    // which: 0 stage, 1 oe
    switch (a.k) {
    case 0: which == 0 ? launch_stage<0, FLUX>(a, grid, st) : launch_oe<0, FLUX>(a, grid, st); break;
    case 1: which == 0 ? launch_stage<1, FLUX>(a, grid, st) : launch_oe<1, FLUX>(a, grid, st); break;
    case 2: which == 0 ? launch_stage<2, FLUX>(a, grid, st) : launch_oe<2, FLUX>(a, grid, st); break;
    default: which == 0 ? launch_stage<3, FLUX>(a, grid, st) : launch_oe<3, FLUX>(a, grid, st); break;
    }
}

void launch_kind(int which, const NuArgs &a, dim3 grid, hipStream_t st) {
    if (a.flux == OECDG_FLUX_ADVECTION) launch_step_kernels<0>(which, a, grid, st);
    else if (a.flux == OECDG_FLUX_BURGERS) launch_step_kernels<1>(which, a, grid, st);
    else launch_step_kernels<2>(which, a, grid, st);
}

void launch_wave(const NuArgs &a, dim3 grid, hipStream_t st) {
    if (a.flux == OECDG_FLUX_ADVECTION) hipLaunchKernelGGL(k_nu_wave<0>, grid, dim3(NB), 0, st, a);
    else if (a.flux == OECDG_FLUX_BURGERS) hipLaunchKernelGGL(k_nu_wave<1>, grid, dim3(NB), 0, st, a);
    else hipLaunchKernelGGL(k_nu_wave<2>, grid, dim3(NB), 0, st, a);
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
    const int nblk = (n + NB - 1) / NB;
    const size_t S1 = (size_t)nc * K1 * n;      // one mesh
    if (!s) {
        s = new NuState();
        s->n = n, s->nc = nc, s->k = k;
        handle_extnu(h) = s;
        if (hipMalloc(&s->geo, sizeof(double) * (5 * (size_t)n + 1)) != hipSuccess ||
            hipMalloc(&s->buf, sizeof(double) * 6 * S1) != hipSuccess ||
            hipMalloc(&s->part, sizeof(double) * 2 * 9 * (size_t)nblk) != hipSuccess ||
            hipMalloc(&s->wpart, sizeof(double) * 2 * (size_t)nblk) != hipSuccess ||
            hipMalloc(&s->slot, sizeof(Slot)) != hipSuccess || hipMalloc(&s->err, sizeof(int) * 4) != hipSuccess ||
            hipMalloc(&s->nexec, sizeof(long long)) != hipSuccess ||
            hipHostMalloc(&s->nexec_h, sizeof(long long)) != hipSuccess ||
            hipHostMalloc(&s->slot_h, sizeof(Slot)) != hipSuccess ||
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
    NUCHK(h, hipMemcpyAsync(s->geo, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, st));
    Slot s0{0.0, 0.0, 0.0, 0, 0};
    NUCHK(h, hipMemcpyAsync(s->slot, &s0, sizeof(Slot), hipMemcpyHostToDevice, st));
    NUCHK(h, hipMemsetAsync(s->err, 0, sizeof(int) * 4, st));
    NUCHK(h, hipMemsetAsync(s->nexec, 0, sizeof(long long), st));

    NuArgs a{};
    a.n = n, a.k = k, a.flux = d.flux, a.oe = d.oe;
    a.L = L, a.hmax = hmax, a.cfl = d.cfl, a.t_end = t_end, a.dt_fixed = dt_fixed;
    a.p0 = d.flux_param[0];                      // advection speed or gamma
    a.edges = s->geo, a.cC = s->geo + n + 1, a.wC = a.cC + n, a.cD = a.wC + n, a.wD = a.cD + n;
    a.part = s->part, a.wpart = s->wpart, a.slot = s->slot, a.nexec = s->nexec, a.err = s->err, a.nblk = nblk;
    double *S1C = s->buf, *S1D = S1C + S1, *S2C = S1D + S1, *S2D = S2C + S1, *TC = S2D + S1, *TD = TC + S1;
    a.tC = TC, a.tD = TD;
    const dim3 grid(nblk, 2);
    const int ns = rk == 1 ? 1 : rk == 2 ? 2 : 3;
    // the kernels of one step; every step after the first has the same arguments
    auto enqueue_step = [&](bool first, hipStream_t q) {
        NuArgs b = a;
        b.unC = uC, b.unD = uD;
        if (first) launch_wave(b, grid, q);          // later steps: written by the last stage's k_nu_oe
        b.pending = !first;
        hipLaunchKernelGGL(k_nu_dt, dim3(1), dim3(WAVE), 0, q, b);
        for (int l = 0; l < ns; ++l) {
            const RKStage r = rk_stage(rk, l);
            b.cn = l == 0 ? 0.0 : r.cn, b.cw = r.cw, b.dd = r.d;
            b.ulC = l == 0 ? uC : (l == 1 ? S1C : S2C);
            b.ulD = l == 0 ? uD : (l == 1 ? S1D : S2D);
            const bool lastst = l == ns - 1;
            b.wave_out = lastst;
            b.oC = lastst ? uC : (l == 0 ? S1C : S2C);
            b.oD = lastst ? uD : (l == 0 ? S1D : S2D);
            launch_kind(0, b, grid, q);
            launch_kind(1, b, grid, q);
        }
    };
    // whole blocks of POLL steps (from a multiple of POLL) replay a captured graph
    if (s->gexec && (s->g_uC != uC || s->g_uD != uD || s->g_tend != t_end || s->g_dt != dt_fixed || s->g_hmax != hmax))
        (void)hipGraphExecDestroy(s->gexec), s->gexec = nullptr;
    auto ensure_graph = [&]() -> int {
        if (s->gexec) return OECDG_OK;
        if (!s->cap) NUCHK(h, hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        NUCHK(h, hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < POLL; ++j) enqueue_step(false, s->cap);
        NUCHK(h, hipStreamEndCapture(s->cap, &gr));
        const hipError_t e = hipGraphInstantiate(&s->gexec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        NUCHK(h, e);
        s->g_uC = uC, s->g_uD = uD, s->g_tend = t_end, s->g_dt = dt_fixed, s->g_hmax = hmax;
        return OECDG_OK;
    };
    int64_t step = 0;
    while (nsteps < 0 || step < nsteps) {
        if (step > 0 && step % POLL == 0 && !std::isinf(t_end)) {
            NUCHK(h, hipMemcpyAsync(s->slot_h, s->slot, sizeof(Slot), hipMemcpyDeviceToHost, st));
            NUCHK(h, hipStreamSynchronize(st));
            if (s->slot_h->done) break;
        }
        if (step > 0 && step % POLL == 0 && (nsteps < 0 || nsteps - step >= POLL)) {
            const int rc = ensure_graph();
            if (rc != OECDG_OK) return rc;
            NUCHK(h, hipGraphLaunch(s->gexec, st));
            step += POLL;
        } else {
            enqueue_step(step == 0, st);
            ++step;
        }
        NUCHK(h, hipGetLastError());
    }
    if (step > 0) hipLaunchKernelGGL(k_nu_advance, dim3(1), dim3(1), 0, st, a);
    NUCHK(h, hipGetLastError());
    NUCHK(h, hipMemcpyAsync(s->slot_h, s->slot, sizeof(Slot), hipMemcpyDeviceToHost, st));
    NUCHK(h, hipMemcpyAsync(s->err_h, s->err, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    NUCHK(h, hipMemcpyAsync(s->nexec_h, s->nexec, sizeof(long long), hipMemcpyDeviceToHost, st));
    NUCHK(h, hipStreamSynchronize(st));
    if (s->err_h[2]) return handle_fail(h, OECDG_EINVAL, "wave speed is zero or not finite");
    if (s->err_h[0]) return handle_fail(h, OECDG_ENONFINITE, "non-finite coefficient");
    if (s->err_h[1]) return handle_fail(h, OECDG_ENONPHYSICAL, "non-physical cell average");
    if (t_out) *t_out = s->slot_h->t;
    if (steps_out) *steps_out = *s->nexec_h;
    return OECDG_OK;
}

}  // namespace oecdg
