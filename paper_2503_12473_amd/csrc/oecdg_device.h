// oecdg_device.h -- device helpers shared by the forward and adjoint kernels:
// flux functions, shared-state loads, order-fixed DPP reductions and the
// reduction of per-tile partial statistics.
#pragma once

#include "oecdg_internal.h"

#include <math.h>

namespace oecdg {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- fluxes ---

template <int FLUX> struct FluxT;

template <> struct FluxT<0> {          // linear advection f = a u
    static constexpr int NC = 1;
    __device__ static inline void f(const double *w, double *o, double a) { o[0] = a * w[0]; }
    __device__ static inline double speed(const double *, double a) { return fabs(a); }
    __device__ static inline bool physical(const double *, double) { return true; }
};

template <> struct FluxT<1> {          // Burgers f = u^2 / 2
    static constexpr int NC = 1;
    __device__ static inline void f(const double *w, double *o, double) { o[0] = 0.5 * w[0] * w[0]; }
    __device__ static inline double speed(const double *u, double) { return fabs(u[0]); }
    __device__ static inline bool physical(const double *, double) { return true; }
};

template <> struct FluxT<2> {          // Euler (rho, m, E), ideal gas
    static constexpr int NC = 3;
    __device__ static inline void f(const double *w, double *o, double g) {
        const double v = w[1] / w[0];
        const double p = (g - 1.0) * (w[2] - 0.5 * w[1] * v);
        o[0] = w[1];
        o[1] = w[1] * v + p;
        o[2] = (w[2] + p) * v;
    }
    // |v| + sqrt(gamma |p| / rho): |v| + c for every physical state, finite
    // where a tolerated non-positive pressure sits at a cell average
    __device__ static inline double speed(const double *u, double g) {
        const double v = u[1] / u[0];
        const double p = (g - 1.0) * (u[2] - 0.5 * u[1] * v);
        return fabs(v) + sqrt(g * fabs(p) / u[0]);
    }
    __device__ static inline bool physical(const double *u, double g) {
        if (!(u[0] > 0.0)) return false;
        const double p = (g - 1.0) * (u[2] - 0.5 * u[1] * u[1] / u[0]);
        return p > 0.0;
    }
};

// Euler between reflective walls: the same flux; 1D kernels instantiated with
// it also carry the wall-ghost code (the others carry none).
template <> struct FluxT<3> : FluxT<2> {};

// ------------------------------------------------------ shared-state access ---
// Between kernel launches plain loads see the previous kernel's stores.  In
// the persistent launch, values written by other workgroups of the same
// launch are read with device-scope atomic loads after the grid barrier.

__device__ inline double ld_d(const double *p, bool coherent) {
    return coherent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
__device__ inline int ld_i(const int *p, bool coherent) {
    return coherent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
__device__ inline long long ld_ll(const long long *p, bool coherent) {
    return coherent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
__device__ inline Slot ld_slot(const Slot *p, bool coherent) {
    Slot s;
    s.t = ld_d(&p->t, coherent);
    s.tau = ld_d(&p->tau, coherent);
    s.tau_max = ld_d(&p->tau_max, coherent);
    s.done = ld_i(&p->done, coherent);
    s.last = ld_i(&p->last, coherent);
    return s;
}

// ------------------------------------------------------ tiles and XCDs ---
// Workgroup b of a launch over n tiles -> its tile (offset from the first).
// Workgroups are dealt to the 8 XCDs in turn (XCD b mod 8), so XCD x gets
// the band of consecutive tiles that starts at x*q + min(x, r) (q = n / 8,
// r = n mod 8; a bijection on [0, n)).  Neighbouring tiles read the cache
// lines at their common edge (planes whose length is not a multiple of 16
// doubles share a line at every tile edge); in one band they fetch them into
// one L2.
__device__ inline int xcd_tile(int b, int n) {
    const int x = b & 7, j = b >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------------- reductions ---

__device__ inline int stat_kind(int j) { return j >= ST_BETA ? 1 : j % 3; }

__device__ inline double stat_identity(int kind) {
    return kind == 0 ? 0.0 : (kind == 1 ? -INFINITY : INFINITY);
}

// Maximum and minimum of two doubles as the bare v_max_f64 / v_min_f64.
// fmax and fmin first canonicalize each operand that the compiler cannot prove
// canonical (every DPP move and every load: one more dependent instruction per
// level of a reduction tree).  For all inputs except signalling NaNs, which no
// arithmetic here produces, the bare instruction returns what fmax and fmin
// return.
__device__ inline double max_d(double x, double y) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
    return r;
}
__device__ inline double min_d(double x, double y) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
    return r;
}

__device__ inline double stat_op(int kind, double x, double y) {
    return kind == 0 ? x + y : (kind == 1 ? max_d(x, y) : min_d(x, y));
}

// Cross-lane data movement with DPP (plain VALU operations, no LDS round
// trip).  A 64-bit value moves as two 32-bit halves; lanes that the control
// does not write keep `old`.
template <int CTRL, int ROWMASK = 0xf>
__device__ inline double dpp_d(double v, double old) {
    const long long x = __builtin_bit_cast(long long, v), o = __builtin_bit_cast(long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// A lane permutation that writes every lane (quad_perm, row mirrors): no
// "old" operand, so none is copied.  Every lane of the wave must be active.
template <int CTRL>
__device__ inline double dpp_all(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Value of the partner lane (lane ^ 1).
__device__ inline double pair_swap(double v) { return dpp_all<0xB1>(v); }   // quad_perm [1,0,3,2]

// Reduction over the 64 lanes of a wave in a fixed tree (pairs, quads, half
// rows, rows, then rows 0+1 and 2+3, then all four); the result is in lane 63.
// Every lane of the wave must be active.
__device__ inline double wave_reduce(int kind, double v) {
    const double id = stat_identity(kind);
    v = stat_op(kind, v, dpp_all<0xB1>(v));            // quad_perm [1,0,3,2]
    v = stat_op(kind, v, dpp_all<0x4E>(v));            // quad_perm [2,3,0,1]
    v = stat_op(kind, v, dpp_all<0x141>(v));           // row_half_mirror
    v = stat_op(kind, v, dpp_all<0x140>(v));           // row_mirror
    v = stat_op(kind, v, dpp_d<0x142, 0xa>(v, id));    // row_bcast:15 into rows 1, 3
    v = stat_op(kind, v, dpp_d<0x143, 0xc>(v, id));    // row_bcast:31 into rows 2, 3
    return v;
}

// Rows of the partial statistics a consumer needs: (mesh, q, kind) for the
// NC components, then the two wave-speed rows.
template <int NC>
__device__ inline int stat_row(int i) {
    if (i >= 6 * NC) return ST_BETA + (i - 6 * NC);
    const int mesh = i / (3 * NC), r = i - mesh * 3 * NC;
    return stat_index(mesh, r / 3, r % 3);
}

// Per-tile partial statistics are stored [tile][NSTAT]: the NSTAT values of a
// tile are contiguous (one 160-byte record, read with 16-byte loads).
__device__ inline const double *part_tile(const double *part, long long tile) { return part + tile * NSTAT; }

// Reduction of the per-tile partial statistics of tiles [tile0, tile0+ntiles)
// in a fixed order: per-thread strided accumulation over tiles, a butterfly
// within each wave, then the waves in order.  Split in two so that the loads of
// the first two tiles per thread can be issued together with the kernel's other
// independent loads.  The wave-speed rows take part only when ns = 6 NC + 2.
template <int NC>
struct Partials {
    static constexpr int NS = 6 * NC + 2;
    double v[2][NS];
};

// One tile's record into v (consumer order i -> row stat_row<NC>(i)).
template <int NC>
__device__ inline void load_tile_record(const double *rec, double (&v)[Partials<NC>::NS]) {
    double r[NSTAT];
    const double2 *q = reinterpret_cast<const double2 *>(rec);
#pragma unroll
    for (int j = 0; j < NSTAT / 2; ++j) {
        const double2 x = q[j];
        r[2 * j] = x.x;
        r[2 * j + 1] = x.y;
    }
#pragma unroll
    for (int i = 0; i < Partials<NC>::NS; ++i) v[i] = r[stat_row<NC>(i)];
}

// The loads of the first two tiles per thread (t and t + NT, clamped to a valid
// tile; the selects are applied in the reduction, so that no wait follows the
// loads before the kernel's other independent loads are issued).  A wave none
// of whose threads has a second tile skips those loads.
template <int NT, int NC>
__device__ inline void load_partials_raw(const double *part, int tile0, int ntiles, Partials<NC> &p) {
    const int tid = threadIdx.x;
    load_tile_record<NC>(part_tile(part, tile0 + min(tid, ntiles - 1)), p.v[0]);
    if (__builtin_amdgcn_readfirstlane(tid) + NT < ntiles) {
        load_tile_record<NC>(part_tile(part, tile0 + min(tid + NT, ntiles - 1)), p.v[1]);
    } else {
#pragma unroll
        for (int i = 0; i < Partials<NC>::NS; ++i) p.v[1][i] = 0.0;   // not used (tid + NT >= ntiles)
    }
}

// Per-wave part of the reduction: the thread's tiles (selects of the first
// two, the rest strided), then a fixed-order butterfly; lane WAVE-1 writes
// scratch[wave][NS].
template <int NT, int NC>
__device__ inline void wave_partials(const Partials<NC> &p, const double *part, int tile0, int ntiles, int ns,
                                     double *scratch) {
    constexpr int NS = Partials<NC>::NS;
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    double acc[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double id = stat_identity(stat_kind(stat_row<NC>(i)));
        const double x0 = (i < ns && tid < ntiles) ? p.v[0][i] : id;
        const double x1 = (i < ns && tid + NT < ntiles) ? p.v[1][i] : id;
        acc[i] = stat_op(stat_kind(stat_row<NC>(i)), x0, x1);
    }
    for (int t = tid + 2 * NT; t < ntiles; t += NT) {   // more than two tiles per thread
        const double *rec = part_tile(part, tile0 + t);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i < ns) {
                const int j = stat_row<NC>(i);
                acc[i] = stat_op(stat_kind(j), acc[i], rec[j]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[i] = wave_reduce(stat_kind(stat_row<NC>(i)), acc[i]);
    if (lane == WAVE - 1) {
#pragma unroll
        for (int i = 0; i < NS; ++i) scratch[wave * NS + i] = acc[i];
    }
}

// The waves' results combined in order by thread i < NS into red[row] (LDS).
template <int NT, int NC>
__device__ void finish_partials(const Partials<NC> &p, const double *part, int tile0, int ntiles, int ns, double *red,
                                double *scratch) {
    constexpr int NS = Partials<NC>::NS;
    constexpr int NW = (NT + WAVE - 1) / WAVE;
    const int tid = threadIdx.x;
    wave_partials<NT, NC>(p, part, tile0, ntiles, ns, scratch);
    __syncthreads();
    if (tid < NS) {
        const int kd = stat_kind(stat_row<NC>(tid));
        double v = scratch[tid];
        for (int w = 1; w < NW; ++w) v = stat_op(kd, v, scratch[w * NS + tid]);
        red[stat_row<NC>(tid)] = v;
    }
    __syncthreads();
}

// The same reduction, with every thread combining the per-wave results itself
// (the order of finish_partials), so that all of them hold all NSTAT rows (rows
// beyond ns are zero) after one barrier.
template <int NT, int NC>
__device__ void finish_partials_all(const Partials<NC> &p, const double *part, int tile0, int ntiles, int ns,
                                    double (&red)[NSTAT], double *scratch) {
    constexpr int NS = Partials<NC>::NS;
    constexpr int NW = (NT + WAVE - 1) / WAVE;
    wave_partials<NT, NC>(p, part, tile0, ntiles, ns, scratch);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NSTAT; ++i) red[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        if (i < ns) {
            const int kd = stat_kind(stat_row<NC>(i));
            double v = scratch[i];
            for (int w = 1; w < NW; ++w) v = stat_op(kd, v, scratch[w * NS + i]);
            red[stat_row<NC>(i)] = v;
        }
    }
}

template <int NT, int NC>
__device__ void reduce_instance(const double *part, int tile0, int ntiles, bool beta, double *red, double *scratch) {
    const int ns = beta ? Partials<NC>::NS : Partials<NC>::NS - 2;
    Partials<NC> p;
    load_partials_raw<NT, NC>(part, tile0, ntiles, p);
    finish_partials<NT, NC>(p, part, tile0, ntiles, ns, red, scratch);
}

}  // namespace oecdg
