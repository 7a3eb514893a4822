// oecdg_noalloc.hip -- oecdg_run_noalloc: oecdg_run for one 1D instance with
// no allocation of any kind, for callers that cannot allocate (code under
// graph capture, serving loops that forbid it).  Its stage buffers, damped
// u^n, partial statistics, step records and error flags live in a fixed
// file-scope device array; inputs and outputs are the caller's.
#include "oecdg.h"
#include "oecdg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>

using namespace oecdg;

// Device memory of oecdg_run_noalloc: a file-scope array on every GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (in host code it is only a stand-in for
// the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is kept per device.
static __device__ __align__(256) double scratch[OECDG_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// The current device's copy of the scratch array (nullptr and e set on failure).
double *noalloc_scratch(hipError_t &e) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        e = hipErrorInvalidDevice;
        return nullptr;
    }
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[dev] = g_scratch_err[dev] == hipSuccess ? static_cast<double *>(p) : nullptr;
    });
    e = g_scratch_err[dev];
    return g_scratch[dev];
}

// Carve n elements of T, 256-byte aligned, from the scratch (in doubles).
template <class T>
T *carve(double *base, size_t &used, size_t n) {
    T *p = reinterpret_cast<T *>(base + used);
    used += ((n * sizeof(T) + 255) / 256) * 256 / sizeof(double);
    return p;
}

}  // namespace

extern "C" {

int oecdg_run_noalloc(const oecdg_desc *d, void *stream, double *uC, double *uD, double t_end, int64_t nsteps,
                      double dt_fixed, double *t_out, int64_t *steps_out) {
#define NACHK(expr)                                  \
    do {                                             \
        if ((expr) != hipSuccess) return OECDG_EHIP; \
    } while (0)
    if (!d || !uC || !uD) return OECDG_EINVAL;
    const char *why = "";
    int rc = validate(*d, why);
    if (rc != OECDG_OK) return rc;
    if (d->dim != 1) return OECDG_EUNSUPPORTED;
    if (nsteps < 0 && !(t_end < INFINITY)) return OECDG_EINVAL;
    if (!(t_end > 0.0)) return OECDG_EINVAL;
    // the instance, tiled as oecdg_init tiles a single instance
    Inst1D I = make_inst(*d);
    const int T = default_tile(I.nd, 1);
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 0;
    const long long plain = (I.nd + T - 1) / T, merged = tail_candidate(I, T) ? I.np / T : plain;
    I.tail = plain > ncu && merged <= ncu && merged < plain && tail_candidate(I, T);
    I.ntiles = I.tail ? I.np / T : (I.nd + T - 1) / T;
    I.npart = I.ntiles + (I.tail ? 1 : 0);
    const int rk = d->rk == 0 ? 3 : d->rk;
    int64_t totC = 0, totD = 0;
    sizes(*d, totC, totD);
    // the scratch: stage buffers, damped u^n, RK4 accumulator, partials, step records, flags
    const size_t state = (size_t)(totC + totD);
    const size_t need = 2 * state + state + (rk == 4 ? state : 0) + (size_t)2 * NSTAT * I.npart + 64;
    if (need > OECDG_NOALLOC_SCRATCH_BYTES / sizeof(double)) return OECDG_ETOOBIG;
    hipError_t e;
    double *base = noalloc_scratch(e);
    if (!base) return OECDG_EHIP;
    size_t used = 0;
    double *B = carve<double>(base, used, 2 * state);
    double *U = carve<double>(base, used, state);
    double *A = rk == 4 ? carve<double>(base, used, state) : nullptr;
    double *part = carve<double>(base, used, (size_t)2 * NSTAT * I.npart);
    Slot *slots = carve<Slot>(base, used, 2);
    Final *fin = carve<Final>(base, used, 1);
    int *err = carve<int>(base, used, 4);
    unsigned *bar = carve<unsigned>(base, used, 2);

    StageArgs a;
    memset(&a, 0, sizeof(a));
    a.ntiles = I.npart;
    a.tbeg = 0;
    a.tend = I.ntiles;
    a.slots = slots;
    a.fin = fin;
    a.part[0] = part;
    a.part[1] = part + (size_t)NSTAT * I.npart;
    a.BC[0] = B;
    a.BC[1] = B + totC;
    a.BD[0] = B + 2 * totC;
    a.BD[1] = B + 2 * totC + totD;
    a.UC = U;
    a.UD = U + totC;
    if (A) {
        a.AC = A;
        a.AD = A + totC;
    }
    a.rk = rk;
    a.ns = rk_stages(rk);
    a.tailwave = I.tail;
    a.err = err;
    a.bar = bar;
    a.spin_limit = 1LL << 25;
    a.damp_input = 1;
    a.ninst = 1;
    a.inst0 = I;
    a.t_end = t_end;
    a.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
    const int flux = d->bc == OECDG_BC_REFLECTIVE ? 3 : d->flux;
    hipStream_t s = (hipStream_t)stream;

    NACHK(hipMemcpyAsync(a.BC[0], uC, sizeof(double) * totC, hipMemcpyDeviceToDevice, s));
    NACHK(hipMemcpyAsync(a.BD[0], uD, sizeof(double) * totD, hipMemcpyDeviceToDevice, s));
    NACHK(launch_init_1d(a, 1, s));      // step records, flags: cleared by a kernel
    StageArgs st = a;
    st.srcC = a.BC[0];
    st.srcD = a.BD[0];
    NACHK(launch_stats_1d(st, I.k, flux, T, s));
    Final fh{0.0, 0.0, 0};
    int eh[4] = {0, 0, 0, 0};
    const long long limit = nsteps >= 0 ? nsteps : LLONG_MAX;
    long long n = 0, prev = -1;
    while (n < limit) {
        const long long chunk = std::min<long long>(64, limit - n);
        for (long long j = n; j < n + chunk; ++j)
            for (int l = 0; l < a.ns; ++l) {
                StageArgs b = a;
                b.l = l;
                b.par = (int)(j & 1);
                b.first = j == 0;
                NACHK(launch_stage_1d(b, I.k, flux, T, s));
            }
        n += chunk;
        NACHK(hipMemcpyAsync(&fh, fin, sizeof(Final), hipMemcpyDeviceToHost, s));
        NACHK(hipMemcpyAsync(eh, err, sizeof(eh), hipMemcpyDeviceToHost, s));
        NACHK(hipStreamSynchronize(s));
        if (eh[0] || eh[1] || eh[2] || fh.t >= t_end) break;
        if (fh.nexec == prev) return OECDG_EINVAL;       // no progress
        prev = fh.nexec;
    }
    StageArgs f = a;
    f.dstC = uC;
    f.dstD = uD;
    NACHK(launch_final_1d(f, I.k, flux, T, s));
    NACHK(hipMemcpyAsync(&fh, fin, sizeof(Final), hipMemcpyDeviceToHost, s));
    NACHK(hipMemcpyAsync(eh, err, sizeof(eh), hipMemcpyDeviceToHost, s));
    NACHK(hipStreamSynchronize(s));
#undef NACHK
    if (t_out) *t_out = fh.t;
    if (steps_out) *steps_out = fh.nexec;
    if (eh[2]) return OECDG_ETIMEOUT;
    if (eh[0]) return OECDG_ENONFINITE;
    if (eh[1]) return OECDG_ENONPHYSICAL;
    return OECDG_OK;
}

}  // extern "C"
