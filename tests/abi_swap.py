"""One sequence of calls of the C interface (include/oecdg.h) against either
implementation: the HIP library (oecdg_*, device arrays) or the oracle's
mirror of it (oecdg_ref_*, host arrays; oracle/oecdg_ref.c).

A test writes the call sequence once and runs it on both, then compares the
results.  Only the pointers differ: torch device tensors for the library,
numpy arrays for the oracle.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from paper_2503_12473_amd._lib import Desc
from paper_2503_12473_amd.api import make_desc
from paper_2503_12473_amd.inputs import BC_INFLOW

_REF_BOUND = False


def _bind_ref(L):
    global _REF_BOUND
    if _REF_BOUND:
        return
    H, D, PD, PI = C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    sig = {
        "state_size": ([C.POINTER(Desc), PI, PI], C.c_int),
        "init": ([C.POINTER(Desc), C.c_int32, C.c_void_p, C.POINTER(H)], C.c_int),
        "batch_offsets": ([H, PI, PI], C.c_int),
        "set_option": ([H, C.c_int32, C.c_int64], C.c_int),
        "set_inflow": ([H, C.c_int32, PD, PD], C.c_int),
        "dt": ([H, D, D, PD], C.c_int),
        "stage": ([H, C.c_int32, C.c_double, C.c_double, D, D, D, D, D, D], C.c_int),
        "run": ([H, D, D, C.c_double, C.c_int64, C.c_double, PD, PI], C.c_int),
        "run_noalloc": ([C.POINTER(Desc), C.c_void_p, D, D, C.c_double, C.c_int64, C.c_double, PD, PI], C.c_int),
        "run_nonuniform": ([H, D, D, D, C.c_double, C.c_int64, C.c_double, PD, PI], C.c_int),
        "adjoint": ([H, D, D, C.c_int64, C.c_double, D, D, D, D, C.c_int32], C.c_int),
        "destroy": ([H], None),
        "strerror": ([C.c_int], C.c_char_p),
        "last_error": ([H], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, "oecdg_ref_" + name)
        fn.argtypes = args
        fn.restype = res
    _REF_BOUND = True


class Impl:
    """kind "hip": liboecdg.so on device arrays; kind "ref": the oracle's mirror on host arrays."""

    def __init__(self, kind: str):
        self.kind = kind
        if kind == "hip":
            from paper_2503_12473_amd import _lib
            self.L, self.pre = _lib.lib(), "oecdg_"
        elif kind == "ref":
            from oracle import ora
            self.L, self.pre = ora.lib(), "oecdg_ref_"
            _bind_ref(self.L)
        else:
            raise ValueError(kind)

    def f(self, name):
        return getattr(self.L, self.pre + name)

    def put(self, a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
        if self.kind == "hip":
            import torch
            t = torch.from_numpy(a.copy()).cuda()
            return t, t.data_ptr()
        b = a.copy()
        return b, b.ctypes.data

    def get(self, buf):
        if self.kind == "hip":
            import torch
            torch.cuda.synchronize()
            return buf.cpu().numpy()
        return buf.copy()

    def check(self, rc, h=None, where=""):
        if rc != 0:
            msg = self.f("last_error")(h).decode() if h is not None else ""
            raise AssertionError(f"{self.pre}{where}: code {rc} ({msg})")


def _descs(probs, cfl, oe, rk):
    return (Desc * len(probs))(*[make_desc(p, cfl, oe, rk) for p in probs])


def run(impl: Impl, probs, states, cfl, t_end=math.inf, nsteps=-1, dt_fixed=0.0, rk=3, oe=True, edges=None):
    """init, batch_offsets, set_inflow, dt, run (or run_nonuniform with edges),
    destroy.  states: [(uC, uD)] per instance.  Returns the per-instance
    outputs, t, steps, dt (instance 0) and the offsets."""
    n = len(probs)
    descs = _descs(probs, cfl, oe, rk)
    sizes = []
    for i in range(n):
        npr, ndu = C.c_int64(), C.c_int64()
        impl.check(impl.f("state_size")(C.byref(descs[i]), C.byref(npr), C.byref(ndu)), where="state_size")
        assert (npr.value, ndu.value) == (np.size(states[i][0]), np.size(states[i][1]))
        sizes.append((npr.value, ndu.value))
    bufC, pC = impl.put(np.concatenate([np.ravel(s[0]) for s in states]))
    bufD, pD = impl.put(np.concatenate([np.ravel(s[1]) for s in states]))
    h = C.c_void_p()
    impl.check(impl.f("init")(descs, n, None, C.byref(h)), where="init")
    try:
        offP, offD = (C.c_int64 * (n + 1))(), (C.c_int64 * (n + 1))()
        impl.check(impl.f("batch_offsets")(h, offP, offD), h, "batch_offsets")
        for i, p in enumerate(probs):
            if getattr(p, "bc", None) == BC_INFLOW:
                left, right = (C.c_double * 3)(*p.inflow[0]), (C.c_double * 3)(*p.inflow[1])
                impl.check(impl.f("set_inflow")(h, i, left, right), h, "set_inflow")
        dt = C.c_double()
        impl.check(impl.f("dt")(h, pC, pD, C.byref(dt)), h, "dt")
        t, steps = C.c_double(), C.c_int64()
        if edges is None:
            rc = impl.f("run")(h, pC, pD, t_end, nsteps, dt_fixed, C.byref(t), C.byref(steps))
        else:
            e = np.ascontiguousarray(edges, dtype=np.float64)
            rc = impl.f("run_nonuniform")(h, e.ctypes.data, pC, pD, t_end, nsteps, dt_fixed, C.byref(t),
                                          C.byref(steps))
        impl.check(rc, h, "run")
        outC, outD = impl.get(bufC), impl.get(bufD)
    finally:
        impl.f("destroy")(h)
    offP, offD = list(offP), list(offD)
    per = [(outC[offP[i]:offP[i + 1]].reshape(np.shape(states[i][0])),
            outD[offD[i]:offD[i + 1]].reshape(np.shape(states[i][1]))) for i in range(n)]
    return {"out": per, "t": t.value, "steps": steps.value, "dt": dt.value, "offP": offP, "offD": offD}


def stage(impl: Impl, prob, cfl, rk, l, dt, tau_max, un, ul):
    """One oecdg_stage call on a single-instance handle."""
    descs = _descs([prob], cfl, True, rk)
    bnC, pnC = impl.put(un[0])
    bnD, pnD = impl.put(un[1])
    blC, plC = impl.put(ul[0])
    blD, plD = impl.put(ul[1])
    boC, poC = impl.put(np.zeros(np.size(un[0])))
    boD, poD = impl.put(np.zeros(np.size(un[1])))
    h = C.c_void_p()
    impl.check(impl.f("init")(descs, 1, None, C.byref(h)), where="init")
    try:
        impl.check(impl.f("stage")(h, l, dt, tau_max, pnC, pnD, plC, plD, poC, poD), h, "stage")
        return (impl.get(boC).reshape(np.shape(un[0])), impl.get(boD).reshape(np.shape(un[1])))
    finally:
        impl.f("destroy")(h)


def run_noalloc(impl: Impl, prob, cfl, state, t_end=math.inf, nsteps=-1, dt_fixed=0.0):
    """oecdg_run_noalloc (no handle)."""
    desc = _descs([prob], cfl, True, 3)
    bC, pC = impl.put(state[0])
    bD, pD = impl.put(state[1])
    t, steps = C.c_double(), C.c_int64()
    impl.check(impl.f("run_noalloc")(desc, None, pC, pD, t_end, nsteps, dt_fixed, C.byref(t), C.byref(steps)),
               where="run_noalloc")
    return ((impl.get(bC).reshape(np.shape(state[0])), impl.get(bD).reshape(np.shape(state[1]))),
            t.value, steps.value)
