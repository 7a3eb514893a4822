"""ctypes binding of the C oracle (test infrastructure only).

Functions take and return numpy float64 arrays in the modal layouts
[nc, k+1, ncell] (1D) and [nc, k+1, k+1, ny, nx] (2D) used by
``paper_2503_12473_amd.inputs``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ORA_OK = 0
ORA_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -4: "ENONFINITE", -5: "ENONPHYSICAL"}


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} failed: {ORA_ERRORS.get(code, code)}")
        self.code = code


class Ora1D(C.Structure):
    _fields_ = [("k", C.c_int), ("nc", C.c_int), ("flux", C.c_int), ("bc", C.c_int), ("n", C.c_long),
                ("xlo", C.c_double), ("xhi", C.c_double), ("a", C.c_double), ("gamma", C.c_double),
                ("allow_negative_pressure", C.c_int), ("pad", C.c_int), ("inflow", (C.c_double * 3) * 2)]


class Ora2D(C.Structure):
    _fields_ = [("k", C.c_int), ("nc", C.c_int), ("flux", C.c_int), ("nx", C.c_long), ("ny", C.c_long),
                ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
                ("ax", C.c_double), ("ay", C.c_double), ("gamma", C.c_double), ("space", C.c_int)]


_lib = None
_variant = None
_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def use_variant(name=None):
    """Switch to a test-only build variant of the oracle (oracle/build.py
    VARIANTS: different, equally valid FP64 rounding), or back (None)."""
    global _lib, _variant
    if name is not None and name not in _build.VARIANTS:
        raise ValueError(f"unknown oracle variant {name!r}")
    _variant = name
    _lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.lib_path(_variant)
        if not os.path.exists(path):
            _build.build(variant=_variant)
        L = C.CDLL(path)
        P1 = C.POINTER(Ora1D)
        L.ora_legendre.restype = C.c_double
        L.ora_legendre.argtypes = [C.c_int, C.c_double]
        L.ora_legendre_deriv.restype = C.c_double
        L.ora_legendre_deriv.argtypes = [C.c_int, C.c_int, C.c_double]
        L.ora_gauss_legendre.argtypes = [C.c_int, _DP, _DP]
        L.ora1d_rhs.argtypes = [P1, C.c_double, _DP, _DP, _DP, _DP]
        L.ora1d_oe.argtypes = [P1, C.c_double, _DP, _DP]
        L.ora1d_delta.argtypes = [P1, _DP, _DP, _DP, _DP]
        L.ora1d_stats.argtypes = [P1, _DP, _DP, _DP, _DP]
        L.ora1d_stats.restype = None
        L.ora1d_max_wavespeed.argtypes = [P1, _DP, _DP]
        L.ora1d_max_wavespeed.restype = C.c_double
        L.ora1d_step.argtypes = [P1, C.c_int, C.c_int, C.c_double, C.c_double, _DP, _DP]
        L.ora1d_ssprk3_stage.argtypes = [P1, C.c_int, C.c_int, C.c_double, C.c_double, _DP, _DP, _DP, _DP, _DP, _DP]
        L.ora1d_rk_stage.argtypes = [P1, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     _DP, _DP, _DP, _DP, _DP, _DP]
        L.ora1d_run.argtypes = [P1, C.c_double, C.c_int, C.c_int, C.c_double, C.c_long, C.c_double,
                                _DP, _DP, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.ora1n_rhs.argtypes = [P1, _DP, C.c_double, _DP, _DP, _DP, _DP]
        L.ora1n_stats.argtypes = [P1, _DP, _DP, _DP, _DP, _DP]
        L.ora1n_delta.argtypes = [P1, _DP, _DP, _DP, _DP, _DP]
        L.ora1n_oe.argtypes = [P1, _DP, C.c_double, _DP, _DP]
        L.ora1n_step.argtypes = [P1, _DP, C.c_int, C.c_int, C.c_double, C.c_double, _DP, _DP]
        L.ora1n_run.argtypes = [P1, _DP, C.c_double, C.c_int, C.c_int, C.c_double, C.c_long, C.c_double,
                                _DP, _DP, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        P2 = C.POINTER(Ora2D)
        L.ora2d_rhs.argtypes = [P2, C.c_double, _DP, _DP, _DP, _DP]
        L.ora2d_oe.argtypes = [P2, C.c_double, _DP, _DP]
        L.ora2d_delta.argtypes = [P2, _DP, _DP, _DP, _DP]
        L.ora2d_stats.argtypes = [P2, _DP, _DP, _DP, _DP]
        L.ora2d_stats.restype = None
        L.ora2d_max_wavespeeds.argtypes = [P2, _DP, _DP, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ora2d_max_wavespeeds.restype = None
        L.ora2d_wavespeed.argtypes = [P2, C.c_int, _DP]
        L.ora2d_wavespeed.restype = C.c_double
        L.ora2d_step.argtypes = [P2, C.c_int, C.c_int, C.c_double, C.c_double, _DP, _DP]
        L.ora2d_rk_stage.argtypes = [P2, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     _DP, _DP, _DP, _DP, _DP, _DP]
        L.ora2d_run.argtypes = [P2, C.c_double, C.c_int, C.c_int, C.c_double, C.c_long, C.c_double,
                                _DP, _DP, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        _lib = L
    return _lib


def _p1(prob):
    p = Ora1D(prob.k, prob.nc, prob.flux, prob.bc, prob.n, prob.xlo, prob.xhi, prob.a, prob.gamma,
              int(prob.allow_negative_pressure), 0)
    for side in range(2):
        for q, v in enumerate(prob.inflow[side] if prob.inflow else ()):
            p.inflow[side][q] = float(v)
    return p


def _arr(u):
    return np.ascontiguousarray(np.asarray(u, dtype=np.float64))


def _check(rc, where):
    if rc != ORA_OK:
        raise OracleError(rc, where)


def gauss_legendre(Q):
    s = np.zeros(Q)
    w = np.zeros(Q)
    lib().ora_gauss_legendre(Q, s, w)
    return s, w


def legendre(n, x, deriv=0):
    return lib().ora_legendre_deriv(n, deriv, float(x))


def rhs1d(prob, tau_max, uC, uD):
    uC, uD = _arr(uC), _arr(uD)
    LC, LD = np.zeros_like(uC), np.zeros_like(uD)
    _check(lib().ora1d_rhs(C.byref(_p1(prob)), tau_max, uC, uD, LC, LD), "rhs1d")
    return LC, LD


def oe1d(prob, tau, uC, uD):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora1d_oe(C.byref(_p1(prob)), tau, uC, uD), "oe1d")
    return uC, uD


def delta1d(prob, uC, uD):
    uC, uD = _arr(uC), _arr(uD)
    dC = np.zeros((prob.k + 1, prob.n))
    dD = np.zeros((prob.k + 1, prob.n_dual))
    _check(lib().ora1d_delta(C.byref(_p1(prob)), uC, uD, dC, dD), "delta1d")
    return dC, dD


def stats1d(prob, uC, uD):
    """avg, sigma as arrays [mesh, q] (mesh 0 primal, 1 dual)."""
    avg = np.zeros(6)
    sig = np.zeros(6)
    lib().ora1d_stats(C.byref(_p1(prob)), _arr(uC), _arr(uD), avg, sig)
    return avg.reshape(2, 3)[:, :prob.nc], sig.reshape(2, 3)[:, :prob.nc]


def max_wavespeed1d(prob, uC, uD):
    return lib().ora1d_max_wavespeed(C.byref(_p1(prob)), _arr(uC), _arr(uD))


def step1d(prob, tau, tau_max, uC, uD, rk=3, oe=True):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora1d_step(C.byref(_p1(prob)), rk, int(oe), tau, tau_max, uC, uD), "step1d")
    return uC, uD


def ssprk3_stage1d(prob, l, tau, tau_max, unC, unD, ulC, ulD, oe=True):
    """One SSP-RK3 stage l from u^n and u^{n,l}, then F_tau (as the library's oecdg_stage)."""
    unC, unD, ulC, ulD = _arr(unC), _arr(unD), _arr(ulC), _arr(ulD)
    oC, oD = np.zeros_like(unC), np.zeros_like(unD)
    _check(lib().ora1d_ssprk3_stage(C.byref(_p1(prob)), l, int(oe), tau, tau_max, unC, unD, ulC, ulD, oC, oD),
           "ssprk3_stage1d")
    return oC, oD


def rk_stage1d(prob, rk, l, tau, tau_max, unC, unD, ulC, ulD, oe=True):
    """One stage l of RK table rk from u^n and u^{n,l}, then F_tau (stages that
    read only u^n, u^{n,l} and L(u^{n,l}))."""
    unC, unD, ulC, ulD = _arr(unC), _arr(unD), _arr(ulC), _arr(ulD)
    oC, oD = np.zeros_like(unC), np.zeros_like(unD)
    _check(lib().ora1d_rk_stage(C.byref(_p1(prob)), rk, l, int(oe), tau, tau_max, unC, unD, ulC, ulD, oC, oD),
           "rk_stage1d")
    return oC, oD


def run1d(prob, uC, uD, t_end=float("inf"), nsteps=-1, cfl=0.3, dt_fixed=0.0, rk=3, oe=True):
    """March to t_end (clipped last step) or nsteps steps; returns (uC, uD, t, steps)."""
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    t = C.c_double(0.0)
    n = C.c_long(0)
    _check(lib().ora1d_run(C.byref(_p1(prob)), cfl, rk, int(oe), t_end, nsteps, dt_fixed, uC, uD,
                           C.byref(t), C.byref(n)), "run1d")
    return uC, uD, t.value, n.value


# ------------------------------------------------ 1D, non-uniform mesh ---
# edges: the n+1 primal cell edges x_{i-1/2} (edges[0] = xlo, edges[n] = xhi);
# periodic problems only; dual cell j is [x_{j-1}, x_j].

def rhs1n(prob, edges, tau_max, uC, uD):
    uC, uD = _arr(uC), _arr(uD)
    LC, LD = np.zeros_like(uC), np.zeros_like(uD)
    _check(lib().ora1n_rhs(C.byref(_p1(prob)), _arr(edges), tau_max, uC, uD, LC, LD), "rhs1n")
    return LC, LD


def stats1n(prob, edges, uC, uD):
    avg, sig = np.zeros(6), np.zeros(6)
    _check(lib().ora1n_stats(C.byref(_p1(prob)), _arr(edges), _arr(uC), _arr(uD), avg, sig), "stats1n")
    return avg.reshape(2, 3)[:, :prob.nc], sig.reshape(2, 3)[:, :prob.nc]


def delta1n(prob, edges, uC, uD):
    dC, dD = np.zeros((prob.k + 1, prob.n)), np.zeros((prob.k + 1, prob.n))
    _check(lib().ora1n_delta(C.byref(_p1(prob)), _arr(edges), _arr(uC), _arr(uD), dC, dD), "delta1n")
    return dC, dD


def oe1n(prob, edges, tau, uC, uD):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora1n_oe(C.byref(_p1(prob)), _arr(edges), tau, uC, uD), "oe1n")
    return uC, uD


def step1n(prob, edges, tau, tau_max, uC, uD, rk=3, oe=True):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora1n_step(C.byref(_p1(prob)), _arr(edges), rk, int(oe), tau, tau_max, uC, uD), "step1n")
    return uC, uD


def run1n(prob, edges, uC, uD, t_end=float("inf"), nsteps=-1, cfl=0.3, dt_fixed=0.0, rk=3, oe=True):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    t = C.c_double(0.0)
    n = C.c_long(0)
    _check(lib().ora1n_run(C.byref(_p1(prob)), _arr(edges), cfl, rk, int(oe), t_end, nsteps, dt_fixed, uC, uD,
                           C.byref(t), C.byref(n)), "run1n")
    return uC, uD, t.value, n.value


# ---------------------------------------------------------------- 2D ---

def _p2(prob):
    return Ora2D(prob.k, prob.nc, prob.flux, prob.nx, prob.ny, prob.xlo, prob.xhi, prob.ylo, prob.yhi,
                 prob.a, prob.b, prob.gamma, prob.space)


def rhs2d(prob, tau_max, uC, uD):
    uC, uD = _arr(uC), _arr(uD)
    LC, LD = np.zeros_like(uC), np.zeros_like(uD)
    _check(lib().ora2d_rhs(C.byref(_p2(prob)), tau_max, uC, uD, LC, LD), "rhs2d")
    return LC, LD


def oe2d(prob, tau, uC, uD):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora2d_oe(C.byref(_p2(prob)), tau, uC, uD), "oe2d")
    return uC, uD


def delta2d(prob, uC, uD):
    """delta^m of every cell: arrays [k+1, ny, nx] for the primal and dual meshes."""
    uC, uD = _arr(uC), _arr(uD)
    dC = np.zeros((prob.k + 1, prob.ny, prob.nx))
    dD = np.zeros((prob.k + 1, prob.ny, prob.nx))
    _check(lib().ora2d_delta(C.byref(_p2(prob)), uC, uD, dC, dD), "delta2d")
    return dC, dD


def stats2d(prob, uC, uD):
    """avg, sigma as arrays [mesh, q]."""
    avg = np.zeros(8)
    sig = np.zeros(8)
    lib().ora2d_stats(C.byref(_p2(prob)), _arr(uC), _arr(uD), avg, sig)
    return avg.reshape(2, 4)[:, :prob.nc], sig.reshape(2, 4)[:, :prob.nc]


def max_wavespeeds2d(prob, uC, uD):
    bx, by = C.c_double(0.0), C.c_double(0.0)
    lib().ora2d_max_wavespeeds(C.byref(_p2(prob)), _arr(uC), _arr(uD), C.byref(bx), C.byref(by))
    return bx.value, by.value


def step2d(prob, tau, tau_max, uC, uD, rk=3, oe=True):
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    _check(lib().ora2d_step(C.byref(_p2(prob)), rk, int(oe), tau, tau_max, uC, uD), "step2d")
    return uC, uD


def rk_stage2d(prob, rk, l, tau, tau_max, unC, unD, ulC, ulD, oe=True):
    """One stage l of RK table rk from u^n and u^{n,l}, then F_tau (2D; stages
    that read only u^n, u^{n,l} and L(u^{n,l}))."""
    unC, unD, ulC, ulD = _arr(unC), _arr(unD), _arr(ulC), _arr(ulD)
    oC, oD = np.zeros_like(unC), np.zeros_like(unD)
    _check(lib().ora2d_rk_stage(C.byref(_p2(prob)), rk, l, int(oe), tau, tau_max, unC, unD, ulC, ulD, oC, oD),
           "rk_stage2d")
    return oC, oD


def run2d(prob, uC, uD, t_end=float("inf"), nsteps=-1, cfl=0.3, dt_fixed=0.0, rk=3, oe=True):
    """March to t_end (clipped last step) or nsteps steps; returns (uC, uD, t, steps)."""
    uC, uD = _arr(uC).copy(), _arr(uD).copy()
    t = C.c_double(0.0)
    n = C.c_long(0)
    _check(lib().ora2d_run(C.byref(_p2(prob)), cfl, rk, int(oe), t_end, nsteps, dt_fixed, uC, uD,
                           C.byref(t), C.byref(n)), "run2d")
    return uC, uD, t.value, n.value
