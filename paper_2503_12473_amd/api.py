"""Python front end of the OECDG library: torch tensors in, C ABI calls out.

Tensors must be float64, contiguous and on the GPU; their data pointers and
the current HIP stream are passed to liboecdg.so.  Nothing here computes any
part of the method.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Sequence

import torch

from . import _lib
from ._lib import Desc, OECDGError, check
from .inputs import Problem1D, Problem2D, FLUX_EULER, BC_INFLOW


def make_desc(prob, cfl: float, oe: bool = True, rk: int = 3) -> Desc:
    d = Desc()
    if isinstance(prob, Problem1D):
        d.dim, d.ny, d.ylo, d.yhi = 1, 1, 0.0, 1.0
        d.nx = prob.n
        d.bc = prob.bc
        d.flux_param[0] = prob.gamma if prob.flux == FLUX_EULER else prob.a
        d.flux_param[1] = 0.0
    elif isinstance(prob, Problem2D):
        d.dim, d.nx, d.ny, d.ylo, d.yhi = 2, prob.nx, prob.ny, prob.ylo, prob.yhi
        d.bc = 0
        if prob.flux == FLUX_EULER:
            d.flux_param[0], d.flux_param[1] = prob.gamma, 0.0
        else:
            d.flux_param[0], d.flux_param[1] = prob.a, prob.b
    else:
        raise TypeError("prob must be a Problem1D or Problem2D")
    d.k, d.flux, d.xlo, d.xhi = prob.k, prob.flux, prob.xlo, prob.xhi
    d.cfl = float(cfl)
    d.oe = 1 if oe else 0
    d.rk = int(rk)
    d.space = int(getattr(prob, "space", 0))
    d.flags = _lib.FLAG_ALLOW_NEGATIVE_PRESSURE if getattr(prob, "allow_negative_pressure", False) else 0
    return d


def _ptr(t: torch.Tensor | None, name: str) -> int | None:
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    return t.data_ptr()


class OECDG:
    """A handle of the C library for one problem or a batch of 1D problems.

    rk selects the time integrator: 3 SSP-RK3 (default), 1 forward Euler,
    2 SSP-RK2, 4 classical RK4 (1D only for rk != 3)."""

    def __init__(self, probs, cfl, oe: bool = True, stream: torch.cuda.Stream | None = None, rk: int = 3):
        if not isinstance(probs, (list, tuple)):
            probs = [probs]
        cfls = cfl if isinstance(cfl, (list, tuple)) else [cfl] * len(probs)
        self.probs = list(probs)
        self.rk = 3 if rk == 0 else int(rk)
        self._L = _lib.lib()
        arr = (Desc * len(probs))(*[make_desc(p, c, oe, rk) for p, c in zip(probs, cfls)])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = self._L.oecdg_init(arr, len(probs), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        check(rc, None, "oecdg_init")
        self._h = h
        n = len(probs)
        offC = (C.c_int64 * (n + 1))()
        offD = (C.c_int64 * (n + 1))()
        check(self._L.oecdg_batch_offsets(self._h, offC, offD), self._h, "oecdg_batch_offsets")
        self.off_primal = list(offC)
        self.off_dual = list(offD)
        for b, p in enumerate(probs):
            if isinstance(p, Problem1D) and p.bc == BC_INFLOW and p.inflow:
                left = (C.c_double * 3)(*[float(v) for v in p.inflow[0]])
                right = (C.c_double * 3)(*[float(v) for v in p.inflow[1]])
                check(self._L.oecdg_set_inflow(self._h, b, left, right), self._h, "oecdg_set_inflow")

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._L.oecdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def set_option(self, key: int, value: int):
        check(self._L.oecdg_set_option(self._h, key, int(value)), self._h, "oecdg_set_option")

    def sizes(self):
        return self.off_primal[-1], self.off_dual[-1]

    def empty_state(self, device="cuda"):
        nC, nD = self.sizes()
        return (torch.empty(nC, dtype=torch.float64, device=device),
                torch.empty(nD, dtype=torch.float64, device=device))

    def dt(self, uC: torch.Tensor, uD: torch.Tensor) -> float:
        out = C.c_double()
        check(self._L.oecdg_dt(self._h, _ptr(uC, "uC"), _ptr(uD, "uD"), C.byref(out)), self._h, "oecdg_dt")
        return out.value

    def stage(self, stage: int, dt: float, tau_max: float, uC_n, uD_n, uC_l=None, uD_l=None, out=None):
        if out is None:
            out = (torch.empty_like(uC_n), torch.empty_like(uD_n))
        rc = self._L.oecdg_stage(self._h, stage, dt, tau_max, _ptr(uC_n, "uC_n"), _ptr(uD_n, "uD_n"),
                                 _ptr(uC_l, "uC_l"), _ptr(uD_l, "uD_l"), _ptr(out[0], "outC"), _ptr(out[1], "outD"))
        check(rc, self._h, "oecdg_stage")
        return out

    def run(self, uC: torch.Tensor, uD: torch.Tensor, t_end: float = math.inf, nsteps: int = -1,
            dt_fixed: float = 0.0):
        """Advance in place; returns (t, steps) of instance 0."""
        t = C.c_double()
        n = C.c_int64()
        rc = self._L.oecdg_run(self._h, _ptr(uC, "uC"), _ptr(uD, "uD"), float(t_end), int(nsteps),
                               float(dt_fixed), C.byref(t), C.byref(n))
        check(rc, self._h, "oecdg_run")
        return t.value, n.value

    def run_nonuniform(self, edges, uC: torch.Tensor, uD: torch.Tensor, t_end: float = math.inf, nsteps: int = -1,
                       dt_fixed: float = 0.0):
        """oecdg_run on the periodic mesh with primal edges `edges` (host, nx+1
        values); advances in place and returns (t, steps)."""
        import numpy as np
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        if e.ndim != 1 or e.size != self.probs[0].n + 1:
            raise ValueError(f"edges must be a 1-D array of nx + 1 = {self.probs[0].n + 1} values, got shape {e.shape}")
        t = C.c_double()
        n = C.c_int64()
        rc = self._L.oecdg_run_nonuniform(self._h, C.c_void_p(e.ctypes.data), _ptr(uC, "uC"), _ptr(uD, "uD"),
                                          float(t_end), int(nsteps), float(dt_fixed), C.byref(t), C.byref(n))
        check(rc, self._h, "oecdg_run_nonuniform")
        return t.value, n.value

    def adjoint(self, uC0, uD0, nsteps: int, dt: float, gC_T, gD_T, checkpoint_every: int = 20):
        gC0 = torch.empty_like(uC0)
        gD0 = torch.empty_like(uD0)
        rc = self._L.oecdg_adjoint(self._h, _ptr(uC0, "uC0"), _ptr(uD0, "uD0"), int(nsteps), float(dt),
                                   _ptr(gC_T, "gC_T"), _ptr(gD_T, "gD_T"), _ptr(gC0, "gC0"), _ptr(gD0, "gD0"),
                                   int(checkpoint_every))
        check(rc, self._h, "oecdg_adjoint")
        return gC0, gD0


def to_device(a, device="cuda") -> torch.Tensor:
    """Flatten a modal numpy array into a contiguous float64 GPU tensor."""
    return torch.as_tensor(a, dtype=torch.float64).reshape(-1).contiguous().to(device)
