"""Discrete-adjoint oracle of 1D scalar RK-OECDG (test infrastructure).

The fully discrete scheme (SSP-RK3 in the c/d form of eq:RKCDG with the OE
step F_tau after every stage, Sec. 2.2) for a scalar flux on a periodic
uniform mesh, written in plain PyTorch CPU float64 operations so that
torch.autograd differentiates it exactly.  It follows the same definitions as
the C oracle (per-cell CDG equations equcdg with k+1 Gauss-Legendre nodes on
each half cell; delta_K^m, sigma_K and beta_K of Sec. 2.2) and is pinned to it
by the tests (forward equality) and to finite differences of the C oracle
(gradient).  Non-smooth points use fixed conventions: d|x|/dx = 0 at x = 0
(torch's), the L-infinity norm in sigma is attributed to the first maximiser
in (cell, sample point) order, a vanishing sigma gives delta = 0 with no
derivative, and the time step is fixed (not differentiated).

Only tests and the smoke check use this module.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from numpy.polynomial import legendre as npleg

from paper_2503_12473_amd.inputs import FLUX_ADVECTION, FLUX_BURGERS, BC_PERIODIC

DT = torch.float64


def _leg(n, x, d=0):
    c = [0.0] * n + [1.0]
    return npleg.legval(x, npleg.legder(c, d)) if d else npleg.legval(x, c)


class Scalar1D:
    """Periodic 1D scalar OECDG (advection or Burgers) on torch tensors [k+1, n]."""

    def __init__(self, prob):
        if prob.nc != 1 or prob.bc != BC_PERIODIC or prob.flux not in (FLUX_ADVECTION, FLUX_BURGERS):
            raise ValueError("scalar periodic advection or Burgers only")
        self.p = prob
        k = prob.k
        self.k, self.n, self.h = k, prob.n, prob.h
        s, w = npleg.leggauss(k + 1)
        # per half (0 left, 1 right): own-cell nodes xi, neighbour coordinate xn
        xi = np.stack([(s - 1) / 2, (s + 1) / 2])
        xn = np.stack([xi[0] + 1, xi[1] - 1])
        m = np.arange(k + 1)
        t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), dtype=DT)
        self.Pown = t([[[_leg(j, x) for x in xi[hf]] for j in m] for hf in range(2)])        # [2, k+1, Q]
        self.dPown = t([[[_leg(j, x, 1) for x in xi[hf]] for j in m] for hf in range(2)])
        self.Pnb = t([[[_leg(j, x) for x in xn[hf]] for j in m] for hf in range(2)])
        self.wq = t(w / 2)
        self.P0 = t([_leg(j, 0.0) for j in m])
        self.Dm0 = t([[_leg(j, 0.0, d) for j in m] for d in m])                               # [d, n]
        self.Dp1 = t([[_leg(j, 1.0, d) for j in m] for d in m])
        self.Dm1 = t([[_leg(j, -1.0, d) for j in m] for d in m])
        pts = np.concatenate([[-1.0], xi[0], xi[1], [1.0]])
        self.SP = t([[_leg(j, x) for j in m] for x in pts])                                     # [nsp, k+1]
        self.cdel = t([(2 * d + 1) * self.h ** (d - 1) * (2.0 / self.h) ** d / ((2 * k - 1) * math.factorial(d))
                       for d in m]) if k > 0 else None

    # ---- flux, wave speed
    def f(self, w):
        return self.p.a * w if self.p.flux == FLUX_ADVECTION else 0.5 * w * w

    def speed(self, ubar):
        return torch.full_like(ubar, abs(self.p.a)) if self.p.flux == FLUX_ADVECTION else torch.abs(ubar)

    # ---- neighbours on the other mesh: (left-half cell, right-half cell)
    @staticmethod
    def nb_primal(uD):
        return uD, torch.roll(uD, -1, dims=1)        # dual i, dual i+1

    @staticmethod
    def nb_dual(uC):
        return torch.roll(uC, 1, dims=1), uC         # primal j-1, primal j

    def _rate(self, own, nl, nr, tau_max):
        """equcdg for one mesh: time derivative of the modal coefficients."""
        k, h = self.k, self.h
        coup = torch.zeros_like(own)
        vol = torch.zeros_like(own)
        for hf, nb in ((0, nl), (1, nr)):
            w = torch.einsum("jg,jc->gc", self.Pnb[hf], nb)              # [Q, n]
            uk = torch.einsum("jg,jc->gc", self.Pown[hf], own)
            fw = self.f(w)
            coup = coup + torch.einsum("g,mg,gc->mc", self.wq, self.Pown[hf], w - uk)
            vol = vol + torch.einsum("g,mg,gc->mc", self.wq, self.dPown[hf], fw)
        fl = self.f(self.P0 @ nl)
        fr = self.f(self.P0 @ nr)
        sgn = torch.tensor([(-1.0) ** j for j in range(k + 1)], dtype=DT)
        edge = fr[None, :] - sgn[:, None] * fl[None, :]
        mass = torch.tensor([2 * j + 1.0 for j in range(k + 1)], dtype=DT)[:, None] / h
        return mass * ((0.5 * h / tau_max) * coup + vol - edge)

    def rhs(self, uC, uD, tau_max):
        return (self._rate(uC, *self.nb_primal(uD), tau_max), self._rate(uD, *self.nb_dual(uC), tau_max))

    # ---- OE step
    def _sigma(self, u):
        avg = u[0].mean()
        vals = (self.SP @ u).transpose(0, 1).reshape(-1)      # (cell, sample point) order
        d = torch.abs(vals - avg)
        return d[torch.argmax(d)]                              # first maximiser

    def _delta(self, own, nl, nr, sigma):
        beta = self.speed(own[0])
        dR = self.Dp1 @ own - self.Dm0 @ nr                   # [d, n] xi-derivatives
        dL = self.Dm1 @ own - self.Dm0 @ nl
        num = self.cdel[:, None] * beta[None, :] * (torch.abs(dR) + torch.abs(dL))
        if float(sigma.detach()) == 0.0:
            return torch.zeros_like(num)
        return num / sigma

    def oe(self, uC, uD, tau):
        if self.k == 0:
            return uC, uD
        dC = self._delta(uC, *self.nb_primal(uD), self._sigma(uC))
        dD = self._delta(uD, *self.nb_dual(uC), self._sigma(uD))
        out = []
        for u, d in ((uC, dC), (uD, dD)):
            S = torch.cumsum(d, dim=0)                         # S_j = sum_{m<=j} delta^m
            fac = torch.exp(-tau * S)
            fac = torch.cat([torch.ones_like(fac[:1]), fac[1:]], dim=0)
            out.append(u * fac)
        return out[0], out[1]

    def step(self, uC, uD, tau, tau_max=None, oe=True):
        tm = tau if tau_max is None else tau_max
        F = (lambda a, b: self.oe(a, b, tau)) if oe else (lambda a, b: (a, b))
        LC, LD = self.rhs(uC, uD, tm)
        s1 = F(uC + tau * LC, uD + tau * LD)
        LC, LD = self.rhs(*s1, tm)
        s2 = F(0.75 * uC + 0.25 * (s1[0] + tau * LC), 0.75 * uD + 0.25 * (s1[1] + tau * LD))
        LC, LD = self.rhs(*s2, tm)
        return F(uC / 3.0 + (2.0 / 3.0) * (s2[0] + tau * LC), uD / 3.0 + (2.0 / 3.0) * (s2[1] + tau * LD))

    def run(self, uC, uD, nsteps, tau, checkpoint_every=0, oe=True):
        """nsteps fixed steps (oe=False: plain CDG, no OE step); with
        checkpoint_every > 0 each segment is recomputed in the backward pass
        (torch.utils.checkpoint)."""
        if checkpoint_every <= 0:
            for _ in range(nsteps):
                uC, uD = self.step(uC, uD, tau, oe=oe)
            return uC, uD
        from torch.utils.checkpoint import checkpoint

        def seg(a, b, m):
            for _ in range(m):
                a, b = self.step(a, b, tau, oe=oe)
            return a, b
        done = 0
        while done < nsteps:
            m = min(checkpoint_every, nsteps - done)
            uC, uD = checkpoint(seg, uC, uD, m, use_reentrant=False)
            done += m
        return uC, uD


class _one_thread:
    """The tensors here are small ([k+1, n]); intra-op threading only adds
    contention (tens of times slower with 8 threads), so run on one."""

    def __enter__(self):
        self.n = torch.get_num_threads()
        torch.set_num_threads(1)

    def __exit__(self, *exc):
        torch.set_num_threads(self.n)


def gradient(prob, uC0, uD0, nsteps, tau, gC_T, gD_T, checkpoint_every=20, oe=True):
    """d<gT, u(T)>/du0 for the fixed-step run (numpy in, numpy out); the
    gradient of any loss J is obtained with gT = dJ/du(T).  oe=False: the
    plain CDG scheme."""
    with _one_thread():
        return _gradient(prob, uC0, uD0, nsteps, tau, gC_T, gD_T, checkpoint_every, oe)


def _gradient(prob, uC0, uD0, nsteps, tau, gC_T, gD_T, checkpoint_every, oe=True):
    s = Scalar1D(prob)
    a = torch.tensor(uC0[0], dtype=DT, requires_grad=True)
    b = torch.tensor(uD0[0], dtype=DT, requires_grad=True)
    oC, oD = s.run(a, b, nsteps, tau, checkpoint_every, oe=oe)
    (oC * torch.tensor(gC_T[0], dtype=DT)).sum().add((oD * torch.tensor(gD_T[0], dtype=DT)).sum()).backward()
    return a.grad.numpy()[None].copy(), b.grad.numpy()[None].copy()


def forward(prob, uC0, uD0, nsteps, tau):
    s = Scalar1D(prob)
    with torch.no_grad(), _one_thread():
        oC, oD = s.run(torch.tensor(uC0[0], dtype=DT), torch.tensor(uD0[0], dtype=DT), nsteps, tau)
    return oC.numpy()[None].copy(), oD.numpy()[None].copy()


def misfit_loss_grad(prob, uC, uD, tC, tD):
    """Loss J = 1/2 sum_meshes sum_cells sum_m h/(2m+1) (a_m - t_m)^2 and dJ/du."""
    w = (prob.h / (2.0 * np.arange(prob.k + 1) + 1.0))[None, :, None]
    J = 0.5 * float((w * (uC - tC) ** 2).sum() + (w * (uD - tD) ** 2).sum())
    return J, w * (uC - tC), w * (uD - tD)
