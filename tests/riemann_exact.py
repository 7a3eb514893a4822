"""Exact solution of the 1D Euler Riemann problem (ideal gas), test pin.

Written from the classical exact-solver construction (E. F. Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", ch. 4): the star-region
pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock
(Rankine-Hugoniot) or rarefaction (isentropic) branch on each side; the
solution is then sampled along x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:                                   # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk                                   # rarefaction
    val = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    der = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return val, der


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(rl, ul, pl, rr, ur, pr, s, g=1.4):
    """Primitive state (rho, u, p) at similarity coordinate s = (x - x0)/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if s <= us:                                  # left of contact
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sl:
                return rl, ul, pl
            rs = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
            return rs, us, ps
        csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
        if s <= ul - cl:
            return rl, ul, pl
        if s >= us - csl:
            return rl * (ps / pl) ** (1 / g), us, ps
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
        rho = rl * (c / cl) ** (2 / (g - 1))
        return rho, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sr:
            return rr, ur, pr
        rs = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
        return rs, us, ps
    csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
    if s >= ur + cr:
        return rr, ur, pr
    if s <= us + csr:
        return rr * (ps / pr) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
    rho = rr * (c / cr) ** (2 / (g - 1))
    return rho, u, pr * (c / cr) ** (2 * g / (g - 1))


def density(states, x, t, x0=0.5, g=1.4):
    rl, pl, rr, pr = states
    xs = np.asarray(x, dtype=np.float64)
    out = np.empty_like(xs)
    for idx, xv in np.ndenumerate(xs):
        out[idx] = sample(rl, 0.0, pl, rr, 0.0, pr, (xv - x0) / t, g)[0]
    return out
