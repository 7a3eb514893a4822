"""High-precision brute force of the 1D RK-OECDG step for Burgers (test pin).

A few full steps of eq:RKCDG with F_tau after every stage, for f(u) = u^2/2
on a small periodic mesh of width-1 cells, in 40-digit arithmetic (mpmath),
by a route of its own:

- the operator from the bilinear form of eq:1D_H restricted to one basis
  function, with the polynomial integrals done exactly on each half cell (no
  quadrature rule; f(u_h) is formed as a polynomial);
- SSP-RK3 in its convex-combination form (three Euler steps);
- delta_K^m of Sec. 2.2 from x-derivatives of the piecewise polynomials at
  the cell edges, sigma and avg from the cell averages and the sample points
  of both halves (the edges and the Gauss nodes with k+1 points, closed forms);
- F_tau as the matrix exponential of the damping ODE of OEstep2D written in a
  monomial basis with generic L2 projections, not the modal closed form.

Layout of a state: u[mesh][m][cell] (mesh 0 primal cells [i, i+1], mesh 1
dual cells centred on the integers, dual cell 0 centred on 0 = n).
"""
from __future__ import annotations

import math

import mpmath

from tests.exact_cdg import legendre_xi

DPS = 40


def _mp(v):
    """mpf from a float, int or Fraction (exactly)."""
    if hasattr(v, "numerator") and hasattr(v, "denominator") and not isinstance(v, float):
        return mpmath.mpf(v.numerator) / v.denominator
    return mpmath.mpf(v)


# ---- polynomials in x with mpf coefficients, lowest degree first ----

def padd(p, q):
    n = max(len(p), len(q))
    zero = mpmath.mpf(0)
    return [(p[i] if i < len(p) else zero) + (q[i] if i < len(q) else zero) for i in range(n)]


def pscale(p, s):
    return [c * s for c in p]


def pmul(p, q):
    out = [mpmath.mpf(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def pder(p):
    return [p[i] * i for i in range(1, len(p))] or [mpmath.mpf(0)]


def peval(p, x):
    v = mpmath.mpf(0)
    for c in reversed(p):
        v = v * x + c
    return v


def pint(p, lo, hi):
    return sum((c * (hi ** (i + 1) - lo ** (i + 1)) / (i + 1) for i, c in enumerate(p)), mpmath.mpf(0))


def basis_poly(m, centre):
    """P_m(2 (x - centre)) as a polynomial in x."""
    out = [mpmath.mpf(0)]
    lin = [-2 * centre, mpmath.mpf(2)]
    powr = [mpmath.mpf(1)]
    for c in legendre_xi(m):
        out = padd(out, pscale(powr, _mp(c)))
        powr = pmul(powr, lin)
    return out


def cell_poly(u, mesh, cell, centre, k):
    out = [mpmath.mpf(0)]
    for m in range(k + 1):
        out = padd(out, pscale(basis_poly(m, centre), u[mesh][m][cell]))
    return out


def burgers(p):
    return pscale(pmul(p, p), mpmath.mpf(1) / 2)


# ---- geometry ----

def _cell(mesh, c, n):
    """Interval [a, b] of cell c and the other mesh's cells centred on a and b."""
    if mesh == 0:
        a = mpmath.mpf(c)
        return a, a + 1, c % n, (c + 1) % n
    a = mpmath.mpf(c) - mpmath.mpf(1) / 2
    return a, a + 1, (c - 1) % n, c % n


# ---- the operator (eq:1D_H) ----

def rhs(u, n, k, tau_max):
    """L(u): for each basis function phi of cell K (mesh M), H(u, phi) over the
    two halves of K and the two edges of K, divided by int phi^2 = 1/(2m+1).
    On a half cell the other mesh holds one polynomial (the cell centred on
    K's edge at that side); at K's edges that polynomial is continuous."""
    tm = _mp(tau_max)
    out = [[[None] * n for _ in range(k + 1)] for _ in range(2)]
    for mesh in range(2):
        for c in range(n):
            a, b, ol, orr = _cell(mesh, c, n)
            mid = (a + b) / 2
            own = cell_poly(u, mesh, c, mid, k)
            other_l = cell_poly(u, 1 - mesh, ol, a, k)
            other_r = cell_poly(u, 1 - mesh, orr, b, k)
            fl, fr = burgers(other_l), burgers(other_r)
            for m in range(k + 1):
                phi = basis_poly(m, mid)
                dphi = pder(phi)
                H = mpmath.mpf(0)
                for oth, f, lo, hi in ((other_l, fl, a, mid), (other_r, fr, mid, b)):
                    diff = padd(own, pscale(oth, -1))
                    integrand = padd(pscale(pmul(diff, phi), -1 / tm), pmul(f, dphi))
                    H += pint(integrand, lo, hi)
                H += peval(fl, a) * peval(phi, a) - peval(fr, b) * peval(phi, b)
                out[mesh][m][c] = H * (2 * m + 1)
    return out


# ---- OE (Sec. 2.2 and the damping ODE) ----

def _gauss_nodes(Q):
    if Q == 1:
        return [mpmath.mpf(0)]
    if Q == 2:
        r = 1 / mpmath.sqrt(3)
        return [-r, r]
    if Q == 3:
        r = mpmath.sqrt(mpmath.mpf(3) / 5)
        return [-r, mpmath.mpf(0), r]
    raise ValueError("k <= 2 only")


def stats(u, n, k):
    """avg[mesh] and sigma[mesh]."""
    xi = [mpmath.mpf(-1)] + [(s - 1) / 2 for s in _gauss_nodes(k + 1)] + \
         [(s + 1) / 2 for s in _gauss_nodes(k + 1)] + [mpmath.mpf(1)]
    avg, sig = [], []
    for mesh in range(2):
        mean = sum((u[mesh][0][c] for c in range(n)), mpmath.mpf(0)) / n
        s = mpmath.mpf(0)
        for c in range(n):
            a, b, _, _ = _cell(mesh, c, n)
            mid = (a + b) / 2
            p = cell_poly(u, mesh, c, mid, k)
            for x in xi:
                s = max(s, abs(peval(p, mid + x / 2) - mean))
        avg.append(mean)
        sig.append(s)
    return avg, sig


def delta(u, n, k):
    """delta[mesh][m][cell] = (2m+1)/((2k-1) m!) beta_K (|d^m(u_K - v)(a)| +
    |d^m(u_K - v)(b)|) / sigma (h = 1), 0 where sigma = 0; beta_K = |avg_K|."""
    _, sig = stats(u, n, k)
    out = [[[mpmath.mpf(0)] * n for _ in range(k + 1)] for _ in range(2)]
    for mesh in range(2):
        for c in range(n):
            a, b, ol, orr = _cell(mesh, c, n)
            own = cell_poly(u, mesh, c, (a + b) / 2, k)
            dl = padd(own, pscale(cell_poly(u, 1 - mesh, ol, a, k), -1))
            dr = padd(own, pscale(cell_poly(u, 1 - mesh, orr, b, k), -1))
            beta = abs(u[mesh][0][c])
            for m in range(k + 1):
                if sig[mesh] == 0:
                    continue
                jl, jr = abs(peval(dl, a)), abs(peval(dr, b))
                out[mesh][m][c] = (2 * m + 1) * beta * (jl + jr) / ((2 * k - 1) * math.factorial(m) * sig[mesh])
                dl, dr = pder(dl), pder(dr)
    return out


def _projector(k, d):
    """L2 projection onto degree <= d on [-1, 1], in the monomial basis xi^p."""
    G = mpmath.matrix(k + 1, k + 1)
    for p in range(k + 1):
        for q in range(k + 1):
            G[p, q] = mpmath.mpf(2) / (p + q + 1) if (p + q) % 2 == 0 else mpmath.mpf(0)
    Gd = mpmath.matrix(d + 1, d + 1)
    for p in range(d + 1):
        for q in range(d + 1):
            Gd[p, q] = G[p, q]
    Gi = mpmath.inverse(Gd)
    P = mpmath.matrix(k + 1, k + 1)
    for p in range(d + 1):
        for q in range(k + 1):
            P[p, q] = sum((Gi[p, r] * G[r, q] for r in range(d + 1)), mpmath.mpf(0))
    return P


def oe(u, n, k, tau):
    """F_tau: each cell's coefficients advanced by the damping ODE
    d/dt int u phi + sum_m delta^m int (u - P^{m-1} u) phi = 0 (P^{-1} := P^0)
    over time tau, delta frozen at the undamped state."""
    if k < 1:
        return u
    dl = delta(u, n, k)
    to_mono = mpmath.matrix(k + 1, k + 1)            # column m: P_m(xi) in monomials
    for m in range(k + 1):
        for p, c in enumerate(legendre_xi(m)):
            to_mono[p, m] = _mp(c)
    from_mono = mpmath.inverse(to_mono)
    eye = mpmath.eye(k + 1)
    proj = [_projector(k, max(m - 1, 0)) for m in range(k + 1)]
    out = [[[None] * n for _ in range(k + 1)] for _ in range(2)]
    for mesh in range(2):
        for c in range(n):
            A = mpmath.zeros(k + 1, k + 1)
            for m in range(k + 1):
                A -= dl[mesh][m][c] * (eye - proj[m])
            v = mpmath.matrix([u[mesh][m][c] for m in range(k + 1)])
            w = from_mono * (mpmath.expm(_mp(tau) * A) * (to_mono * v))
            for m in range(k + 1):
                out[mesh][m][c] = w[m]
    return out


# ---- time stepping (eq:RKCDG, SSP-RK3) ----

def _axpy(alpha, x, beta, y):
    return [[[alpha * x[s][m][c] + beta * y[s][m][c] for c in range(len(x[s][m]))]
             for m in range(len(x[s]))] for s in range(2)]


def step(u, n, k, tau, tau_max):
    """u_1 = F(u + tau L(u)); u_2 = F(3/4 u + 1/4 (u_1 + tau L(u_1)));
    u^{n+1} = F(1/3 u + 2/3 (u_2 + tau L(u_2)))."""
    t = _mp(tau)
    e1 = _axpy(1, u, t, rhs(u, n, k, tau_max))
    u1 = oe(e1, n, k, tau)
    e2 = _axpy(1, u1, t, rhs(u1, n, k, tau_max))
    u2 = oe(_axpy(mpmath.mpf(3) / 4, u, mpmath.mpf(1) / 4, e2), n, k, tau)
    e3 = _axpy(1, u2, t, rhs(u2, n, k, tau_max))
    return oe(_axpy(mpmath.mpf(1) / 3, u, mpmath.mpf(2) / 3, e3), n, k, tau)


def run(uC, uD, n, k, tau, tau_max, nsteps):
    """nsteps steps from float arrays uC, uD [k+1][n]; returns float lists."""
    with mpmath.workdps(DPS):
        u = [[[_mp(float(v)) for v in row] for row in arr] for arr in (uC, uD)]
        for _ in range(nsteps):
            u = step(u, n, k, tau, tau_max)
        return [[[float(v) for v in row] for row in mesh] for mesh in u]
