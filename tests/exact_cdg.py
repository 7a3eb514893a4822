"""Exact rational evaluation of the 1D CDG bilinear form (test pin).

An independent second formulation of the spatial operator: instead of the
per-cell equations (equcdg) that the oracle follows, this module evaluates
the global bilinear form H(u, phi) of eq. (eq:1D_H), Sec. 2.1, for a linear
flux f(u) = a u on a periodic mesh, with polynomials in exact rational
arithmetic (``fractions.Fraction``).  It is used to pin the oracle's operator
and to check the approximate skew-symmetry lemma (lem:skew-symm, Sec. 3.1)
exactly.

Mesh: n primal cells [i, i+1] (h = 1), dual cells centred on the integers.
"""
from __future__ import annotations

from fractions import Fraction as F


# ---- rational polynomials in x, coefficient lists (lowest degree first) ----

def padd(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def pscale(p, s):
    return [c * s for c in p]


def pmul(p, q):
    out = [F(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def pder(p):
    return [p[i] * i for i in range(1, len(p))] or [F(0)]


def peval(p, x):
    v = F(0)
    for c in reversed(p):
        v = v * x + c
    return v


def pint(p, lo, hi):
    v = F(0)
    for i, c in enumerate(p):
        v += c * (F(hi) ** (i + 1) - F(lo) ** (i + 1)) / (i + 1)
    return v


def legendre_xi(m):
    """P_m(xi) as rational coefficients in xi (Bonnet recurrence)."""
    P = [[F(1)], [F(0), F(1)]]
    for j in range(1, m):
        nxt = padd(pscale([F(0)] + P[j], F(2 * j + 1, j + 1)), pscale(P[j - 1], F(-j, j + 1)))
        P.append(nxt)
    return P[m]


def compose_affine(p, s, t):
    """p(s*x + t) as a polynomial in x."""
    out = [F(0)]
    lin = [F(t), F(s)]
    powr = [F(1)]
    for c in p:
        out = padd(out, pscale(powr, c))
        powr = pmul(powr, lin)
    return out


def basis_poly(m, centre):
    """P_m(2 (x - centre)) on a cell of width 1."""
    return compose_affine(legendre_xi(m), F(2), F(-2) * F(centre))


# ---- the bilinear form --------------------------------------------------------

def _piece(coeffs, mesh, p, n, k):
    """Polynomial of a field (coeffs[mesh][m][cell]) on half-interval p."""
    if mesh == 0:
        i = p // 2
        centre = F(2 * i + 1, 2)
        cell = i % n
    else:
        j = (p + 1) // 2
        centre = F(j)
        cell = j % n
    out = [F(0)]
    for m in range(k + 1):
        c = coeffs[mesh][m][cell]
        if c != 0:
            out = padd(out, pscale(basis_poly(m, centre), c))
    return out


def linear_flux(a):
    """f(u) = a u, as (polynomial map, value map)."""
    a = F(a)
    return (lambda p: pscale(p, a)), (lambda v: a * v)


def burgers_flux():
    """f(u) = u^2 / 2, as (polynomial map, value map): the composition of a
    piecewise polynomial with f stays a polynomial, so H stays exact."""
    return (lambda p: pscale(pmul(p, p), F(1, 2))), (lambda v: v * v / 2)


def bilinear(u, phi, n, k, a, tau_max, flux=None):
    """H(u, phi) of eq:1D_H (exact), with f(u) = a u unless flux = (polynomial
    map, value map) names another polynomial flux.

    u, phi: nested lists [mesh][m][cell] of rationals."""
    fpoly, fval = flux if flux is not None else linear_flux(a)
    H = F(0)
    tm = F(tau_max)
    for p in range(2 * n):
        lo, hi = F(p, 2), F(p + 1, 2)
        f1, f2 = _piece(phi, 0, p, n, k), _piece(phi, 1, p, n, k)
        if not any(f1) and not any(f2):
            continue                                # phi vanishes on this piece
        u1, u2 = _piece(u, 0, p, n, k), _piece(u, 1, p, n, k)
        d = padd(u1, pscale(u2, -1))
        e = padd(f1, pscale(f2, -1))
        integrand = padd(pscale(pmul(d, e), -1 / tm),
                         padd(pmul(fpoly(u2), pder(f1)), pmul(fpoly(u1), pder(f2))))
        H += pint(integrand, lo, hi)
    # primal edges X = 0..n-1: f(u2)(X) [phi1(X^-) - phi1(X^+)]
    for X in range(n):
        pl, pr = (2 * X - 1) % (2 * n), 2 * X
        xl = F(X) if pl != 2 * n - 1 else F(n)      # left limit taken on the wrapped piece
        u2 = peval(_piece(u, 1, pr, n, k), F(X))
        jump = peval(_piece(phi, 0, pl, n, k), xl) - peval(_piece(phi, 0, pr, n, k), F(X))
        H -= fval(u2) * jump
    # dual edges Y = X + 1/2: f(u1)(Y) [phi2(Y^-) - phi2(Y^+)]
    for X in range(n):
        Y = F(2 * X + 1, 2)
        u1 = peval(_piece(u, 0, 2 * X, n, k), Y)
        jump = peval(_piece(phi, 1, 2 * X, n, k), Y) - peval(_piece(phi, 1, 2 * X + 1, n, k), Y)
        H -= fval(u1) * jump
    return H


def operator_rhs(u, n, k, tau_max, flux):
    """L(u) of M dL/dt = H(u, .) (exact): L[mesh][m][cell] = H(u, e) / int e^2
    for every basis function e (h = 1, so int P_m(2(x - c))^2 = 1 / (2m + 1))."""
    out = [[[F(0)] * n for _ in range(k + 1)] for _ in range(2)]
    for idx in range(2 * (k + 1) * n):
        mesh, rem = divmod(idx, (k + 1) * n)
        m, cell = divmod(rem, n)
        out[mesh][m][cell] = bilinear(u, unit(idx, n, k), n, k, 0, tau_max, flux) * (2 * m + 1)
    return out


def gram(u, phi, n, k):
    """int (u1 - u2)(phi1 - phi2) dx (exact)."""
    G = F(0)
    for p in range(2 * n):
        d = padd(_piece(u, 0, p, n, k), pscale(_piece(u, 1, p, n, k), -1))
        e = padd(_piece(phi, 0, p, n, k), pscale(_piece(phi, 1, p, n, k), -1))
        G += pint(pmul(d, e), F(p, 2), F(p + 1, 2))
    return G


def unit(idx, n, k):
    """Basis vector number idx in the flat order [mesh][m][cell]."""
    v = [[[F(0)] * n for _ in range(k + 1)] for _ in range(2)]
    mesh, rem = divmod(idx, (k + 1) * n)
    m, cell = divmod(rem, n)
    v[mesh][m][cell] = F(1)
    return v


def operator_matrix(n, k, a, tau_max):
    """A[r][c] = H(e_c, e_r) and G[r][c] = gram(e_c, e_r) over all basis vectors."""
    N = 2 * (k + 1) * n
    basis = [unit(i, n, k) for i in range(N)]
    A = [[bilinear(basis[c], basis[r], n, k, a, tau_max) for c in range(N)] for r in range(N)]
    G = [[gram(basis[c], basis[r], n, k) for c in range(N)] for r in range(N)]
    return A, G
