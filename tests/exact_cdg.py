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


def bilinear(u, phi, n, k, a, tau_max):
    """H(u, phi) of eq:1D_H with f(u) = a u (exact).

    u, phi: nested lists [mesh][m][cell] of rationals."""
    H = F(0)
    a = F(a)
    tm = F(tau_max)
    for p in range(2 * n):
        lo, hi = F(p, 2), F(p + 1, 2)
        u1, u2 = _piece(u, 0, p, n, k), _piece(u, 1, p, n, k)
        f1, f2 = _piece(phi, 0, p, n, k), _piece(phi, 1, p, n, k)
        d = padd(u1, pscale(u2, -1))
        e = padd(f1, pscale(f2, -1))
        integrand = padd(pscale(pmul(d, e), -1 / tm),
                         padd(pscale(pmul(u2, pder(f1)), a), pscale(pmul(u1, pder(f2)), a)))
        H += pint(integrand, lo, hi)
    # primal edges X = 0..n-1: f(u2)(X) [phi1(X^-) - phi1(X^+)]
    for X in range(n):
        pl, pr = (2 * X - 1) % (2 * n), 2 * X
        xl = F(X) if pl != 2 * n - 1 else F(n)      # left limit taken on the wrapped piece
        u2 = peval(_piece(u, 1, pr, n, k), F(X))
        jump = peval(_piece(phi, 0, pl, n, k), xl) - peval(_piece(phi, 0, pr, n, k), F(X))
        H -= a * u2 * jump
    # dual edges Y = X + 1/2: f(u1)(Y) [phi2(Y^-) - phi2(Y^+)]
    for X in range(n):
        Y = F(2 * X + 1, 2)
        u1 = peval(_piece(u, 0, 2 * X, n, k), Y)
        jump = peval(_piece(phi, 1, 2 * X, n, k), Y) - peval(_piece(phi, 1, 2 * X + 1, n, k), Y)
        H -= a * u1 * jump
    return H


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
