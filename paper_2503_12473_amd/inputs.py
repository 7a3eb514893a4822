"""Seeded synthetic inputs for the OECDG workloads.

This module only builds problem descriptions and initial data: it draws the
seeded random parameters, evaluates the analytic initial conditions, and
L2-projects them onto the Legendre modal bases of the primal and dual meshes
(the projection-based initialisation discussed after the optimal error
theorem, Sec. 3.3).  It holds none of the method's arithmetic (no CDG
operator, no damping, no time stepping), so both the HIP path and the CPU
oracle can take their inputs from it.

Mesh convention shared by every consumer: primal cell i of a 1D mesh of n
cells on [xlo, xhi] is [xlo + i h, xlo + (i+1) h]; dual cell j is centred on
the left edge of primal cell j, i.e. [xlo + (j - 1/2) h, xlo + (j + 1/2) h],
for j = 0..n-1 (periodic) or j = 0..n (outflow).  Modal arrays are C-contiguous
float64 of shape [nc, k+1, ncell].  In 2D, primal cell (i, j) is
[xlo + i hx, xlo + (i+1) hx] x [ylo + j hy, ylo + (j+1) hy], dual cell (i, j)
is centred on the primal vertex (xlo + i hx, ylo + j hy), and arrays have
shape [nc, k+1, k+1, ny, nx] (mode a in x, mode b in y).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.polynomial import legendre as _npleg

FLUX_ADVECTION = 0
FLUX_BURGERS = 1
FLUX_EULER = 2
BC_PERIODIC = 0
BC_OUTFLOW = 1
BC_REFLECTIVE = 2
BC_INFLOW = 3

GAMMA = 1.4


@dataclasses.dataclass(frozen=True)
class Problem1D:
    k: int
    nc: int
    flux: int
    bc: int
    n: int
    xlo: float
    xhi: float
    a: float = 1.0          # advection speed
    gamma: float = GAMMA    # adiabatic index
    allow_negative_pressure: bool = False   # Euler: a cell average with p <= 0 is not an error
    inflow: tuple = ()      # BC_INFLOW: (left ghost state, right ghost state), conserved variables

    @property
    def h(self) -> float:
        return (self.xhi - self.xlo) / self.n

    @property
    def n_dual(self) -> int:
        return self.n if self.bc == BC_PERIODIC else self.n + 1

    def shapes(self):
        return (self.nc, self.k + 1, self.n), (self.nc, self.k + 1, self.n_dual)

    def dofs(self) -> int:
        return self.nc * (self.k + 1) * (self.n + self.n_dual)


@dataclasses.dataclass(frozen=True)
class Problem2D:
    k: int
    nc: int
    flux: int
    nx: int
    ny: int
    xlo: float
    xhi: float
    ylo: float
    yhi: float
    a: float = 1.0
    b: float = 1.0
    gamma: float = GAMMA
    space: int = 0          # 0: tensor Q^k; 1: total degree P^k (modes a + b > k are zero)

    @property
    def hx(self) -> float:
        return (self.xhi - self.xlo) / self.nx

    @property
    def hy(self) -> float:
        return (self.yhi - self.ylo) / self.ny

    def shape(self):
        return (self.nc, self.k + 1, self.k + 1, self.ny, self.nx)

    def dofs(self) -> int:
        return 2 * self.nc * (self.k + 1) ** 2 * self.nx * self.ny


# --------------------------------------------------------------------------
# L2 projection of initial data (8 Gauss points on each half cell / quadrant)
# --------------------------------------------------------------------------

def _half_rule(nq: int = 8):
    s, w = _npleg.leggauss(nq)
    xi = np.concatenate([(s - 1.0) / 2.0, (s + 1.0) / 2.0])
    wi = np.concatenate([w / 2.0, w / 2.0])
    return xi, wi


def _legendre_table(k: int, xi: np.ndarray) -> np.ndarray:
    return np.stack([_npleg.legval(xi, [0.0] * m + [1.0]) for m in range(k + 1)])


def project_1d(func, prob: Problem1D, nq: int = 8, exact_constants: bool = False):
    """Project func (x of any shape -> array [nc, *x.shape]) on both meshes.

    Each cell is split at its centre so that jumps on primal edges or dual
    centres are integrated exactly.  exact_constants: where a component takes
    one value at every quadrature point of a cell, its projection is that
    value with all higher modes exactly zero (the quadrature would leave them
    at rounding level, and a component that is uniform over a whole mesh then
    has a rounding-level sigma instead of zero)."""
    xi, wi = _half_rule(nq)
    P = _legendre_table(prob.k, xi)                       # [k+1, G]
    norm = (2.0 * np.arange(prob.k + 1) + 1.0) / 2.0
    h = prob.h

    def proj(centres):
        x = centres[:, None] + 0.5 * h * xi[None, :]     # [ncell, G]
        vals = np.asarray(func(x), dtype=np.float64).reshape(prob.nc, *x.shape)
        a = np.einsum("qcg,mg,g->qmc", vals, P, wi) * norm[None, :, None]
        if exact_constants:
            const = np.all(vals == vals[:, :, :1], axis=2)  # [nc, ncell]
            a[:, 0, :] = np.where(const, vals[:, :, 0], a[:, 0, :])
            a[:, 1:, :] = np.where(const[:, None, :], 0.0, a[:, 1:, :])
        return np.ascontiguousarray(a)

    cC = prob.xlo + (np.arange(prob.n) + 0.5) * h
    cD = prob.xlo + np.arange(prob.n_dual) * h
    return proj(cC), proj(cD)


def project_2d(func, prob: Problem2D, nq: int = 8, chunk_rows: int = 64):
    """Project func (x, y -> [nc, *x.shape]) on both 2D meshes (tensor Q^k modes)."""
    xi, wi = _half_rule(nq)
    P = _legendre_table(prob.k, xi)
    norm = (2.0 * np.arange(prob.k + 1) + 1.0) / 2.0
    K1 = prob.k + 1
    # M[(g, h), (a, b)] = w_g w_h P_a(xi_g) P_b(xi_h) (2a+1)(2b+1)/4
    M = np.einsum("ag,bh,g,h,a,b->ghab", P, P, wi, wi, norm, norm).reshape(-1, K1 * K1)
    hx, hy = prob.hx, prob.hy
    out = []
    for shift in (0.5, 0.0):                              # primal centres, dual centres
        cx = prob.xlo + (np.arange(prob.nx) + shift) * hx
        res = np.empty(prob.shape(), dtype=np.float64)
        for j0 in range(0, prob.ny, chunk_rows):
            j1 = min(prob.ny, j0 + chunk_rows)
            cy = prob.ylo + (np.arange(j0, j1) + shift) * hy
            X = cx[None, :, None, None] + 0.5 * hx * xi[None, None, :, None]
            Y = cy[:, None, None, None] + 0.5 * hy * xi[None, None, None, :]
            X, Y = np.broadcast_arrays(X, Y)              # [rows, nx, Gx, Gy]
            vals = np.asarray(func(X, Y), dtype=np.float64).reshape(prob.nc, *X.shape)
            G = X.shape[2]
            # one matrix product: point values [.., Gx*Gy] -> modes [.., a*b]
            a = (vals.reshape(-1, G * G) @ M).reshape(prob.nc, j1 - j0, prob.nx, K1, K1)
            res[:, :, :, j0:j1, :] = a.transpose(0, 3, 4, 1, 2)
        if prob.space == 1:                               # P^k: the orthogonal projection drops a + b > k
            res = to_pk(prob, res)
        out.append(np.ascontiguousarray(res))
    return out[0], out[1]


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def euler_conserved(rho, u, p, gamma=GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def advection_sine(n: int, k: int, phase: float = 0.0, xlo=0.0, xhi=2.0 * math.pi, a=1.0, freq=1.0):
    """u_t + a u_x = 0 on a periodic interval, u0 = sin(freq*(x - xlo)*2pi/L + phase)."""
    prob = Problem1D(k=k, nc=1, flux=FLUX_ADVECTION, bc=BC_PERIODIC, n=n, xlo=xlo, xhi=xhi, a=a)
    L = xhi - xlo
    uC, uD = project_1d(lambda x: np.sin(freq * 2.0 * math.pi * (x - xlo) / L + phase)[None], prob)
    return prob, uC, uD


def advection_phases(seed: int, count: int = 1):
    """Seeded phases phi ~ U[0, 2 pi) for sin(x + phi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * math.pi, size=count)


def advection_square(n: int, k: int, lo=0.5 * math.pi, hi=1.5 * math.pi, xlo=0.0, xhi=2.0 * math.pi):
    """Square wave: 1 on [lo, hi], 0 elsewhere, periodic."""
    prob = Problem1D(k=k, nc=1, flux=FLUX_ADVECTION, bc=BC_PERIODIC, n=n, xlo=xlo, xhi=xhi, a=1.0)
    L = xhi - xlo

    def f(x):
        y = np.mod(x - xlo, L) + xlo
        return ((y >= lo) & (y < hi)).astype(np.float64)[None]

    uC, uD = project_1d(f, prob)
    return prob, uC, uD


def quasi_uniform_edges(n: int, xlo: float, xhi: float, ratio: float = 1.5, seed: int = 0):
    """Edges x_{i-1/2}, i = 0..n, of a seeded non-uniform mesh of [xlo, xhi]:
    widths proportional to 1 + r_i with r_i ~ U[0, ratio - 1], so that the
    largest width is at most ratio times the smallest."""
    rng = np.random.default_rng(seed)
    w = 1.0 + rng.uniform(0.0, ratio - 1.0, size=n)
    e = np.concatenate([[0.0], np.cumsum(w)])
    e = xlo + (xhi - xlo) * (e / e[-1])
    e[0], e[-1] = xlo, xhi
    return e


def smooth_graded_edges(n: int, xlo: float, xhi: float, amp: float = 0.3):
    """Edges of a smoothly graded mesh: the image of a uniform mesh of [0, 1]
    under s -> s + amp sin(2 pi s) / (2 pi), scaled to [xlo, xhi] (widths vary
    between (1 - amp) and (1 + amp) times L/n; amp < 1)."""
    s = np.arange(n + 1) / n
    e = xlo + (xhi - xlo) * (s + amp * np.sin(2.0 * math.pi * s) / (2.0 * math.pi))
    e[0], e[-1] = xlo, xhi
    return e


def project_1d_edges(func, nc: int, k: int, edges: np.ndarray, nq: int = 8):
    """Project a periodic func (x -> [nc, *x.shape]) onto the primal cells
    [edges[i], edges[i+1]] and the dual cells [x_{j-1}, x_j] between primal
    centres (dual cell 0 starts at x_{n-1} minus the period).  Each cell is
    split where the other mesh has an edge, so jumps there are integrated
    exactly.  Returns arrays [nc, k+1, n]."""
    edges = np.asarray(edges, dtype=np.float64)
    n, L = edges.size - 1, edges[-1] - edges[0]
    s, wq = _npleg.leggauss(nq)
    norm = (2.0 * np.arange(k + 1) + 1.0) / 2.0
    c = 0.5 * (edges[:-1] + edges[1:])
    cm1 = np.concatenate([[c[-1] - L], c[:-1]])

    def proj(lo, split, hi):
        cen, wid = 0.5 * (lo + hi), hi - lo
        out = np.zeros((nc, k + 1, n))
        for a, b in ((lo, split), (split, hi)):
            x = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * s[None, :]
            xi = 2.0 * (x - cen[:, None]) / wid[:, None]
            vals = np.asarray(func(x), dtype=np.float64).reshape(nc, *x.shape)
            P = np.stack([_npleg.legval(xi, [0.0] * m + [1.0]) for m in range(k + 1)])   # [k+1, n, G]
            jac = (0.5 * (b - a) / wid)[:, None] * wq[None, :] * 2.0                     # dx / (w/2) weights
            out += np.einsum("qcg,mcg,cg->qmc", vals, P, jac)
        return np.ascontiguousarray(out * norm[None, :, None])

    return proj(edges[:-1], c, edges[1:]), proj(cm1, edges[:-1], c)


def advection_sine_edges(edges: np.ndarray, k: int, a: float = 1.0, freq: int = 1):
    """u_t + a u_x = 0, u0 = sin(2 pi freq (x - xlo)/L), on the periodic mesh given by its edges."""
    edges = np.asarray(edges, dtype=np.float64)
    xlo, xhi = float(edges[0]), float(edges[-1])
    prob = Problem1D(k=k, nc=1, flux=FLUX_ADVECTION, bc=BC_PERIODIC, n=edges.size - 1, xlo=xlo, xhi=xhi, a=a)
    L = xhi - xlo
    uC, uD = project_1d_edges(lambda x: np.sin(freq * 2.0 * math.pi * (x - xlo) / L)[None], 1, k, edges)
    return prob, uC, uD


def riemann_states(seed: int):
    """(rho_L, p_L, rho_R, p_R), each ~ U[0.1, 1], drawn in that order; u = 0."""
    rng = np.random.default_rng(seed)
    rl, pl, rr, pr = rng.uniform(0.1, 1.0, size=4)
    return float(rl), float(pl), float(rr), float(pr)


def euler_riemann(n: int, k: int, states, x0=0.5, xlo=0.0, xhi=1.0, gamma=GAMMA):
    """1D Euler two-state Riemann problem with outflow boundaries."""
    rl, pl, rr, pr = states
    prob = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=BC_OUTFLOW, n=n, xlo=xlo, xhi=xhi, gamma=gamma)

    def f(x):
        left = x < x0
        rho = np.where(left, rl, rr)
        p = np.where(left, pl, pr)
        return euler_conserved(rho, np.zeros_like(rho), p, gamma)

    uC, uD = project_1d(f, prob)
    return prob, uC, uD


def mirror_extend(func, xlo: float, xhi: float):
    """Euler initial data continued past reflective walls at xlo and xhi:
    density and energy mirrored, momentum mirrored and negated (the dual cells
    centred on the walls reach half a cell outside the domain)."""
    def g(x):
        x = np.asarray(x, dtype=np.float64)
        lo, hi = x < xlo, x > xhi
        xr = np.where(lo, 2.0 * xlo - x, np.where(hi, 2.0 * xhi - x, x))
        v = np.array(func(xr), dtype=np.float64)
        v[1] = np.where(lo | hi, -v[1], v[1])
        return v
    return g


def euler_blast_waves(n: int, k: int, pressures=(1000.0, 0.01, 100.0), densities=(1.0, 1.0, 1.0), gamma=GAMMA,
                      allow_negative_pressure=True):
    """Two interacting blast waves (Sec. 4): [0, 1] with reflective walls,
    u = 0 and (rho, p) = (densities[0], pressures[0]) on x < 0.1,
    (densities[1], pressures[1]) on 0.1 < x < 0.9, (densities[2],
    pressures[2]) on x > 0.9 (the paper's rho = 1 and p = 1000, 0.01, 100 by
    default).  With the paper's data a cell average or two next to the
    weaker blast carries a small non-positive pressure for a few hundred steps,
    which the problem tolerates (allow_negative_pressure)."""
    prob = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=BC_REFLECTIVE, n=n, xlo=0.0, xhi=1.0, gamma=gamma,
                     allow_negative_pressure=allow_negative_pressure)
    pl, pm, pr = (float(v) for v in pressures)
    rl, rm, rr = (float(v) for v in densities)

    def f(x):
        p = np.where(x < 0.1, pl, np.where(x > 0.9, pr, pm))
        rho = np.where(x < 0.1, rl, np.where(x > 0.9, rr, rm))
        return euler_conserved(rho, np.zeros_like(x), p, gamma)

    uC, uD = project_1d(mirror_extend(f, 0.0, 1.0), prob, exact_constants=True)
    return prob, uC, uD


SHU_OSHER_LEFT = (3.857143, 2.629369, 10.33333)   # (rho, v, p) behind the shock, x < -4


def euler_shu_osher(n: int, k: int, gamma=GAMMA):
    """Shu-Osher problem (Sec. 4): [-5, 5], (rho, v, p) = (3.857143, 2.629369,
    10.33333) for x < -4 and (1 + 0.2 sin(5x), 0, 1) for x > -4, with inflow
    boundaries: the ghost cells hold the post-shock state on the left and the
    initial state at x = 5 on the right for the whole run."""
    rl, vl, pl = SHU_OSHER_LEFT
    left = tuple(float(v) for v in euler_conserved(np.array(rl), np.array(vl), np.array(pl), gamma))
    right = tuple(float(v) for v in euler_conserved(np.array(1.0 + 0.2 * math.sin(25.0)), np.array(0.0),
                                                      np.array(1.0), gamma))
    prob = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=BC_INFLOW, n=n, xlo=-5.0, xhi=5.0, gamma=gamma,
                     inflow=(left, right))

    def f(x):                           # beyond x = 5 (the last dual cell): the right ghost state
        sh = x < -4.0
        rho = np.where(sh, rl, 1.0 + 0.2 * np.sin(5.0 * np.minimum(x, 5.0)))
        return euler_conserved(rho, np.where(sh, vl, 0.0), np.where(sh, pl, 1.0), gamma)

    uC, uD = project_1d(f, prob)
    return prob, uC, uD


def euler_walls_smooth(n: int, k: int, xlo=0.0, xhi=1.0, bc=BC_REFLECTIVE, gamma=GAMMA):
    """Smooth Euler data that are symmetric about x = 0 and periodic with
    period 2: rho = 1.2 + 0.3 cos(pi x), u = 0.4 sin(pi x),
    p = 1 + 0.2 cos(2 pi x).  On [0, 1] with walls they are their own mirror
    extension; on [-1, 1] with periodic boundaries they give the doubled
    problem whose right half the walled one reproduces."""
    prob = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=bc, n=n, xlo=xlo, xhi=xhi, gamma=gamma)

    def f(x):
        return euler_conserved(1.2 + 0.3 * np.cos(np.pi * x), 0.4 * np.sin(np.pi * x),
                               1.0 + 0.2 * np.cos(2.0 * np.pi * x), gamma)

    uC, uD = project_1d(f, prob)
    return prob, uC, uD


def burgers_fourier_params(seed: int, modes: int = 8):
    """A_j ~ N(0, 0.3^2) then phi_j ~ U[0, 2 pi), j = 1..modes."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, 0.3, size=modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    return A, phi


def burgers_fourier(n: int, k: int, seed: int, modes: int = 8):
    """Burgers on [0, 2 pi] periodic, u0 = sum_j A_j sin(j x + phi_j)."""
    A, phi = burgers_fourier_params(seed, modes)
    prob = Problem1D(k=k, nc=1, flux=FLUX_BURGERS, bc=BC_PERIODIC, n=n, xlo=0.0, xhi=2.0 * math.pi)

    def f(x):
        v = np.zeros_like(x)
        for j in range(modes):
            v = v + A[j] * np.sin((j + 1) * x + phi[j])
        return v[None]

    uC, uD = project_1d(f, prob)
    return prob, uC, uD, (A, phi)


def burgers_sine(n: int, k: int):
    """Burgers on [0, 2 pi] periodic, u0 = sin x + 0.5 (smooth accuracy example)."""
    prob = Problem1D(k=k, nc=1, flux=FLUX_BURGERS, bc=BC_PERIODIC, n=n, xlo=0.0, xhi=2.0 * math.pi)
    uC, uD = project_1d(lambda x: (np.sin(x) + 0.5)[None], prob)
    return prob, uC, uD


def batch_instances(seed: int, count: int = 512, nmin=128, nmax=8192, kset=(1, 2, 3), k_fixed=None):
    """Per instance, in order: N ~ U{nmin..nmax}, k ~ U{kset}, then the four
    Riemann state draws (rho_L, p_L, rho_R, p_R) ~ U[0.1, 1]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.choice(np.asarray(kset)))
        st = tuple(float(v) for v in rng.uniform(0.1, 1.0, size=4))
        out.append((n, k_fixed if k_fixed is not None else k, st))
    return out


def _project_quadrants_sine(prob: Problem2D, cst, sin_amp, nq: int = 8):
    """Both meshes' projections of f(x, y) = cst[Q] + sin_amp[Q] sin(2 pi (x + y))
    where Q is the domain quadrant (split at the middle of [xlo, xhi] x [ylo, yhi],
    periodic) of the point; cst, sin_amp: [4, nc] in the order SW, SE, NW, NE.
    The same Gauss rule as project_2d (nq points per direction on each quarter
    of a cell), factorised with sin(a + b) = sin a cos b + cos a sin b, so it
    costs O(cells) instead of O(cells * nq^2)."""
    xi, wi = _half_rule(nq)
    G = nq
    P = _legendre_table(prob.k, xi)                           # [K1, 2G]
    K1 = prob.k + 1
    norm = (2.0 * np.arange(K1) + 1.0) / 2.0
    Lx, Ly = prob.xhi - prob.xlo, prob.yhi - prob.ylo
    out = []
    for shift in (0.5, 0.0):                                  # primal centres, dual centres
        cx = prob.xlo + (np.arange(prob.nx) + shift) * prob.hx
        cy = prob.ylo + (np.arange(prob.ny) + shift) * prob.hy
        res = np.zeros(prob.shape())
        # per column / row and quarter side s: I[s][a] (constant), S[.., s, a], C[.., s, a]
        def sums(c, h):
            x = c[:, None] + 0.5 * h * xi[None, :]                # [n, 2G]
            wP = (wi[None, :] * P)                                # [K1, 2G]
            I = np.stack([wP[:, :G].sum(axis=1), wP[:, G:].sum(axis=1)]) * norm[None, :]
            sn, cs = np.sin(2.0 * math.pi * x), np.cos(2.0 * math.pi * x)
            S = np.stack([sn[:, :G] @ wP[:, :G].T, sn[:, G:] @ wP[:, G:].T], axis=1) * norm[None, None, :]
            C = np.stack([cs[:, :G] @ wP[:, :G].T, cs[:, G:] @ wP[:, G:].T], axis=1) * norm[None, None, :]
            mid = np.stack([c - 0.25 * h, c + 0.25 * h], axis=1)   # quarter centres [n, 2]
            return I, S, C, mid
        Ix, Sx, Cx, mx = sums(cx, prob.hx)
        Iy, Sy, Cy, my = sums(cy, prob.hy)
        qx = (np.mod(mx - prob.xlo, Lx) >= 0.5 * Lx).astype(np.int64)   # [nx, 2]
        qy = (np.mod(my - prob.ylo, Ly) >= 0.5 * Ly).astype(np.int64)   # [ny, 2]
        for sx in range(2):
            for sy in range(2):
                qd = qx[None, :, sx] + 2 * qy[:, sy, None]         # [ny, nx]
                Cq = np.asarray(cst)[qd].transpose(2, 0, 1)        # [nc, ny, nx]
                Sq = np.asarray(sin_amp)[qd].transpose(2, 0, 1)
                for a in range(K1):
                    for b in range(K1):
                        res[:, a, b] += Cq * (Ix[sx, a] * Iy[sy, b])
                        res[:, a, b] += Sq * (Cy[:, sy, b][:, None] * Sx[:, sx, a][None, :]
                                              + Sy[:, sy, b][:, None] * Cx[:, sx, a][None, :])
        out.append(np.ascontiguousarray(res))
    return out[0], out[1]


def to_pk(prob: Problem2D, u: np.ndarray) -> np.ndarray:
    """The P^k part of a tensor-mode array: modes a + b > k set to zero (the
    L2 projection onto P^k, the basis being orthogonal)."""
    u = np.array(u, dtype=np.float64, copy=True)
    for ia in range(prob.k + 1):
        for ib in range(prob.k + 1):
            if ia + ib > prob.k:
                u[:, ia, ib] = 0.0
    return u


def euler2d_quadrants(n: int, k: int, seed: int, gamma=GAMMA, fast: bool = True, space: int = 0):
    """2D Euler on [0,1]^2 periodic: rho = 1 + 0.2 sin(2 pi (x+y)) + rho_q and
    (u, v, p) = (u_q, v_q, p_q) on the four quadrants split at 0.5, with
    (rho_q, p_q) ~ U[0.2, 1] and u_q, v_q ~ U[-0.5, 0.5], drawn per quadrant in
    the order SW, SE, NW, NE as (rho, p, u, v).  The conserved variables are
    affine in sin(2 pi (x+y)) on each quadrant; fast=True projects them with
    the factorised rule, fast=False with the generic point-value projection."""
    rng = np.random.default_rng(seed)
    quads = []
    for _ in range(4):
        rq, pq = rng.uniform(0.2, 1.0, size=2)
        uq, vq = rng.uniform(-0.5, 0.5, size=2)
        quads.append((rq, pq, uq, vq))
    quads = np.asarray(quads)
    prob = Problem2D(k=k, nc=4, flux=FLUX_EULER, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, gamma=gamma,
                     space=space)
    if fast:
        rq, pq, uq, vq = quads.T
        r0 = 1.0 + rq
        ke = uq * uq + vq * vq
        cst = np.stack([r0, r0 * uq, r0 * vq, pq / (gamma - 1.0) + 0.5 * r0 * ke], axis=1)
        amp = np.stack([0.2 + 0 * rq, 0.2 * uq, 0.2 * vq, 0.1 * ke], axis=1)
        uC, uD = _project_quadrants_sine(prob, cst, amp)
        if space == 1:
            uC, uD = np.ascontiguousarray(to_pk(prob, uC)), np.ascontiguousarray(to_pk(prob, uD))
        return prob, uC, uD, quads

    def f(X, Y):
        xm = np.mod(X, 1.0)
        ym = np.mod(Y, 1.0)
        qi = (xm >= 0.5).astype(np.int64) + 2 * (ym >= 0.5).astype(np.int64)
        rq, pq, uq, vq = (quads[:, c][qi] for c in range(4))
        rho = 1.0 + 0.2 * np.sin(2.0 * math.pi * (X + Y)) + rq
        E = pq / (gamma - 1.0) + 0.5 * rho * (uq * uq + vq * vq)
        return np.stack([rho, rho * uq, rho * vq, E])

    uC, uD = project_2d(f, prob)
    return prob, uC, uD, quads


def euler2d_smooth(n: int, k: int, gamma=GAMMA):
    """Steady smooth 2D Euler solution rho = 1 + 0.2 sin(pi (x - y)), u = v = p = 1 on [0,2]^2."""
    prob = Problem2D(k=k, nc=4, flux=FLUX_EULER, nx=n, ny=n, xlo=0.0, xhi=2.0, ylo=0.0, yhi=2.0, gamma=gamma)

    def f(X, Y):
        rho = 1.0 + 0.2 * np.sin(math.pi * (X - Y))
        one = np.ones_like(X)
        return np.stack([rho, rho, rho, 1.0 / (gamma - 1.0) + rho])

    uC, uD = project_2d(f, prob)
    return prob, uC, uD


def advection2d_sine(n: int, k: int, space: int = 0):
    """u_t + u_x + u_y = 0 on [0,1]^2 periodic, u0 = sin^2(pi (x + y))
    (Sec. 4, the data of Table 2Dlinear_accuracy); space 1 = P^k."""
    prob = Problem2D(k=k, nc=1, flux=FLUX_ADVECTION, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, space=space)
    uC, uD = project_2d(lambda X, Y: (np.sin(math.pi * (X + Y)) ** 2)[None], prob)
    return prob, uC, uD
