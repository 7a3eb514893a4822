"""Pins of the 2D CPU oracle (tensor Q^k, periodic Cartesian primal/dual
meshes) against facts fixed by the paper and by the mathematics:

- consistency: for a global polynomial shared by both meshes and a linear
  flux, the operator of eq. (eq:2D_H) reduces to the L2 projection of
  -div f on every cell whose neighbours do not wrap (the coupling vanishes,
  volume and edge terms integrate by parts exactly);
- the approximate skew-symmetry lemma of Sec. 3.1 in 2D, with the overlap
  Gram matrix built from exact polynomial integrals (not the oracle's
  quadrature);
- without OE, data independent of y reduce the 2D scheme to the pinned 1D
  scheme (advection and Euler);
- the damping coefficients of Sec. 2.2 on worked examples with closed-form
  values (m = 0 and m = 1, unequal hx, hy and velocity components);
- delta vanishes where both meshes hold the same polynomial; the OE step is
  the exact exponential of the damping ODE with the total-degree rule for
  the tensor space; conservation on each mesh; the spectral radii;
- a soft convergence rate on the steady smooth Euler solution (Sec. 4).
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as Pw

from oracle import ora
from paper_2503_12473_amd import inputs
from paper_2503_12473_amd.inputs import Problem2D, Problem1D, FLUX_ADVECTION, FLUX_EULER, BC_PERIODIC


# ------------------------------------------------------------ helpers ---

def _shifted_power(c, centre, half):
    """Power-series coefficients in t of sum_i c[i] (centre + half t)^i."""
    out = np.zeros(len(c))
    for i, ci in enumerate(c):
        term = Pw.polypow([centre, half], i) if i else np.array([1.0])
        out[: len(term)] += ci * term
    return out


def _cell_legendre(Cpow, xc, yc, hx, hy):
    """Legendre coefficients [a, b] on the cell centred at (xc, yc) of the
    polynomial sum_ij Cpow[i, j] x^i y^j (degree <= k in each variable)."""
    K1 = Cpow.shape[0]
    B = np.zeros((K1, K1))              # power coefficients in (xi, eta)
    for j in range(K1):
        B[:, j] = _shifted_power(Cpow[:, j], xc, hx / 2)
    for d in range(K1):
        B[d, :] = _shifted_power(B[d, :], yc, hy / 2)
    T = np.zeros((K1, K1))
    for e in range(K1):
        leg = L.poly2leg(B[:, e])
        T[: len(leg), e] = leg
    out = np.zeros((K1, K1))
    for a in range(K1):
        leg = L.poly2leg(T[a, :])
        out[a, : len(leg)] = leg
    return out


def _project_poly(prob, Cpow_list):
    """Both meshes' exact coefficients of the global polynomials (one per component)."""
    out = []
    for shift in (0.5, 0.0):
        u = np.zeros(prob.shape())
        for iy in range(prob.ny):
            for ix in range(prob.nx):
                xc = prob.xlo + (ix + shift) * prob.hx
                yc = prob.ylo + (iy + shift) * prob.hy
                for q, Cp in enumerate(Cpow_list):
                    u[q, :, :, iy, ix] = _cell_legendre(Cp, xc, yc, prob.hx, prob.hy)
        out.append(u)
    return out[0], out[1]


def _interior(prob, mesh):
    """Cells whose overlapping cells on the other mesh are reached without
    the periodic wrap."""
    if mesh == 0:
        return slice(0, prob.nx - 1), slice(0, prob.ny - 1)
    return slice(1, prob.nx), slice(1, prob.ny)


def _adv(k, nx=6, ny=5, xlo=0.0, xhi=1.5, ylo=0.0, yhi=1.0, a=1.3, b=-0.6):
    return Problem2D(k=k, nc=1, flux=FLUX_ADVECTION, nx=nx, ny=ny, xlo=xlo, xhi=xhi, ylo=ylo, yhi=yhi, a=a, b=b)


# ------------------------------------------------- operator pins ---

@pytest.mark.parametrize("k", [1, 2, 3])
def test_rhs_is_projection_of_minus_divergence_for_shared_polynomial(k):
    prob = _adv(k)
    rng = np.random.default_rng(k)
    Cp = rng.normal(size=(k + 1, k + 1))
    uC, uD = _project_poly(prob, [Cp])
    LC, LD = ora.rhs2d(prob, 0.01, uC, uD)
    # -(a p_x + b p_y) as a power series
    dx = np.zeros_like(Cp)
    dy = np.zeros_like(Cp)
    for i in range(k + 1):
        for j in range(k + 1):
            if i:
                dx[i - 1, j] += i * Cp[i, j]
            if j:
                dy[i, j - 1] += j * Cp[i, j]
    eC, eD = _project_poly(prob, [-(prob.a * dx + prob.b * dy)])
    for mesh, (got, exp) in enumerate(((LC, eC), (LD, eD))):
        sx, sy = _interior(prob, mesh)
        g, e = got[..., sy, sx], exp[..., sy, sx]
        assert np.abs(g - e).max() <= 1e-11 * max(1.0, np.abs(e).max())


def _x_overlap(k, shift):
    """int over the overlap half of P_a(xi) P_c(xi + shift) dxi, [a, c];
    shift +1: xi in [-1, 0], shift -1: xi in [0, 1]."""
    lo, hi = (-1.0, 0.0) if shift > 0 else (0.0, 1.0)
    M = np.zeros((k + 1, k + 1))
    for a in range(k + 1):
        pa = L.leg2poly([0] * a + [1])
        for c in range(k + 1):
            pc = _shifted_power(L.leg2poly([0] * c + [1]), shift, 1.0)
            prod = Pw.polymul(pa, pc)
            I = Pw.polyint(prod)
            M[a, c] = Pw.polyval(hi, I) - Pw.polyval(lo, I)
    return M


@pytest.mark.parametrize("k", [1, 2])
def test_skew_symmetry_lemma_2d(k):
    """M L + (M L)^T = -(2/tau_max) G for a linear flux, with G the Gram
    matrix of (u^C - u^D) built from exact overlap integrals."""
    prob = _adv(k, nx=3, ny=3, xlo=0.0, xhi=1.2, ylo=0.0, yhi=0.9, a=1.3, b=-0.6)
    tm = 0.05
    shp = prob.shape()
    nC = int(np.prod(shp))
    N = 2 * nC
    Lm = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        LC, LD = ora.rhs2d(prob, tm, e[:nC].reshape(shp), e[nC:].reshape(shp))
        Lm[:, j] = np.concatenate([LC.ravel(), LD.ravel()])
    K1 = k + 1
    hx, hy = prob.hx, prob.hy
    mass = np.zeros(shp)
    for a in range(K1):
        for b in range(K1):
            mass[0, a, b] = hx * hy / ((2 * a + 1) * (2 * b + 1))
    Mv = np.concatenate([mass.ravel(), mass.ravel()])
    ML = Mv[:, None] * Lm
    # Gram matrix of (h1 - h2): [[M, -X], [-X^T, M]], X = int phi^C phi^D
    X = np.zeros((nC, nC))
    idx = np.arange(nC).reshape(shp)
    Ox = {s: _x_overlap(k, s) for s in (1.0, -1.0)}
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            for sx in (0, 1):
                for sy in (0, 1):
                    dx_, dy_ = (ix + sx) % prob.nx, (iy + sy) % prob.ny      # dual cell of this quadrant
                    Ix = Ox[1.0 if sx == 0 else -1.0]
                    Iy = Ox[1.0 if sy == 0 else -1.0]
                    for a in range(K1):
                        for b in range(K1):
                            for c in range(K1):
                                for d in range(K1):
                                    X[idx[0, a, b, iy, ix], idx[0, c, d, dy_, dx_]] += \
                                        (hx / 2) * (hy / 2) * Ix[a, c] * Iy[b, d]
    G = np.block([[np.diag(mass.ravel()), -X], [-X.T, np.diag(mass.ravel())]])
    R = ML + ML.T + (2.0 / tm) * G
    assert np.abs(R).max() <= 1e-12 * np.abs(ML).max()


def test_no_oe_y_independent_advection_reduces_to_1d():
    k, n = 2, 12
    p2 = Problem2D(k=k, nc=1, flux=FLUX_ADVECTION, nx=n, ny=3, xlo=0.0, xhi=2 * math.pi, ylo=0.0, yhi=1.0,
                   a=1.0, b=0.0)
    p1 = Problem1D(k=k, nc=1, flux=FLUX_ADVECTION, bc=BC_PERIODIC, n=n, xlo=0.0, xhi=2 * math.pi, a=1.0)
    f = lambda X, Y: (np.sin(X) + 0.3 * np.cos(2 * X))[None]
    uC, uD = inputs.project_2d(f, p2)
    vC, vD = inputs.project_1d(lambda x: (np.sin(x) + 0.3 * np.cos(2 * x))[None], p1)
    dt = 0.05
    oC, oD, _, _ = ora.run2d(p2, uC, uD, nsteps=3, dt_fixed=dt, oe=False)
    rC, rD, _, _ = ora.run1d(p1, vC, vD, nsteps=3, dt_fixed=dt, oe=False)
    for o, r in ((oC, rC), (oD, rD)):
        for iy in range(p2.ny):
            assert np.abs(o[0, :, 0, iy, :] - r[0]).max() <= 1e-13
        assert np.abs(o[0, :, 1:, :, :]).max() <= 1e-13


def test_no_oe_y_independent_euler_reduces_to_1d():
    k, n = 2, 10
    p2 = Problem2D(k=k, nc=4, flux=FLUX_EULER, nx=n, ny=2, xlo=0.0, xhi=1.0, ylo=0.0, yhi=0.5)
    p1 = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=BC_PERIODIC, n=n, xlo=0.0, xhi=1.0)
    rho = lambda x: 1.0 + 0.3 * np.sin(2 * math.pi * x)
    vel = lambda x: 0.4 + 0.2 * np.cos(2 * math.pi * x)
    pr = lambda x: 1.0 + 0.1 * np.sin(4 * math.pi * x)
    g = p2.gamma

    def f2(X, Y):
        r, u, p = rho(X), vel(X), pr(X)
        return np.stack([r, r * u, 0 * X, p / (g - 1) + 0.5 * r * u * u])

    uC, uD = inputs.project_2d(f2, p2)
    vC, vD = inputs.project_1d(lambda x: inputs.euler_conserved(rho(x), vel(x), pr(x)), p1)
    dt = 0.004
    oC, oD, _, _ = ora.run2d(p2, uC, uD, nsteps=3, dt_fixed=dt, oe=False)
    rC, rD, _, _ = ora.run1d(p1, vC, vD, nsteps=3, dt_fixed=dt, oe=False)
    for o, r in ((oC, rC), (oD, rD)):
        for q2, q1 in ((0, 0), (1, 1), (3, 2)):
            for iy in range(p2.ny):
                assert np.abs(o[q2, :, 0, iy, :] - r[q1]).max() <= 1e-12 * np.abs(r[q1]).max()
        assert np.abs(o[2]).max() <= 1e-13
        assert np.abs(o[:, :, 1:]).max() <= 1e-12


# --------------------------------------------------------- OE pins ---

def _delta_problem():
    return _adv(2, nx=6, ny=6, xlo=0.0, xhi=2.0, ylo=0.0, yhi=1.0, a=1.3, b=0.6)


def test_delta_worked_example_constant_jump():
    """Dual cell (2,2) holds 1, every other cell 0 except primal (5,5) = 1
    (so that sigma_C != 0).  Closed forms (k = 2, 2k - 1 = 3): primal (2,2)
    sees the jump on the south half of its west edge and the west half of its
    south edge (edge means 1/2); dual (2,2) sees it on all four edges."""
    prob = _delta_problem()
    uC = np.zeros(prob.shape())
    uD = np.zeros(prob.shape())
    uD[0, 0, 0, 2, 2] = 1.0
    uC[0, 0, 0, 5, 5] = 1.0
    dC, dD = ora.delta2d(prob, uC, uD)
    sig = 1.0 - 1.0 / 36.0
    a, b, hx, hy = abs(prob.a), abs(prob.b), prob.hx, prob.hy
    exp_C = (a / hx * 0.5 + b / hy * 0.5) / (3.0 * sig)
    exp_D = (2 * a / hx + 2 * b / hy) / (3.0 * sig)
    assert dC[0, 2, 2] == pytest.approx(exp_C, rel=1e-14)
    assert dD[0, 2, 2] == pytest.approx(exp_D, rel=1e-14)
    assert np.all(dC[1:, 2, 2] == 0.0) and np.all(dD[1:, 2, 2] == 0.0)
    # primal cells that do not touch the dual cell's support see nothing
    assert dC[0, 4, 0] == 0.0


def test_delta_worked_example_linear_jump():
    """Dual (2,2) holds u = xi (mode (1,0) = 1): on primal (2,2) the value
    jump vanishes on the west edge (the dual's centre line) and averages 1/4
    on the south edge; the x-derivative jump 2/hx gives edge means 1/hx on
    both, so delta^0 = |b|/(4 hy 3 sigma), delta^1 = (|a|+|b|)/(hx sigma)."""
    prob = _delta_problem()
    uC = np.zeros(prob.shape())
    uD = np.zeros(prob.shape())
    uD[0, 1, 0, 2, 2] = 1.0
    uC[0, 0, 0, 5, 5] = 1.0
    dC, dD = ora.delta2d(prob, uC, uD)
    sig = 1.0 - 1.0 / 36.0
    a, b, hx, hy = abs(prob.a), abs(prob.b), prob.hx, prob.hy
    assert dC[0, 2, 2] == pytest.approx(b / (4 * hy) / (3 * sig), rel=1e-13)
    assert dC[1, 2, 2] == pytest.approx((a + b) / (hx * sig), rel=1e-13)
    assert dC[2, 2, 2] == 0.0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_delta_vanishes_for_shared_polynomial(k):
    prob = _adv(k, nx=5, ny=5)
    rng = np.random.default_rng(10 + k)
    Cp = rng.normal(size=(k + 1, k + 1))
    uC, uD = _project_poly(prob, [Cp])
    dC, dD = ora.delta2d(prob, uC, uD)
    scale = np.abs(dC).max()
    for mesh, d in enumerate((dC, dD)):
        sx, sy = _interior(prob, mesh)
        # interior cells see the same polynomial on both meshes: zero up to rounding
        assert np.abs(d[:, sy, sx]).max() <= 1e-9 * max(scale, 1.0)
    assert scale > 0.0                 # the wrapped cells do see a jump


def test_oe_identity_when_sigma_zero():
    prob = _adv(2)
    uC = np.full(prob.shape(), 0.0)
    uC[0, 0, 0] = 0.7
    uD = uC.copy()
    oC, oD = ora.oe2d(prob, 0.3, uC, uD)
    assert np.array_equal(oC, uC) and np.array_equal(oD, uD)


@pytest.mark.parametrize("k", [1, 2])
def test_oe_is_exact_exponential_with_total_degree_rule(k):
    prob, uC, uD, _ = inputs.euler2d_quadrants(6, k, seed=3)
    tau = 0.01
    dC, dD = ora.delta2d(prob, uC, uD)
    oC, oD = ora.oe2d(prob, tau, uC, uD)
    for u, o, d in ((uC, oC, dC), (uD, oD, dD)):
        S = np.cumsum(d, axis=0)                       # S[m] = sum_{m' <= m} delta^m'
        for a in range(k + 1):
            for b in range(k + 1):
                if a + b == 0:
                    assert np.array_equal(o[:, 0, 0], u[:, 0, 0])
                    continue
                fac = np.exp(-tau * S[min(a + b, k)])
                assert np.allclose(o[:, a, b], u[:, a, b] * fac[None], rtol=1e-14, atol=0)
        assert np.all(np.abs(o) <= np.abs(u))


def test_conservation_on_each_mesh():
    prob, uC, uD, _ = inputs.euler2d_quadrants(8, 2, seed=0)
    oC, oD, _, n = ora.run2d(prob, uC, uD, nsteps=2, cfl=0.3)
    assert n == 2
    for u, o in ((uC, oC), (uD, oD)):
        s0 = u[:, 0, 0].sum(axis=(1, 2))
        s1 = o[:, 0, 0].sum(axis=(1, 2))
        assert np.all(np.abs(s1 - s0) <= 1e-13 * np.abs(u[:, 0, 0]).sum(axis=(1, 2)))


def test_wavespeeds_of_a_constant_state():
    prob = Problem2D(k=2, nc=4, flux=FLUX_EULER, nx=4, ny=4, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0)
    rho, u, v, p, g = 0.8, -0.3, 0.5, 0.6, prob.gamma
    uC = np.zeros(prob.shape())
    uC[:, 0, 0] = np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])[:, None, None]
    bx, by = ora.max_wavespeeds2d(prob, uC, uC.copy())
    c = math.sqrt(g * p / rho)
    assert bx == pytest.approx(abs(u) + c, rel=1e-14)
    assert by == pytest.approx(abs(v) + c, rel=1e-14)


def test_constant_state_is_preserved():
    prob = Problem2D(k=2, nc=4, flux=FLUX_EULER, nx=4, ny=4, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0)
    uC = np.zeros(prob.shape())
    uC[:, 0, 0] = np.array([1.1, 0.2, -0.1, 2.0])[:, None, None]
    oC, oD, _, _ = ora.run2d(prob, uC, uC.copy(), nsteps=3, cfl=0.3)
    assert np.abs(oC - uC).max() <= 1e-14 and np.abs(oD - uC).max() <= 1e-14


def test_steady_smooth_euler_converges_soft():
    """Steady solution rho = 1 + 0.2 sin(pi(x - y)), u = v = p = 1 on [0,2]^2
    (Sec. 4): the drift of the cell averages after a short time falls at a
    rate near k + 1 = 3 for Q2 (soft pin: >= 2.5)."""
    errs = []
    for n in (8, 16):
        prob, uC, uD = inputs.euler2d_smooth(n, 2)
        oC, _, _, _ = ora.run2d(prob, uC, uD, t_end=0.05, cfl=0.3)
        errs.append(np.abs(oC[0, 0, 0] - uC[0, 0, 0]).mean())
    rate = math.log2(errs[0] / errs[1])
    assert rate >= 2.5, (errs, rate)


# ------------------------------------------------- P^k space ---

@pytest.mark.parametrize("k", [1, 2, 3])
def test_pk_step_is_the_galerkin_restriction(k):
    """The total-degree space P^k (Sec. 2.1), OE off, linear advection: the
    P^k Galerkin operator is T A T, with A the tensor-space operator (columns
    from the oracle's right-hand side with space 0) and T the projection onto
    the modes a + b <= k (the basis is orthogonal); one SSP-RK3 step with
    space 1 equals the third-order stability polynomial of tau T A T."""
    prob_q = _adv(k, nx=4, ny=3)
    prob_p = Problem2D(**{**prob_q.__dict__, "space": 1})
    shape = prob_q.shape()
    n1 = int(np.prod(shape))
    keep = np.zeros(shape, dtype=bool)
    for a in range(k + 1):
        for b in range(k + 1):
            keep[:, a, b] = a + b <= k
    T = np.diag(np.concatenate([keep.ravel(), keep.ravel()]).astype(float))
    tau_max = 0.05
    A = np.zeros((2 * n1, 2 * n1))
    for j in range(2 * n1):
        e = np.zeros(2 * n1)
        e[j] = 1.0
        LC, LD = ora.rhs2d(prob_q, tau_max, e[:n1].reshape(shape), e[n1:].reshape(shape))
        A[:, j] = np.concatenate([LC.ravel(), LD.ravel()])
    Ap = T @ A @ T
    u = T @ np.random.default_rng(k).normal(size=2 * n1)
    tau = 0.8 * tau_max
    ref, term = u.copy(), u.copy()
    for j in range(1, 4):
        term = tau * (Ap @ term) / j
        ref += term
    oC, oD = ora.step2d(prob_p, tau, tau_max, u[:n1].reshape(shape), u[n1:].reshape(shape), rk=3, oe=False)
    got = np.concatenate([oC.ravel(), oD.ravel()])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_pk_run_keeps_the_space_and_conserves():
    prob, uC, uD, _ = inputs.euler2d_quadrants(8, 2, seed=4, space=1)
    oC, oD, _, _ = ora.run2d(prob, uC, uD, nsteps=4, cfl=0.3)
    for a, b in ((1, 2), (2, 1), (2, 2)):
        assert np.all(oC[:, a, b] == 0.0) and np.all(oD[:, a, b] == 0.0)
    for u0, u1 in ((uC, oC), (uD, oD)):
        np.testing.assert_allclose(u1[:, 0, 0].sum(axis=(-1, -2)), u0[:, 0, 0].sum(axis=(-1, -2)), rtol=1e-13)


@pytest.mark.parametrize("k,rk", [(1, 2), (2, 3)])
def test_pk_advection_converges_at_order_k_plus_1(k, rk):
    """Table 2Dlinear_accuracy's problem (sin^2(pi (x + y)), velocity (1, 1)),
    P^k with an RK method of order k+1, to t = 0.2 on 8^2 -> 16^2 (k = 1) or
    16^2 -> 32^2 (k = 2): rate >= k + 1 - 0.25 in the l2 norm."""
    s, w = L.leggauss(8)
    errs = []
    for n in ((8, 16) if k == 1 else (16, 32)):
        prob, uC, uD = inputs.advection2d_sine(n, k, space=1)
        oC, _, t, _ = ora.run2d(prob, uC, uD, t_end=0.2, cfl=0.45 if k == 1 else 0.33, rk=rk)
        P = np.stack([L.legval(s, [0.0] * m + [1.0]) for m in range(k + 1)])
        vals = np.einsum("abyx,ag,bh->yxgh", oC[0], P, P)
        xc = (np.arange(n) + 0.5) / n
        X = xc[None, :, None, None] + 0.5 / n * s[None, None, :, None]
        Y = xc[:, None, None, None] + 0.5 / n * s[None, None, None, :]
        e = vals - np.sin(np.pi * (X + Y - 2 * t)) ** 2
        errs.append(math.sqrt((e ** 2 * (w[:, None] * w[None, :] / 4)).sum() / n ** 2))
    rate = math.log2(errs[0] / errs[1])
    assert rate >= k + 1 - 0.25, (errs, rate)


@pytest.mark.parametrize("rk", [1, 2, 3, 4])
@pytest.mark.parametrize("space", [0, 1])
def test_single_stages_compose_to_a_step_2d(rk, space):
    """eq:RKCDG stage by stage in 2D: chaining the single-stage function over
    the stages of forward Euler, SSP-RK2 and SSP-RK3 gives the oracle's step
    (both spaces); the last stage of classical RK4 is refused."""
    prob, uC, uD = inputs.advection2d_sine(6, 2, space=space)
    tau_max = 0.02
    tau = 0.9 * tau_max
    ul = (uC, uD)
    for l in range(rk):
        if rk == 4 and l == 3:
            with pytest.raises(ora.OracleError):
                ora.rk_stage2d(prob, rk, l, tau, tau_max, uC, uD, *ul)
            return
        ul = ora.rk_stage2d(prob, rk, l, tau, tau_max, uC, uD, *ul)
    rC, rD = ora.step2d(prob, tau, tau_max, uC, uD, rk=rk)
    np.testing.assert_allclose(ul[0], rC, rtol=1e-14, atol=1e-14 * np.abs(rC).max())
    np.testing.assert_allclose(ul[1], rD, rtol=1e-14, atol=1e-14 * np.abs(rD).max())
