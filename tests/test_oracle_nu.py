"""Pins of the non-uniform-mesh 1D oracle (Sec. 2.1 meshes, eq:1D_H, Sec. 2.2).

Each check rests on something other than the oracle itself: the uniform
oracle (separately pinned) on a uniform mesh, the exactness of the scheme for
globally polynomial data, conservation through the domain integrals, the
invariance of the method under a scaling of space and speed, and the order
of accuracy on smooth data.
"""
import math

import numpy as np
import pytest

from oracle import ora
from paper_2503_12473_amd import inputs


def _uniform_edges(prob):
    return prob.xlo + np.arange(prob.n + 1) * prob.h


def _meshes(n, L=2.0 * math.pi):
    return {"graded": inputs.smooth_graded_edges(n, 0.0, L, 0.3),
            "random": inputs.quasi_uniform_edges(n, 0.0, L, 1.5, seed=3)}


@pytest.mark.parametrize("k", [1, 2, 3])
def test_uniform_mesh_reduces_to_uniform_oracle(k):
    for prob, uC, uD in (inputs.advection_sine(16, k, phase=0.4),
                         inputs.advection_square(16, k)):
        e = _uniform_edges(prob)
        for a, b in zip(ora.rhs1d(prob, 0.1, uC, uD), ora.rhs1n(prob, e, 0.1, uC, uD)):
            np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * max(1.0, np.abs(a).max()))
        for a, b in zip(ora.delta1d(prob, uC, uD), ora.delta1n(prob, e, uC, uD)):
            np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-12)
        for a, b in zip(ora.step1d(prob, 0.05, 0.1, uC, uD), ora.step1n(prob, e, 0.05, 0.1, uC, uD)):
            np.testing.assert_allclose(b, a, rtol=0, atol=1e-13)
        for a, b in zip(ora.stats1d(prob, uC, uD), ora.stats1n(prob, e, uC, uD)):
            np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-15)


def test_uniform_mesh_reduces_to_uniform_oracle_euler():
    # periodic smooth Euler state: rho = 1 + 0.2 sin(2 pi x), v = 0.5, p = 1
    prob = inputs.Problem1D(k=2, nc=3, flux=inputs.FLUX_EULER, bc=inputs.BC_PERIODIC, n=32, xlo=0.0, xhi=1.0)
    f = lambda x: inputs.euler_conserved(1.0 + 0.2 * np.sin(2 * np.pi * x), 0.5 + 0 * x, 1.0 + 0 * x)
    uC, uD = inputs.project_1d(f, prob)
    e = _uniform_edges(prob)
    for a, b in zip(ora.rhs1d(prob, 0.02, uC, uD), ora.rhs1n(prob, e, 0.02, uC, uD)):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-11 * np.abs(a).max())
    for a, b in zip(ora.step1d(prob, 0.01, 0.02, uC, uD), ora.step1n(prob, e, 0.01, 0.02, uC, uD)):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-13)


def _poly_state(edges, k, coeffs):
    """A global polynomial projected on both meshes (exact: degree <= k)."""
    n = edges.size - 1
    p = np.polynomial.Polynomial(coeffs)
    uC, uD = inputs.project_1d_edges(lambda x: p(x)[None], 1, k, edges)
    return p, uC, uD, n


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("mesh", ["graded", "random"])
def test_polynomial_data_is_exact(k, mesh):
    """For u = one polynomial of degree <= k on both meshes, the two meshes agree
    on every overlap: the coupling term and every derivative jump vanish, and
    the CDG operator returns the projection of -a p' exactly (away from the
    periodic seam, where the polynomial is not periodic)."""
    edges = _meshes(12, L=1.0)[mesh]
    a = 1.7
    coeffs = [0.3, -1.1, 0.8, 0.45][: k + 1]
    p, uC, uD, n = _poly_state(edges, k, coeffs)
    prob = inputs.Problem1D(k=k, nc=1, flux=inputs.FLUX_ADVECTION, bc=inputs.BC_PERIODIC, n=n, xlo=0.0, xhi=1.0, a=a)
    LC, LD = ora.rhs1n(prob, edges, 0.01, uC, uD)
    dp = p.deriv()
    eC, eD = inputs.project_1d_edges(lambda x: (-a * dp(x))[None], 1, k, edges)
    inner = slice(2, n - 2)
    np.testing.assert_allclose(LC[..., inner], eC[..., inner], rtol=0, atol=1e-11)
    np.testing.assert_allclose(LD[..., inner], eD[..., inner], rtol=0, atol=1e-11)
    dC, dD = ora.delta1n(prob, edges, uC, uD)
    assert np.abs(dC[:, inner]).max() < 1e-9 * np.abs(dC).max()
    assert np.abs(dD[:, inner]).max() < 1e-9 * np.abs(dD).max()


def test_polynomial_data_is_exact_burgers_k1():
    edges = _meshes(12, L=1.0)["random"]
    p, uC, uD, n = _poly_state(edges, 1, [0.6, 0.9])
    prob = inputs.Problem1D(k=1, nc=1, flux=inputs.FLUX_BURGERS, bc=inputs.BC_PERIODIC, n=n, xlo=0.0, xhi=1.0)
    LC, LD = ora.rhs1n(prob, edges, 0.01, uC, uD)
    eC, eD = inputs.project_1d_edges(lambda x: (-p(x) * p.deriv()(x))[None], 1, 1, edges)
    inner = slice(2, n - 2)
    np.testing.assert_allclose(LC[..., inner], eC[..., inner], rtol=0, atol=1e-12)
    np.testing.assert_allclose(LD[..., inner], eD[..., inner], rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_conservation_through_domain_integrals(k):
    """Periodic: the flux terms telescope, so sum_K w_K dū_K/dt over the primal
    mesh is (1/tau_max)(int u^D - int u^C) and over the dual mesh the negative."""
    edges = _meshes(20)["random"]
    prob, uC, uD = inputs.advection_sine_edges(edges, k, freq=2)
    rng = np.random.default_rng(5)
    uD = uD + 0.05 * rng.standard_normal(uD.shape)          # make the meshes differ
    tau_max = 0.07
    LC, LD = ora.rhs1n(prob, edges, tau_max, uC, uD)
    wC = np.diff(edges)
    c = 0.5 * (edges[:-1] + edges[1:])
    wD = np.diff(np.concatenate([[c[-1] - (edges[-1] - edges[0])], c]))
    IC, ID = float(wC @ uC[0, 0]), float(wD @ uD[0, 0])
    np.testing.assert_allclose(wC @ LC[0, 0], (ID - IC) / tau_max, rtol=1e-11)
    np.testing.assert_allclose(wD @ LD[0, 0], (IC - ID) / tau_max, rtol=1e-11)
    # the step conserves sum_K w_K ū_K of both meshes together; OE keeps every cell average
    sC, sD = ora.step1n(prob, edges, 0.02, tau_max, uC, uD, rk=3, oe=True)
    np.testing.assert_allclose(wC @ sC[0, 0] + wD @ sD[0, 0], IC + ID, rtol=1e-13)
    oC, oD = ora.oe1n(prob, edges, 0.05, uC, uD)
    assert np.array_equal(oC[:, 0], uC[:, 0]) and np.array_equal(oD[:, 0], uD[:, 0])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_statistics_are_domain_means(k):
    """avg is the domain mean (width-weighted): for 0.5 + sin it is 0.5 on
    any mesh, where the plain mean of the cell averages is not."""
    edges = _meshes(24)["random"]
    prob = inputs.Problem1D(k=k, nc=1, flux=inputs.FLUX_ADVECTION, bc=inputs.BC_PERIODIC, n=24, xlo=0.0,
                            xhi=2.0 * math.pi)
    uC, uD = inputs.project_1d_edges(lambda x: (0.5 + np.sin(x))[None], 1, k, edges)
    avg, sig = ora.stats1n(prob, edges, uC, uD)
    np.testing.assert_allclose(avg, 0.5, rtol=0, atol=1e-13)
    assert abs(uC[0, 0].mean() - 0.5) > 1e-4                 # the unweighted mean differs
    np.testing.assert_allclose(sig, 1.0, rtol=0, atol=0.05 if k == 1 else 0.01)


def test_space_and_speed_scaling_invariance():
    """Scaling x by s and the speed by s leaves the modal coefficients of every
    step unchanged: h^{m-1} times the m-th derivative times beta in delta, the
    mass w_K/(2m+1), d/dx and tau_max = C h / beta all scale consistently."""
    k = 2
    e1 = _meshes(20, L=1.0)["random"]
    s = 3.0
    prob1, uC, uD = inputs.advection_sine_edges(e1, k, a=1.0)
    e3 = e1 * s
    e3[-1] = s
    prob3 = inputs.Problem1D(k=k, nc=1, flux=inputs.FLUX_ADVECTION, bc=inputs.BC_PERIODIC, n=20, xlo=0.0, xhi=s, a=s)
    a1 = ora.run1n(prob1, e1, uC, uD, nsteps=25, cfl=0.1)
    a3 = ora.run1n(prob3, e3, uC, uD, nsteps=25, cfl=0.1)
    assert a1[3] == a3[3] == 25
    np.testing.assert_allclose(a3[2], a1[2], rtol=1e-12)
    np.testing.assert_allclose(a3[0], a1[0], rtol=0, atol=1e-11)
    np.testing.assert_allclose(a3[1], a1[1], rtol=0, atol=1e-11)
    d1 = ora.delta1n(prob1, e1, a1[0], a1[1])
    d3 = ora.delta1n(prob3, e3, a1[0], a1[1])
    for x, y in zip(d1, d3):
        np.testing.assert_allclose(y, x, rtol=1e-10, atol=1e-12)


def _avg_error(prob, edges, uC, t):
    L = prob.xhi - prob.xlo
    a, b = edges[:-1], edges[1:]
    w = 2.0 * math.pi / L
    ex = -(np.cos(w * (b - prob.a * t - prob.xlo)) - np.cos(w * (a - prob.a * t - prob.xlo))) / (w * (b - a))
    return np.abs(uC[0, 0] - ex).max()


@pytest.mark.parametrize("mesh", ["graded", "random"])
@pytest.mark.parametrize("k,cfl", [(1, 0.2), (2, 0.1)])
def test_order_on_nonuniform_meshes(mesh, k, cfl):
    """Smooth advection to t = 1: the cell-average error falls at least at the
    optimal rate k+1 of the error estimate (Sec. 3) on quasi-uniform meshes."""
    errs = []
    for n in (20, 40, 80):
        edges = _meshes(n)[mesh] if mesh == "graded" else inputs.quasi_uniform_edges(n, 0.0, 2 * math.pi, 1.5, seed=1)
        prob, uC, uD = inputs.advection_sine_edges(edges, k)
        oC, _, t, _ = ora.run1n(prob, edges, uC, uD, t_end=1.0, cfl=cfl)
        assert t == 1.0
        errs.append(_avg_error(prob, edges, oC, t))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > k + 0.5, (errs, rates)


def test_rejects_bad_meshes():
    prob, uC, uD = inputs.advection_sine(8, 1)
    e = _uniform_edges(prob)
    bad = e.copy()
    bad[3], bad[4] = bad[4], bad[3]
    with pytest.raises(ora.OracleError):
        ora.rhs1n(prob, bad, 0.1, uC, uD)
    shifted = e + 0.1
    with pytest.raises(ora.OracleError):
        ora.rhs1n(prob, shifted, 0.1, uC, uD)
    outflow = inputs.Problem1D(k=1, nc=1, flux=0, bc=inputs.BC_OUTFLOW, n=8, xlo=prob.xlo, xhi=prob.xhi)
    with pytest.raises(ora.OracleError):
        ora.rhs1n(outflow, e, 0.1, uC, uD)


def test_time_step_uses_the_largest_width():
    """tau_max = C_CFL h / beta with h = max_i h_i (Sec. 2.1): for advection at
    speed a the march to t_end takes ceil(t_end a / (C h)) steps."""
    edges = inputs.quasi_uniform_edges(30, 0.0, 1.0, 1.8, seed=2)
    hmax, hmean = np.diff(edges).max(), 1.0 / 30
    prob, uC, uD = inputs.advection_sine_edges(edges, 1, a=2.0)
    t_end, cfl = 0.2, 0.2
    _, _, t, steps = ora.run1n(prob, edges, uC, uD, t_end=t_end, cfl=cfl)
    assert t == t_end
    assert steps == math.ceil(t_end * 2.0 / (cfl * hmax))
    assert steps != math.ceil(t_end * 2.0 / (cfl * hmean))
