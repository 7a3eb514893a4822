"""GPU parity of the 2D total-degree space P^2 (the paper's own 2D space,
Sec. 2.1) against the 2D oracle, through the C ABI.

The library keeps the tensor layout and zeroes the modes a + b > 2 of every
stage output (in an orthogonal basis that is the P^2 Galerkin scheme); the
oracle truncates every stage's combination.  Bar: 1e-10 relative L-infinity
over both meshes, all components and modes.
"""
import numpy as np
import pytest

from tests.parity import rel

from oracle import ora
from paper_2503_12473_amd import inputs
from paper_2503_12473_amd.api import OECDG, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-10
HIGH = [(1, 2), (2, 1), (2, 2)]          # the tensor slots outside P^2


def _rel(g, r):
    return rel(g[0], g[1], r[0], r[1])


def _gpu_run(prob, uC, uD, cfl, oe=True, **kw):
    print(f"[pk] nx={prob.nx} nc={prob.nc} space={prob.space} oe={oe} {kw}", flush=True)
    with OECDG(prob, cfl, oe=oe) as s:
        a, b = to_device(uC), to_device(uD)
        t, n = s.run(a, b, **kw)
        return (a.cpu().numpy().reshape(uC.shape), b.cpu().numpy().reshape(uD.shape)), t, n


def _high_modes_zero(u):
    return all(np.all(u[:, i, j] == 0.0) for i, j in HIGH)


@pytest.mark.parametrize("n", [20, 37])
def test_advection_p2_run(n):
    """u_t + u_x + u_y = 0, sin^2(pi (x + y)), CFL 0.33, to t = 0.2 (ragged tiles)."""
    prob, uC, uD = inputs.advection2d_sine(n, 2, space=1)
    g, t, gn = _gpu_run(prob, uC, uD, 0.33, t_end=0.2)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, t_end=0.2, cfl=0.33)
    assert (gn, t) == (rn, rt)
    assert _rel(g, (rC, rD)) <= TOL
    assert _high_modes_zero(g[0]) and _high_modes_zero(g[1])


@pytest.mark.parametrize("oe", [True, False])
def test_euler_p2_quadrants(oe):
    prob, uC, uD, _ = inputs.euler2d_quadrants(16, 2, seed=0, space=1)
    g, t, gn = _gpu_run(prob, uC, uD, 0.3, oe=oe, nsteps=6)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, nsteps=6, cfl=0.3, oe=oe)
    assert gn == rn == 6 and t == pytest.approx(rt, rel=1e-14)
    assert _rel(g, (rC, rD)) <= TOL
    assert _high_modes_zero(g[0]) and _high_modes_zero(g[1])


def test_p2_differs_from_q2():
    """The same data in Q^2 and P^2 give different runs (the space matters)."""
    probq, uC, uD = inputs.advection2d_sine(16, 2, space=0)
    probp, pC, pD = inputs.advection2d_sine(16, 2, space=1)
    gq, _, _ = _gpu_run(probq, uC, uD, 0.33, nsteps=10)
    gp, _, _ = _gpu_run(probp, pC, pD, 0.33, nsteps=10)
    assert _rel(gp, gq) > 1e-6


def test_input_high_modes_are_ignored():
    """oecdg_run with P^2 drops whatever the input holds in the slots a + b > 2."""
    prob, uC, uD = inputs.advection2d_sine(24, 2, space=1)
    rng = np.random.default_rng(3)
    nC, nD = uC.copy(), uD.copy()
    for i, j in HIGH:
        nC[:, i, j] = rng.normal(size=nC[:, i, j].shape)
        nD[:, i, j] = rng.normal(size=nD[:, i, j].shape)
    a, _, _ = _gpu_run(prob, uC, uD, 0.33, nsteps=4)
    b, _, _ = _gpu_run(prob, nC, nD, 0.33, nsteps=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_full_mesh_p2_properties():
    """Euler quadrant data in P^2 on the full 1024^2 mesh, 20 steps: per-mesh
    conservation of every component's cell averages, positive density and
    pressure, high slots exactly zero."""
    prob, uC, uD, _ = inputs.euler2d_quadrants(1024, 2, seed=0, space=1)
    g, _, gn = _gpu_run(prob, uC, uD, 0.3, nsteps=20)
    assert gn == 20
    for u0, u1 in ((uC, g[0]), (uD, g[1])):
        s0, s1 = u0[:, 0, 0].sum(axis=(-1, -2)), u1[:, 0, 0].sum(axis=(-1, -2))
        assert np.all(np.abs(s1 - s0) <= 1e-11 * np.abs(u0[:, 0, 0]).sum(axis=(-1, -2)) + 1e-9)
        rho = u1[0, 0, 0]
        p = 0.4 * (u1[3, 0, 0] - 0.5 * (u1[1, 0, 0] ** 2 + u1[2, 0, 0] ** 2) / rho)
        assert rho.min() > 0 and p.min() > 0
        assert _high_modes_zero(u1)


def test_single_stage_ignores_high_slots():
    """oecdg_stage with P^2: the slots a + b > 2 of u^n and u^l are not read,
    and the output's are zero."""
    prob, uC, uD, _ = inputs.euler2d_quadrants(16, 2, seed=2, space=1)
    rng = np.random.default_rng(5)
    nC, nD = uC.copy(), uD.copy()
    for i, j in HIGH:
        nC[:, i, j] = rng.normal(size=nC[:, i, j].shape)
        nD[:, i, j] = rng.normal(size=nD[:, i, j].shape)
    outs = []
    for c, d in ((uC, uD), (nC, nD)):
        with OECDG(prob, 0.3) as s:
            dt = s.dt(to_device(c), to_device(d))
            o = s.stage(1, 0.8 * dt, dt, to_device(c), to_device(d), to_device(c), to_device(d))
            outs.append((o[0].cpu().numpy().reshape(uC.shape), o[1].cpu().numpy().reshape(uD.shape)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert _high_modes_zero(outs[0][0]) and _high_modes_zero(outs[0][1])
