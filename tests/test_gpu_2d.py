"""2D path (tensor Q2, periodic primal/dual Cartesian meshes) against the 2D
CPU oracle, through the C ABI.  Bar: 1e-10 relative L-infinity over both
meshes and all components and modes (the FP64 plain-path tolerance)."""
import math

import numpy as np
import pytest

from tests.parity import rel
import torch

from oracle import ora
from paper_2503_12473_amd import inputs
from paper_2503_12473_amd.api import OECDG, to_device
from paper_2503_12473_amd.inputs import Problem2D, FLUX_ADVECTION, FLUX_EULER

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _rel(g, r):
    return rel(g[0], g[1], r[0], r[1])


def _gpu_run(prob, uC, uD, cfl, oe=True, **kw):
    with OECDG(prob, cfl, oe=oe) as s:
        a, b = to_device(uC), to_device(uD)
        t, n = s.run(a, b, **kw)
        return (a.cpu().numpy().reshape(uC.shape), b.cpu().numpy().reshape(uD.shape)), t, n


def _quadrants(n, seed):
    prob, uC, uD, _ = inputs.euler2d_quadrants(n, 2, seed=seed)
    return prob, uC, uD


@pytest.mark.parametrize("n,steps", [(8, 1), (16, 1), (16, 6)])
def test_euler_quadrants_match_oracle(n, steps):
    prob, uC, uD = _quadrants(n, 0)
    print(f"[2d] euler quadrants n={n} steps={steps}", flush=True)
    g, t, gn = _gpu_run(prob, uC, uD, 0.3, nsteps=steps)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, nsteps=steps, cfl=0.3)
    assert gn == rn == steps and t == pytest.approx(rt, rel=1e-14)
    e = _rel(g, (rC, rD))
    print(f"[2d] rel err {e:.3e}", flush=True)
    assert e <= TOL


def test_ragged_tiles_and_rectangular_cells():
    """nx, ny not multiples of the 8 x 8 tile; hx != hy; seeded smooth + jump data."""
    prob0, _, _ = _quadrants(8, 1)
    prob = Problem2D(k=2, nc=4, flux=FLUX_EULER, nx=12, ny=10, xlo=0.0, xhi=1.2, ylo=0.0, yhi=0.7)
    rng = np.random.default_rng(7)
    quads = rng.uniform(0.3, 1.0, size=(4, 4))

    def f(X, Y):
        qi = (np.mod(X, 1.2) >= 0.6).astype(int) + 2 * (np.mod(Y, 0.7) >= 0.35).astype(int)
        rho = 1.0 + 0.2 * np.sin(2 * math.pi * X / 1.2) + quads[qi, 0]
        u, v, p = quads[qi, 1] - 0.6, quads[qi, 2] - 0.6, quads[qi, 3]
        return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])

    uC, uD = inputs.project_2d(f, prob)
    g, _, _ = _gpu_run(prob, uC, uD, 0.3, nsteps=3)
    rC, rD, _, _ = ora.run2d(prob, uC, uD, nsteps=3, cfl=0.3)
    assert _rel(g, (rC, rD)) <= TOL


def test_small_mesh_wraps_inside_one_tile():
    prob = Problem2D(k=2, nc=4, flux=FLUX_EULER, nx=4, ny=3, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0)
    _, uC8, uD8, _ = inputs.euler2d_quadrants(8, 2, seed=2)
    uC = np.ascontiguousarray(uC8[..., :3, :4])
    uD = np.ascontiguousarray(uD8[..., :3, :4])
    g, _, _ = _gpu_run(prob, uC, uD, 0.3, nsteps=2)
    rC, rD, _, _ = ora.run2d(prob, uC, uD, nsteps=2, cfl=0.3)
    assert _rel(g, (rC, rD)) <= TOL


def test_advection_sine_matches_oracle():
    prob, uC, uD = inputs.advection2d_sine(16, 2)
    prob = Problem2D(k=2, nc=1, flux=FLUX_ADVECTION, nx=16, ny=16, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, a=1.0, b=-0.7)
    uC, uD = inputs.project_2d(lambda X, Y: (np.sin(math.pi * (X + Y)) ** 2)[None], prob)
    g, _, _ = _gpu_run(prob, uC, uD, 0.3, nsteps=8)
    rC, rD, _, _ = ora.run2d(prob, uC, uD, nsteps=8, cfl=0.3)
    assert _rel(g, (rC, rD)) <= TOL


def test_without_oe_matches_oracle():
    prob, uC, uD = _quadrants(16, 3)
    g, _, _ = _gpu_run(prob, uC, uD, 0.2, oe=False, nsteps=3)
    rC, rD, _, _ = ora.run2d(prob, uC, uD, nsteps=3, cfl=0.2, oe=False)
    assert _rel(g, (rC, rD)) <= TOL


def test_run_to_final_time_clips_last_step():
    prob, uC, uD = _quadrants(8, 4)
    g, t, n = _gpu_run(prob, uC, uD, 0.3, t_end=0.02)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, t_end=0.02, cfl=0.3)
    assert t == 0.02 and rt == 0.02 and n == rn
    assert _rel(g, (rC, rD)) <= TOL


def test_fixed_step():
    prob, uC, uD = _quadrants(8, 5)
    g, _, n = _gpu_run(prob, uC, uD, 0.3, nsteps=4, dt_fixed=1e-3)
    rC, rD, _, _ = ora.run2d(prob, uC, uD, nsteps=4, dt_fixed=1e-3)
    assert n == 4 and _rel(g, (rC, rD)) <= TOL


def test_dt_matches_oracle_wavespeeds():
    prob, uC, uD = _quadrants(16, 6)
    with OECDG(prob, 0.3) as s:
        dt = s.dt(to_device(uC), to_device(uD))
    bx, by = ora.max_wavespeeds2d(prob, uC, uD)
    assert dt == pytest.approx(0.3 / (bx / prob.hx + by / prob.hy), rel=1e-14)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_single_stage_matches_oracle_composition(l):
    """oecdg_stage: F_tau(c_l0 u^n + c_ll u^l + tau d_ll L(u^l)) from the oracle's operator and OE."""
    prob, uC, uD = _quadrants(8, 7)
    prob2, vC, vD = _quadrants(8, 8)
    tau, tm = 2e-3, 3e-3
    c = {0: (0.0, 1.0, 1.0), 1: (0.75, 0.25, 0.25), 2: (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)}[l]
    ul = (uC, uD) if l == 0 else (vC, vD)
    LC, LD = ora.rhs2d(prob, tm, *ul)
    hC = c[0] * uC + (c[1] * ul[0] + tau * c[2] * LC)
    hD = c[0] * uD + (c[1] * ul[1] + tau * c[2] * LD)
    if l == 0:
        hC, hD = ul[0] + tau * LC, ul[1] + tau * LD
    rC, rD = ora.oe2d(prob, tau, hC, hD)
    with OECDG(prob, 0.3) as s:
        out = s.stage(l, tau, tm, to_device(uC), to_device(uD),
                      None if l == 0 else to_device(vC), None if l == 0 else to_device(vD))
        g = (out[0].cpu().numpy().reshape(uC.shape), out[1].cpu().numpy().reshape(uD.shape))
    assert _rel(g, (rC, rD)) <= 1e-12


def test_conservation_and_positivity_64():
    prob, uC, uD = _quadrants(64, 0)
    g, _, n = _gpu_run(prob, uC, uD, 0.3, nsteps=20)
    for u0, u1 in ((uC, g[0]), (uD, g[1])):
        s0 = u0[:, 0, 0].sum(axis=(1, 2))
        s1 = u1[:, 0, 0].sum(axis=(1, 2))
        assert np.all(np.abs(s1 - s0) <= 1e-12 * np.abs(u0[:, 0, 0]).sum(axis=(1, 2)))
        assert np.all(u1[0, 0, 0] > 0.0)


@pytest.mark.timeout(300)
def test_full_workload_conserves_stays_physical_and_repeats():
    """The 2D workload at full size (1024^2 primal + dual, Q2, CFL 0.3, 500
    steps), beyond what the oracle can run: the cell averages of every
    component sum to their initial values on each mesh (the operator is
    conservative and OE keeps the averages), density and pressure stay
    positive at every cell average, and a second run gives the same bits."""
    prob, uC, uD = _quadrants(1024, 0)
    g, t, n = _gpu_run(prob, uC, uD, 0.3, nsteps=500)
    assert n == 500 and np.isfinite(t)
    g2, t2, n2 = _gpu_run(prob, uC, uD, 0.3, nsteps=500)
    assert n2 == n and t2 == t and np.array_equal(g[0], g2[0]) and np.array_equal(g[1], g2[1])
    gamma = prob.gamma
    for u0, u1 in ((uC, g[0]), (uD, g[1])):
        assert np.isfinite(u1).all()
        s0 = u0[:, 0, 0].sum(axis=(1, 2))
        s1 = u1[:, 0, 0].sum(axis=(1, 2))
        assert np.all(np.abs(s1 - s0) <= 1e-11 * np.abs(u0[:, 0, 0]).sum(axis=(1, 2))), (s0, s1)
        rho, mx, my, E = u1[0, 0, 0], u1[1, 0, 0], u1[2, 0, 0], u1[3, 0, 0]
        p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
        assert rho.min() > 0.0 and p.min() > 0.0


def test_nonfinite_input_is_reported():
    """A NaN in a higher mode of one cell: the 2D run stops with ENONFINITE."""
    from paper_2503_12473_amd import _lib
    prob, uC, uD = _quadrants(16, 0)
    uC = uC.copy()
    uC[2, 1, 1, 5, 7] = float("nan")
    with pytest.raises(_lib.OECDGError) as e:
        _gpu_run(prob, uC, uD, 0.3, nsteps=3)
    assert e.value.code == _lib.ENONFINITE
