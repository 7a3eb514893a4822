"""GPU parity of the 2D path at degrees k = 1 and 3 (the paper's P^k of
Sec. 2.1 and the tensor Q^k), and of the 2D RK methods of eq:RKCDG other than
SSP-RK3 (forward Euler, SSP-RK2, classical RK4: the order-(k+1) integrators
of the accuracy tests, Sec. 4), against the 2D oracle through the C ABI.

Meshes are ragged against the tiles (8 x 8 cells for k = 1, 4 x 4 for k = 3)
and use h_x != h_y where stated.  Bar, per component: relative L-infinity
<= 1e-10 after the run (<= 1e-12 for a single stage), equal step counts and
final times.
"""
import numpy as np
import pytest

from oracle import ora
from paper_2503_12473_amd import _lib, inputs
from paper_2503_12473_amd.api import OECDG, to_device
from paper_2503_12473_amd.inputs import Problem2D, FLUX_ADVECTION, FLUX_EULER
from tests.parity import rel

pytestmark = pytest.mark.gpu

TOL = 1e-10
ACC_CFL = {1: 0.45, 2: 0.33, 3: 0.31}    # the paper's CFL numbers for accuracy tests
ACC_RK = {1: 2, 2: 3, 3: 4}              # order k + 1


def _gpu_run(prob, uC, uD, cfl, oe=True, rk=3, **kw):
    print(f"[2d-k] k={prob.k} nx={prob.nx} ny={prob.ny} nc={prob.nc} space={prob.space} rk={rk} oe={oe} {kw}",
          flush=True)
    with OECDG(prob, cfl, oe=oe, rk=rk) as s:
        a, b = to_device(uC), to_device(uD)
        t, n = s.run(a, b, **kw)
        return a.cpu().numpy().reshape(uC.shape), b.cpu().numpy().reshape(uD.shape), t, n


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("k", [1, 3])
def test_advection_run(k, space):
    """sin^2(pi (x + y)) advected with (1, 1), N = 21 (ragged tiles), to t = 0.15,
    with the order-(k+1) RK method and the paper's accuracy CFL."""
    prob, uC, uD = inputs.advection2d_sine(21, k, space=space)
    gC, gD, t, n = _gpu_run(prob, uC, uD, ACC_CFL[k], rk=ACC_RK[k], t_end=0.15)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, t_end=0.15, cfl=ACC_CFL[k], rk=ACC_RK[k])
    assert (n, t) == (rn, rt)
    assert rel(gC, gD, rC, rD) <= TOL


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("k", [1, 3])
def test_euler_quadrants(k, space):
    """2D Euler quadrant data (the 2D workload's states), N = 18, 6 SSP-RK3 steps."""
    prob, uC, uD, _ = inputs.euler2d_quadrants(18, k, seed=0, space=space)
    gC, gD, t, n = _gpu_run(prob, uC, uD, 0.3, nsteps=6)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, nsteps=6, cfl=0.3)
    assert n == rn == 6 and t == pytest.approx(rt, rel=1e-14)
    assert rel(gC, gD, rC, rD) <= TOL


@pytest.mark.parametrize("rk", [1, 2, 4])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_rk_methods_euler(k, rk):
    """Forward Euler, SSP-RK2 and classical RK4 in 2D on Euler quadrant data,
    rectangular cells (h_x != h_y), 5 steps."""
    prob0, uC, uD, _ = inputs.euler2d_quadrants(14, k, seed=1)
    prob = Problem2D(k=k, nc=4, flux=FLUX_EULER, nx=14, ny=14, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0)
    cfl = 0.1 if rk == 1 else 0.25
    gC, gD, t, n = _gpu_run(prob, uC, uD, cfl, rk=rk, nsteps=5)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, nsteps=5, cfl=cfl, rk=rk)
    assert n == rn == 5 and t == pytest.approx(rt, rel=1e-14)
    assert rel(gC, gD, rC, rD) <= TOL


@pytest.mark.parametrize("rk", [2, 4])
def test_rk_methods_advection_p2(rk):
    prob, uC, uD = inputs.advection2d_sine(19, 2, space=1)
    gC, gD, t, n = _gpu_run(prob, uC, uD, 0.3, rk=rk, t_end=0.1)
    rC, rD, rt, rn = ora.run2d(prob, uC, uD, t_end=0.1, cfl=0.3, rk=rk)
    assert (n, t) == (rn, rt)
    assert rel(gC, gD, rC, rD) <= TOL


@pytest.mark.parametrize("k", [1, 3])
def test_single_stages(k):
    """oecdg_stage for each SSP-RK3 stage at k = 1 and 3 against one oracle stage
    (built from the oracle's operator and damping), and the RK4 stages that read
    only u^n and u^l; RK4's last stage is refused."""
    prob, uC, uD, _ = inputs.euler2d_quadrants(12, k, seed=2)
    tau = 0.2 / (2.0 / prob.hx)
    rng = np.random.default_rng(5)
    lC = uC * (1 + 0.01 * rng.standard_normal(uC.shape))
    lD = uD * (1 + 0.01 * rng.standard_normal(uD.shape))
    for rk, stages in ((3, (0, 1, 2)), (4, (0, 1, 2))):
        c, d = _tables(rk)
        with OECDG(prob, 0.3, rk=rk) as s:
            gn = (to_device(uC), to_device(uD))
            gl = (to_device(lC), to_device(lD))
            for l in stages:
                print(f"[2d-k] stage rk={rk} k={k} l={l}", flush=True)
                oC, oD = s.stage(l, tau, 1.2 * tau, gn[0], gn[1], gl[0], gl[1])
                inC, inD = (uC, uD) if l == 0 else (lC, lD)
                LC, LD = ora.rhs2d(prob, 1.2 * tau, inC, inD)
                hC = (c[l][0] * uC if l > 0 else 0.0) + c[l][l] * inC + tau * d[l][l] * LC
                hD = (c[l][0] * uD if l > 0 else 0.0) + c[l][l] * inD + tau * d[l][l] * LD
                rC, rD = ora.oe2d(prob, tau, hC, hD)
                assert rel(oC.cpu().numpy(), oD.cpu().numpy(), rC, rD) <= 1e-12, (rk, l)
            if rk == 4:
                with pytest.raises(_lib.OECDGError) as e:
                    s.stage(3, tau, tau, gn[0], gn[1], gl[0], gl[1])
                assert e.value.code == _lib.EUNSUPPORTED


def _tables(rk):
    c = np.zeros((4, 4))
    d = np.zeros((4, 4))
    if rk == 3:
        c[0, 0], d[0, 0] = 1, 1
        c[1, 0], c[1, 1], d[1, 1] = 0.75, 0.25, 0.25
        c[2, 0], c[2, 2], d[2, 2] = 1 / 3, 2 / 3, 2 / 3
    else:
        c[0, 0], d[0, 0] = 1, 0.5
        c[1, 0], d[1, 1] = 1, 0.5
        c[2, 0], d[2, 2] = 1, 1
    return c, d


def test_full_size_p3_conserves_and_stays_physical():
    """k = 3 on a 512^2 Euler quadrant mesh for 4 steps (16384 tiles of 4 x 4):
    per-mesh conservation of every component's cell averages and positivity."""
    prob, uC, uD, _ = inputs.euler2d_quadrants(512, 3, seed=0)
    gC, gD, t, n = _gpu_run(prob, uC, uD, 0.2, nsteps=4)
    assert n == 4
    for u0, u1 in ((uC, gC), (uD, gD)):
        s0 = u0[:, 0, 0].sum(axis=(1, 2))
        s1 = u1[:, 0, 0].sum(axis=(1, 2))
        assert np.all(np.abs(s1 - s0) <= 1e-11 * np.abs(u0[:, 0, 0]).sum(axis=(1, 2)))
    g = prob.gamma
    for u in (gC, gD):
        rho = u[0, 0, 0]
        p = (g - 1) * (u[3, 0, 0] - 0.5 * (u[1, 0, 0] ** 2 + u[2, 0, 0] ** 2) / rho)
        assert rho.min() > 0 and p.min() > 0
