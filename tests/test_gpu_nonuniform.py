"""GPU parity of oecdg_run_nonuniform (periodic non-uniform 1D meshes, Sec. 2.1)
against the non-uniform oracle.

Meshes: the seeded random mesh (widths ratio <= 1.5) and the smooth grading of
amplitude 0.3; sizes span several workgroups of 64 cells with a ragged tail.
Bar: relative L-infinity error <= 1e-10 after the run, equal step counts and
final times.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ora
from paper_2503_12473_amd import _lib, inputs
from paper_2503_12473_amd.api import OECDG, to_device
from tests.test_gpu_1d import RUN_TOL, _rel

pytestmark = pytest.mark.gpu


def _mesh(kind, n, xlo=0.0, xhi=2.0 * math.pi, seed=0):
    if kind == "graded":
        return inputs.smooth_graded_edges(n, xlo, xhi, 0.3)
    return inputs.quasi_uniform_edges(n, xlo, xhi, 1.5, seed=seed)


def _gpu(prob, edges, uC, uD, cfl, rk=3, oe=True, **kw):
    with OECDG(prob, cfl, oe=oe, rk=rk) as s:
        a, b = to_device(uC), to_device(uD)
        t, n = s.run_nonuniform(edges, a, b, **kw)
        torch.cuda.synchronize()
        return a.cpu().numpy().reshape(uC.shape), b.cpu().numpy().reshape(uD.shape), t, n


def _burgers(edges, k):
    e = np.asarray(edges)
    prob = inputs.Problem1D(k=k, nc=1, flux=inputs.FLUX_BURGERS, bc=inputs.BC_PERIODIC, n=e.size - 1,
                            xlo=float(e[0]), xhi=float(e[-1]))
    uC, uD = inputs.project_1d_edges(lambda x: (np.sin(x) + 0.5)[None], 1, k, e)
    return prob, uC, uD


def _euler(edges, k):
    e = np.asarray(edges)
    prob = inputs.Problem1D(k=k, nc=3, flux=inputs.FLUX_EULER, bc=inputs.BC_PERIODIC, n=e.size - 1,
                            xlo=float(e[0]), xhi=float(e[-1]))
    L = prob.xhi - prob.xlo
    f = lambda x: inputs.euler_conserved(1.0 + 0.2 * np.sin(2 * np.pi * (x - prob.xlo) / L), 0.5 + 0 * x, 1.0 + 0 * x)
    uC, uD = inputs.project_1d_edges(f, 3, k, e)
    return prob, uC, uD


@pytest.mark.parametrize("kind", ["graded", "random"])
@pytest.mark.parametrize("k,cfl", [(1, 0.2), (2, 0.1), (3, 0.08)])
def test_advection_run(kind, k, cfl):
    """sin x on [0, 2 pi], N = 600 (nine full workgroups of 64 cells and a ragged one), to T = 1."""
    edges = _mesh(kind, 600)
    prob, uC, uD = inputs.advection_sine_edges(edges, k)
    gC, gD, t, n = _gpu(prob, edges, uC, uD, cfl, t_end=1.0)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, t_end=1.0, cfl=cfl)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("kind", ["graded", "random"])
@pytest.mark.parametrize("rk,k,cfl", [(3, 2, 0.1), (2, 1, 0.2), (1, 0, 0.3)])
def test_burgers_through_shock(kind, rk, k, cfl):
    """sin x + 0.5, N = 300, through shock formation to T = 2.2 (OE active in every stage)."""
    edges = _mesh(kind, 300, seed=4)
    prob, uC, uD = _burgers(edges, k)
    gC, gD, t, n = _gpu(prob, edges, uC, uD, cfl, rk=rk, t_end=2.2)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, t_end=2.2, cfl=cfl, rk=rk)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k,oe", [(2, True), (2, False), (1, True), (3, True)])
def test_euler_smooth(k, oe):
    """Smooth periodic Euler density wave, N = 513, 40 steps."""
    edges = _mesh("random", 513, 0.0, 1.0, seed=7)
    prob, uC, uD = _euler(edges, k)
    cfl = {1: 0.15, 2: 0.1, 3: 0.08}[k]
    gC, gD, t, n = _gpu(prob, edges, uC, uD, cfl, oe=oe, nsteps=40)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, nsteps=40, cfl=cfl, oe=oe)
    # the Euler wave speed goes through a square root and divisions, so the
    # summed steps agree to rounding (a final time t_end is hit exactly)
    assert n == rn == 40 and abs(t - rt) <= 1e-13 * rt
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_uniform_edges_match_uniform_path():
    """On a uniform mesh the non-uniform entry point equals oecdg_run to rounding."""
    prob, uC, uD = inputs.advection_sine(1000, 2, phase=0.3)
    edges = prob.xlo + np.arange(prob.n + 1) * prob.h
    edges[-1] = prob.xhi
    gC, gD, t, n = _gpu(prob, edges, uC, uD, 0.1, t_end=0.5)
    with OECDG(prob, 0.1) as s:
        a, b = to_device(uC), to_device(uD)
        t2, n2 = s.run(a, b, t_end=0.5)
        hC, hD = a.cpu().numpy().reshape(uC.shape), b.cpu().numpy().reshape(uD.shape)
    assert n == n2 and abs(t - t2) == 0.0
    assert _rel(gC, gD, hC, hD) <= RUN_TOL


def test_full_size_mesh():
    """N = 16384, k = 2, SSP-RK3, 20 steps on a random mesh: parity with the
    oracle at the size of the 1D headline workload, and conservation of the
    width-weighted totals of both meshes."""
    edges = _mesh("random", 16384, seed=11)
    prob, uC, uD = inputs.advection_sine_edges(edges, 2)
    gC, gD, t, n = _gpu(prob, edges, uC, uD, 0.1, nsteps=20)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, nsteps=20, cfl=0.1)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL
    wC = np.diff(edges)
    c = 0.5 * (edges[:-1] + edges[1:])
    wD = np.diff(np.concatenate([[c[-1] - (edges[-1] - edges[0])], c]))
    tot0 = wC @ uC[0, 0] + wD @ uD[0, 0]
    np.testing.assert_allclose(wC @ gC[0, 0] + wD @ gD[0, 0], tot0, rtol=0, atol=1e-12)


def test_repeat_calls_and_step_limit():
    """nsteps limit with t_end = inf; two calls on one handle give the same bits."""
    edges = _mesh("graded", 777)
    prob, uC, uD = inputs.advection_sine_edges(edges, 1)
    with OECDG(prob, 0.2) as s:
        outs = []
        for _ in range(2):
            a, b = to_device(uC), to_device(uD)
            t, n = s.run_nonuniform(edges, a, b, nsteps=9)
            outs.append((a.cpu().numpy(), b.cpu().numpy(), t, n))
    assert outs[0][3] == outs[1][3] == 9 and outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, nsteps=9, cfl=0.2)
    assert rt == outs[0][2]
    assert _rel(outs[0][0].reshape(uC.shape), outs[0][1].reshape(uD.shape), rC, rD) <= RUN_TOL


def test_errors():
    edges = _mesh("random", 64)
    prob, uC, uD = inputs.advection_sine_edges(edges, 1)
    bad = edges.copy()
    bad[5], bad[6] = bad[6], bad[5]
    with OECDG(prob, 0.2) as s:
        a, b = to_device(uC), to_device(uD)
        with pytest.raises(_lib.OECDGError, match="invalid"):
            s.run_nonuniform(bad, a, b, nsteps=1)
        with pytest.raises(_lib.OECDGError, match="invalid"):
            s.run_nonuniform(edges + 0.1, a, b, nsteps=1)
    with OECDG(prob, 0.2, rk=4) as s:
        with pytest.raises(_lib.OECDGError, match="unsupported"):
            s.run_nonuniform(edges, to_device(uC), to_device(uD), nsteps=1)
    with OECDG(prob, 0.2) as s:
        a, b = to_device(uC), to_device(uD)
        with pytest.raises(ValueError, match="edges"):       # the wrapper checks the length (nx + 1)
            s.run_nonuniform(edges[:-1], a, b, nsteps=1)
        with pytest.raises(ValueError, match="edges"):
            s.run_nonuniform(edges[None], a, b, nsteps=1)
    out = inputs.Problem1D(k=1, nc=1, flux=0, bc=inputs.BC_OUTFLOW, n=64, xlo=prob.xlo, xhi=prob.xhi)
    with OECDG(out, 0.2) as s:
        a, b = s.empty_state()
        with pytest.raises(_lib.OECDGError, match="unsupported"):
            s.run_nonuniform(edges, a, b, nsteps=1)


def test_bench_workload_full_size():
    """The measured non-uniform workload itself: periodic Euler density wave on
    the seed-0 random mesh of N = 16384 cells (width ratio <= 1.5), P2, SSP-RK3,
    CFL 0.1, 10 steps through the same entry point."""
    edges = inputs.quasi_uniform_edges(16384, 0.0, 1.0, 1.5, seed=0)
    prob, uC, uD = _euler(edges, 2)
    gC, gD, t, n = _gpu(prob, edges, uC, uD, 0.1, nsteps=10)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, nsteps=10, cfl=0.1)
    assert n == rn == 10 and abs(t - rt) <= 1e-13 * rt
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_more_workgroups_than_threads():
    """N = 70000: 1094 workgroups, more than the 384 partials per row that the
    192 threads reducing their statistics load at first, so the strided part of
    that reduction runs too."""
    edges = _mesh("random", 70000, seed=13)
    prob, uC, uD = inputs.advection_sine_edges(edges, 1, freq=3)
    gC, gD, t, n = _gpu(prob, edges, uC, uD, 0.2, nsteps=5)
    rC, rD, rt, rn = ora.run1n(prob, edges, uC, uD, nsteps=5, cfl=0.2)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL
