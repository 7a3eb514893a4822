"""GPU parity of reflective walls (1D Euler) against the oracle.

Ghost primal cells -1 and n mirror cells 0 and n-1 (mode m times (-1)^m, the
momentum negated); the kernel loads the mirror of the undamped cells for the
damping coefficients and re-mirrors the damped cells before the operator.
Bar: relative L-infinity error <= 1e-10 after the run, equal step counts and
final times.  The paper's data (rho = 1, p = 1000, 0.01, 100) run with the
problem's tolerance of a non-positive cell-average pressure; most cases use
pressures (100, 1, 10) and densities (1, 0.5, 0.8), which keep every cell
average physical.  Meshes put the jumps at x = 0.1 and 0.9 on primal cell
edges (N a multiple of 10).
"""
import numpy as np
import pytest
import torch

from oracle import ora
from paper_2503_12473_amd import _lib, inputs
from paper_2503_12473_amd.api import OECDG, to_device
from tests.test_gpu_1d import RUN_TOL, _rel, gpu_run

pytestmark = pytest.mark.gpu

BLAST = dict(pressures=(100.0, 1.0, 10.0), densities=(1.0, 0.5, 0.8))
CFL = {1: 0.52, 2: 0.3, 3: 0.2}        # the paper's values for discontinuous data


@pytest.mark.parametrize("k", [1, 2, 3])
def test_blast_waves_run(k):
    """Two blast waves between walls, N = 960 (the paper's mesh), to T = 0.004."""
    prob, uC, uD = inputs.euler_blast_waves(960, k, **BLAST)
    gC, gD, t, ns = gpu_run(prob, uC, uD, CFL[k], t_end=0.004)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.004, cfl=CFL[k])
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k", [1, 2, 3])
def test_paper_blast_waves_run(k):
    """The paper's two-blast-wave data themselves (rho = 1, p = 1000, 0.01, 100),
    N = 960, 150 steps: the uniform density stays exactly uniform through the
    first stage on both sides (its sigma is exactly zero), and the cell
    averages that carry a small non-positive pressure next to the weaker
    blast are tolerated by the problem's flag on both sides."""
    prob, uC, uD = inputs.euler_blast_waves(960, k)
    assert prob.allow_negative_pressure
    gC, gD, t, ns = gpu_run(prob, uC, uD, CFL[k], nsteps=150)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=150, cfl=CFL[k])
    assert ns == rn == 150 and t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_paper_blast_waves_strict_mode_reports_the_pressure():
    """Without the flag, the same data end in ENONPHYSICAL, as in the oracle."""
    prob, uC, uD = inputs.euler_blast_waves(960, 2, allow_negative_pressure=False)
    with pytest.raises(ora.OracleError):
        ora.run1d(prob, uC, uD, nsteps=20, cfl=0.3)
    with pytest.raises(_lib.OECDGError) as e:
        gpu_run(prob, uC, uD, 0.3, nsteps=20)
    assert e.value.code == _lib.ENONPHYSICAL


@pytest.mark.parametrize("oe", [True, False])
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("n", [37, 128, 130])
def test_smooth_walls_run(n, k, oe):
    """Smooth data with walls (one tile, a mesh that ends on a tile boundary
    so that a tile holds only the last dual cell, a ragged tail), OE on and off."""
    prob, uC, uD = inputs.euler_walls_smooth(n, k)
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.3, oe=oe, t_end=0.05)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.05, cfl=0.3, oe=oe)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("tile", [32, 64, 128])
def test_execution_modes_and_tiles(tile):
    """Eager, graph and persistent launches give identical bits; N = 640 puts
    the last dual cell alone in a tile for tiles 32 to 128."""
    prob, uC, uD = inputs.euler_blast_waves(640, 2, **BLAST)
    outs = [gpu_run(prob, uC, uD, 0.3, mode=m, tile=tile, t_end=0.01)
            for m in (_lib.MODE_EAGER, _lib.MODE_GRAPH, _lib.MODE_PERSISTENT)]
    assert outs[0][3] > 70
    for o in outs[1:]:
        assert o[2] == outs[0][2] and o[3] == outs[0][3]
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.01, cfl=0.3)
    assert outs[0][3] == rn
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


def test_full_size_steps():
    """N = 16000 with walls (the benchmark's scale, jumps on cell edges), 12
    steps, against the oracle."""
    prob, uC, uD = inputs.euler_blast_waves(16000, 2, **BLAST)
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.3, nsteps=12)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=12, cfl=0.3)
    assert ns == rn == 12
    assert t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_full_size_conservation_and_wall_parity():
    """N = 16000, P2, 400 steps (beyond the oracle's quick reach): the
    integrals over [0, 1] of density and energy on both meshes stay constant
    and the wall dual cells keep even density and energy, odd momentum."""
    prob, uC, uD = inputs.euler_blast_waves(16000, 2, **BLAST)
    gC, gD, _, ns = gpu_run(prob, uC, uD, 0.3, nsteps=400)
    assert ns == 400

    def integrals(c, d):
        return c[:, 0].sum(axis=-1), d[:, 0, 1:-1].sum(axis=-1) + 0.5 * (d[:, 0, 0] + d[:, 0, -1])

    (c0, d0), (c1, d1) = integrals(uC, uD), integrals(gC, gD)
    for q in (0, 2):
        assert c1[q] == pytest.approx(c0[q], rel=1e-12)
        assert d1[q] == pytest.approx(d0[q], rel=1e-12)
    scale = np.abs(gD).max()
    for j in (0, prob.n_dual - 1):
        for q in range(3):
            for m in range(3):
                if m % 2 != (1 if q == 1 else 0):
                    assert abs(gD[q, m, j]) <= 1e-13 * scale, (j, q, m)
    rho = gC[0, 0]
    p = 0.4 * (gC[2, 0] - 0.5 * gC[1, 0] ** 2 / rho)
    assert rho.min() > 0 and p.min() > 0


def test_batch_of_walls_and_outflow():
    """Walled and outflow instances of mixed degree in one batch: each matches
    its own oracle run."""
    specs = [inputs.euler_blast_waves(300, 2, **BLAST), inputs.euler_riemann(257, 1, inputs.riemann_states(0)),
             inputs.euler_walls_smooth(100, 3), inputs.euler_blast_waves(129, 1, **BLAST)]
    probs = [s[0] for s in specs]
    print(f"[walls batch] {len(probs)} instances, 20 steps", flush=True)
    with OECDG(probs, 0.15) as s:
        gC = torch.cat([to_device(x[1]) for x in specs])
        gD = torch.cat([to_device(x[2]) for x in specs])
        s.run(gC, gD, nsteps=20)
        offC, offD = s.off_primal, s.off_dual
        gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    for b, (p, uC, uD) in enumerate(specs):
        rC, rD, _, _ = ora.run1d(p, uC, uD, nsteps=20, cfl=0.15)
        bC = gC[offC[b]:offC[b + 1]].reshape(rC.shape)
        bD = gD[offD[b]:offD[b + 1]].reshape(rD.shape)
        assert _rel(bC, bD, rC, rD) <= RUN_TOL, b


def test_walls_need_the_euler_flux():
    prob = inputs.Problem1D(k=1, nc=1, flux=inputs.FLUX_BURGERS, bc=inputs.BC_REFLECTIVE, n=64, xlo=0.0, xhi=1.0)
    with pytest.raises(_lib.OECDGError) as e:
        OECDG(prob, 0.2)
    assert e.value.code == _lib.EUNSUPPORTED


@pytest.mark.parametrize("rk,k,cfl", [(4, 3, 0.2), (2, 1, 0.45)])
def test_walls_with_other_rk_methods(rk, k, cfl):
    """Walls combined with classical RK4 (the accumulated damped stages) and
    SSP-RK2, blast-wave data, N = 640, to T = 0.004."""
    prob, uC, uD = inputs.euler_blast_waves(640, k, **BLAST)
    gC, gD, t, ns = gpu_run(prob, uC, uD, cfl, rk=rk, t_end=0.004)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.004, cfl=cfl, rk=rk)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_walls_with_tail_tile():
    """Walls on N = 16384 (dual cell 16384, on the right wall, carried by the
    last tile's extra wave), smooth data, 15 steps against the oracle."""
    prob, uC, uD = inputs.euler_walls_smooth(16384, 2)
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.3, nsteps=15)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=15, cfl=0.3)
    assert ns == rn == 15
    assert _rel(gC, gD, rC, rD) <= RUN_TOL
