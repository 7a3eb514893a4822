"""GPU parity of inflow boundaries (1D Euler) against the oracle.

The primal ghost cells left of cell 0 and right of cell n-1 hold fixed states
given with oecdg_set_inflow (the examples of Sec. 4 that prescribe incoming
states); the dual mesh has n+1 cells as with outflow.  Workload: the
Shu-Osher problem of Sec. 4 on [-5, 5] with the post-shock state held on the
left.  Bar, per component: relative L-infinity error <= 1e-10 after the run,
equal step counts and final times.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import ora
from paper_2503_12473_amd import _lib, inputs
from paper_2503_12473_amd.api import OECDG, to_device
from paper_2503_12473_amd.inputs import Problem1D, BC_INFLOW, BC_OUTFLOW, FLUX_EULER
from tests.test_gpu_1d import RUN_TOL, _rel, gpu_run

pytestmark = pytest.mark.gpu

CFL = {1: 0.52, 2: 0.3, 3: 0.2}        # the paper's values for discontinuous data


@pytest.mark.parametrize("k", [1, 2, 3])
def test_shu_osher_run(k):
    """Shu-Osher, 200 cells (the paper's mesh), to t = 0.3."""
    prob, uC, uD = inputs.euler_shu_osher(200, k)
    gC, gD, t, n = gpu_run(prob, uC, uD, CFL[k], t_end=0.3)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.3, cfl=CFL[k])
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k", [1, 2, 3])
def test_shu_osher_ragged_and_modes(k):
    """N = 1030 (ragged last tile), 40 steps; eager, graph and persistent
    launches give identical bits."""
    prob, uC, uD = inputs.euler_shu_osher(1030, k)
    outs = [gpu_run(prob, uC, uD, CFL[k], mode=m, nsteps=40)
            for m in (_lib.MODE_EAGER, _lib.MODE_GRAPH, _lib.MODE_PERSISTENT)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=40, cfl=CFL[k])
    assert outs[0][3] == rn == 40
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


def test_inflow_equals_outflow_while_the_boundary_state_is_unchanged():
    """Ghost states equal to the initial end states: the inflow run is the
    outflow run until a wave reaches a boundary (Riemann data, 20 steps)."""
    states = (0.8, 0.9, 0.3, 0.2)
    po, uC, uD = inputs.euler_riemann(400, 2, states)
    left = tuple(map(float, inputs.euler_conserved(np.array(0.8), np.array(0.0), np.array(0.9))))
    right = tuple(map(float, inputs.euler_conserved(np.array(0.3), np.array(0.0), np.array(0.2))))
    pi = Problem1D(k=2, nc=3, flux=FLUX_EULER, bc=BC_INFLOW, n=400, xlo=0.0, xhi=1.0, inflow=(left, right))
    oC, oD, to, no = gpu_run(po, uC, uD, 0.15, nsteps=20)
    iC, iD, ti, ni = gpu_run(pi, uC, uD, 0.15, nsteps=20)
    assert (no, to) == (ni, ti)
    assert _rel(iC, iD, oC, oD) <= 1e-13


def test_batch_of_inflow_outflow_and_wall_instances():
    """A batch mixing inflow (Shu-Osher), outflow (Riemann) and reflective
    (blast waves) instances, each against its own oracle run."""
    specs = [inputs.euler_shu_osher(200, 2), inputs.euler_riemann(300, 2, inputs.riemann_states(3)),
             inputs.euler_blast_waves(400, 2, pressures=(100.0, 1.0, 10.0), densities=(1.0, 0.5, 0.8)),
             inputs.euler_shu_osher(130, 1)]
    probs = [s[0] for s in specs]
    with OECDG(probs, 0.2) as s:
        a = to_device(np.concatenate([x[1].ravel() for x in specs]))
        b = to_device(np.concatenate([x[2].ravel() for x in specs]))
        s.run(a, b, nsteps=25)
        A, B = a.cpu().numpy(), b.cpu().numpy()
        offC, offD = s.off_primal, s.off_dual
    for i, (p, uC, uD) in enumerate(specs):
        rC, rD, _, rn = ora.run1d(p, uC, uD, nsteps=25, cfl=0.2)
        gC = A[offC[i]:offC[i + 1]].reshape(uC.shape)
        gD = B[offD[i]:offD[i + 1]].reshape(uD.shape)
        assert _rel(gC, gD, rC, rD) <= RUN_TOL, i


def test_inflow_states_are_required_and_checked():
    prob, uC, uD = inputs.euler_shu_osher(64, 1)
    bare = Problem1D(k=1, nc=3, flux=FLUX_EULER, bc=BC_INFLOW, n=64, xlo=-5.0, xhi=5.0)
    with OECDG(bare, 0.3) as s:
        a, b = to_device(uC), to_device(uD)
        with pytest.raises(_lib.OECDGError) as e:
            s.run(a, b, nsteps=1)
        assert e.value.code == _lib.EINVAL
        L = _lib.lib()
        st = (C.c_double * 3)(1.0, 0.0, 2.5)
        assert L.oecdg_set_inflow(s._h, 1, st, st) == _lib.EINVAL        # instance out of range
        assert L.oecdg_set_inflow(s._h, 0, st, st) == _lib.OK
        s.run(a, b, nsteps=1)
    out = Problem1D(k=1, nc=3, flux=FLUX_EULER, bc=BC_OUTFLOW, n=64, xlo=-5.0, xhi=5.0)
    with OECDG(out, 0.3) as s:
        st = (C.c_double * 3)(1.0, 0.0, 2.5)
        assert _lib.lib().oecdg_set_inflow(s._h, 0, st, st) == _lib.EINVAL  # not an inflow instance
