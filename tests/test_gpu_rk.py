"""GPU parity of the RK methods besides SSP-RK3 against the oracle.

eq:RKCDG with the c/d tables of forward Euler, SSP-RK2 (Heun) and classical
fourth-order RK, the OE step after every stage; Sec. 4 pairs P^k with an RK
method of order k+1 for its accuracy tests (CFL 0.45, 0.33, 0.31 for P1, P2,
P3).  Bar: relative L-infinity error <= 1e-10 after the run, equal step
counts and final times (as for SSP-RK3).
"""
import numpy as np
import pytest
import torch

from oracle import ora
from paper_2503_12473_amd import _lib, inputs
from paper_2503_12473_amd.api import OECDG, to_device
from tests.test_gpu_1d import RUN_TOL, _rel, gpu_run

pytestmark = pytest.mark.gpu

# (rk, k, CFL): order k+1 pairs of the accuracy tests, plus RK4 and SSP-RK2 at P2
PAIRS = [(1, 0, 0.45), (2, 1, 0.45), (4, 3, 0.31), (4, 2, 0.33), (2, 2, 0.2)]


@pytest.mark.parametrize("rk,k,cfl", PAIRS)
@pytest.mark.parametrize("n", [1000, 2053])
def test_euler_riemann_run(rk, k, cfl, n):
    """1D Euler Riemann workload states (seed 0), outflow, to T = 0.01."""
    prob, uC, uD = inputs.euler_riemann(n, k, inputs.riemann_states(0))
    gC, gD, t, ns = gpu_run(prob, uC, uD, cfl, rk=rk, t_end=0.01)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.01, cfl=cfl, rk=rk)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("rk,k,cfl", [(2, 1, 0.45), (4, 3, 0.31), (4, 2, 0.33)])
def test_advection_sine_full_run(rk, k, cfl):
    """Linear advection, [0, 2pi] periodic, N = 128, sin(x + phi), T = 1."""
    phi = float(inputs.advection_phases(0)[0])
    prob, uC, uD = inputs.advection_sine(128, k, phase=phi)
    gC, gD, t, n = gpu_run(prob, uC, uD, cfl, rk=rk, t_end=1.0)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=1.0, cfl=cfl, rk=rk)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("rk", [1, 2, 4])
def test_burgers_to_shock(rk):
    """Burgers N = 256 through shock formation (t = 2.2, sin x + 0.5); the OE
    step is active in every stage."""
    k = {1: 0, 2: 1, 4: 3}[rk]
    cfl = {1: 0.45, 2: 0.45, 4: 0.31}[rk]
    prob, uC, uD = inputs.burgers_sine(256, k)
    gC, gD, t, ns = gpu_run(prob, uC, uD, cfl, rk=rk, t_end=2.2)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=2.2, cfl=cfl, rk=rk)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("rk,k", [(2, 1), (4, 3)])
def test_euler_riemann_full_size_steps(rk, k):
    """N = 16384 (all tiles, ragged dual tail) for 12 steps."""
    prob, uC, uD = inputs.euler_riemann(16384, k, inputs.riemann_states(1))
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.15, rk=rk, nsteps=12)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=12, cfl=0.15, rk=rk)
    assert ns == rn == 12
    assert t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("rk", [1, 2, 4])
def test_execution_modes_bitwise_identical(rk):
    """Eager launches, the captured graph (its stage parities depend on the
    number of stages per step) and the persistent launch: identical bits."""
    k = {1: 0, 2: 1, 4: 2}[rk]
    prob, uC, uD = inputs.euler_riemann(3000, k, inputs.riemann_states(2))
    outs = [gpu_run(prob, uC, uD, 0.15, mode=m, tile=64, rk=rk, t_end=0.004)
            for m in (_lib.MODE_EAGER, _lib.MODE_GRAPH, _lib.MODE_PERSISTENT)]
    assert outs[0][3] > 70                    # more steps than one captured graph holds
    for o in outs[1:]:
        assert o[2] == outs[0][2] and o[3] == outs[0][3]
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.004, cfl=0.15, rk=rk)
    assert outs[0][3] == rn
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


@pytest.mark.parametrize("rk", [2, 4])
def test_batched_instances_match_their_own_runs(rk):
    """Instances of uneven N and mixed k in one handle with classical RK4 or
    SSP-RK2: each matches the oracle run of that instance alone."""
    specs = inputs.batch_instances(seed=7, count=5, nmin=100, nmax=700)
    probs, states = [], []
    for n, k, st in specs:
        p, uC, uD = inputs.euler_riemann(n, k, st)
        probs.append(p)
        states.append((uC, uD))
    print(f"[batched rk={rk}] 5 instances, k = {[p.k for p in probs]}, 25 steps", flush=True)
    with OECDG(probs, 0.15, rk=rk) as s:
        gC = torch.cat([to_device(u[0]) for u in states])
        gD = torch.cat([to_device(u[1]) for u in states])
        s.run(gC, gD, nsteps=25)
        offC, offD = s.off_primal, s.off_dual
        gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    for b, (p, (uC, uD)) in enumerate(zip(probs, states)):
        rC, rD, _, rn = ora.run1d(p, uC, uD, nsteps=25, cfl=0.15, rk=rk)
        bC = gC[offC[b]:offC[b + 1]].reshape(rC.shape)
        bD = gD[offD[b]:offD[b + 1]].reshape(rD.shape)
        assert _rel(bC, bD, rC, rD) <= RUN_TOL, b


@pytest.mark.parametrize("rk", [1, 2, 3, 4])
def test_single_stage_follows_the_rk_method(rk):
    """oecdg_stage computes stage l of the handle's method (1e-12 against the
    oracle's single stage); the last stage of classical RK4 is refused, and a
    stage index past the method's stages is invalid."""
    prob, uC, uD = inputs.euler_riemann(130, 2, inputs.riemann_states(0))
    rng = np.random.default_rng(rk)
    lC = uC * (1.0 + 0.01 * rng.standard_normal(uC.shape))
    lD = uD * (1.0 + 0.01 * rng.standard_normal(uD.shape))
    tau = 0.1 * prob.h
    s = {1: 1, 2: 2, 3: 3, 4: 4}[rk]
    with OECDG(prob, 0.15, rk=rk) as h:
        for l in range(s):
            print(f"[stage] rk={rk} l={l}", flush=True)
            if rk == 4 and l == 3:
                with pytest.raises(_lib.OECDGError) as e:
                    h.stage(l, tau, 1.3 * tau, to_device(uC), to_device(uD), to_device(lC), to_device(lD))
                assert e.value.code == _lib.EUNSUPPORTED
                continue
            ulC, ulD = (uC, uD) if l == 0 else (lC, lD)
            o = h.stage(l, tau, 1.3 * tau, to_device(uC), to_device(uD), to_device(ulC), to_device(ulD))
            rC, rD = ora.rk_stage1d(prob, rk, l, tau, 1.3 * tau, uC, uD, ulC, ulD)
            gC, gD = o[0].cpu().numpy().reshape(rC.shape), o[1].cpu().numpy().reshape(rD.shape)
            assert _rel(gC, gD, rC, rD) <= 1e-12, l
        with pytest.raises(_lib.OECDGError) as e:
            h.stage(s, tau, 1.3 * tau, to_device(uC), to_device(uD), to_device(lC), to_device(lD))
        assert e.value.code == _lib.EINVAL


def test_adjoint_refuses_other_rk_methods():
    prob, uC, uD, _ = inputs.burgers_fourier(64, 2, seed=0)
    with OECDG(prob, 0.3, rk=4) as s:
        with pytest.raises(_lib.OECDGError) as e:
            s.adjoint(to_device(uC), to_device(uD), 3, 0.01, to_device(uC), to_device(uD), 2)
        assert e.value.code == _lib.EUNSUPPORTED
