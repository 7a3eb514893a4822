"""GPU parity of the 1D HIP path against the CPU oracle (through the C ABI).

Floating-point bar, per component (tests/parity.py): relative L-infinity
error (max |gpu - oracle| over all coefficients of both meshes divided by
max |oracle| of that component) <= 1e-10 after a full run, <= 1e-12 for a
single stage; step counts and final times equal.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ora
from paper_2503_12473_amd import inputs
from paper_2503_12473_amd import _lib
from paper_2503_12473_amd.api import OECDG, to_device
from paper_2503_12473_amd.inputs import Problem1D, BC_OUTFLOW, BC_PERIODIC, FLUX_ADVECTION, FLUX_BURGERS, FLUX_EULER
from tests.parity import rel

pytestmark = pytest.mark.gpu

RUN_TOL = 1e-10
STAGE_TOL = 1e-12


def _rel(gC, gD, rC, rD):
    return rel(gC, gD, rC, rD)


def gpu_run(prob, uC, uD, cfl, mode=None, tile=None, oe=True, rk=3, **kw):
    print(f"[gpu_run] flux={prob.flux} k={prob.k} n={prob.n} bc={prob.bc} mode={mode} tile={tile} rk={rk} {kw}",
          flush=True)
    with OECDG(prob, cfl, oe=oe, rk=rk) as s:
        if mode is not None:
            s.set_option(_lib.OPT_MODE, mode)
        if tile is not None:
            s.set_option(_lib.OPT_TILE, tile)
        gC, gD = to_device(uC), to_device(uD)
        t, n = s.run(gC, gD, **kw)
        return gC.cpu().numpy().reshape(uC.shape), gD.cpu().numpy().reshape(uD.shape), t, n


def _state(prob, rng):
    """A physical random state (Euler: positive density and pressure)."""
    sC, sD = prob.shapes()
    decay = (0.3 ** np.arange(prob.k + 1))[None, :, None]
    uC = rng.normal(scale=0.1, size=sC) * decay
    uD = rng.normal(scale=0.1, size=sD) * decay
    if prob.flux == FLUX_EULER:
        for u in (uC, uD):
            u[0, 0] += 1.0
            u[2, 0] += 2.5
    else:
        uC[0, 0] += 0.5
        uD[0, 0] += 0.5
    return np.ascontiguousarray(uC), np.ascontiguousarray(uD)


CASES = [(FLUX_ADVECTION, BC_PERIODIC), (FLUX_BURGERS, BC_PERIODIC), (FLUX_EULER, BC_OUTFLOW), (FLUX_EULER, BC_PERIODIC),
         (FLUX_ADVECTION, BC_OUTFLOW)]


@pytest.mark.parametrize("flux,bc", CASES)
@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [37, 130])
def test_single_stage_parity(flux, bc, k, n):
    """oecdg_stage == one SSP-RK3 stage of eq:RKCDG followed by F_tau."""
    rng = np.random.default_rng(100 * k + n + 7 * flux)
    nc = 3 if flux == FLUX_EULER else 1
    prob = Problem1D(k=k, nc=nc, flux=flux, bc=bc, n=n, xlo=0.0, xhi=1.0, a=-1.3)
    unC, unD = _state(prob, rng)
    ulC, ulD = _state(prob, rng)
    tau = 0.1 * prob.h
    with OECDG(prob, 0.2) as s:
        gn = (to_device(unC), to_device(unD))
        gl = (to_device(ulC), to_device(ulD))
        for l in range(3):
            print(f"[stage] flux={flux} bc={bc} k={k} n={n} l={l}", flush=True)
            oC, oD = s.stage(l, tau, 1.3 * tau, gn[0], gn[1], gl[0], gl[1])
            rC, rD = ora.ssprk3_stage1d(prob, l, tau, 1.3 * tau, unC, unD, unC if l == 0 else ulC,
                                        unD if l == 0 else ulD)
            e = _rel(oC.cpu().numpy().reshape(rC.shape), oD.cpu().numpy().reshape(rD.shape), rC, rD)
            assert e <= STAGE_TOL, (l, e)


def _uniform_density_state(prob):
    """Euler data with density exactly 1 and momentum exactly 0 (every mode), the
    energy a smooth wave plus a jump: the first stage leaves the density exactly
    constant, so its sigma vanishes."""
    f = lambda x: inputs.euler_conserved(1.0 + 0 * x, 0 * x, 1.0 + 0.5 * np.sin(2 * np.pi * x) + 0.7 * (x > 0.3))
    uC, uD = inputs.project_1d(f, prob)
    for u in (uC, uD):
        u[0] = 0.0
        u[0, 0] = 1.0
        u[1] = 0.0
    return np.ascontiguousarray(uC), np.ascontiguousarray(uD)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("bc", [BC_OUTFLOW, BC_PERIODIC])
def test_zero_sigma_component_is_skipped(bc, k):
    """sigma_q = 0 (Sec. 2.2: delta_K^m is zero when the component equals its
    mean everywhere; with several components the max runs over the others).
    Euler, N = 300 (ragged tiles): the undamped output of the first stage has
    an exactly uniform density on both meshes in the oracle and in the library
    (whose coupling integrates the overlap exactly, so a constant with no flux
    has exactly zero rate), and the library must skip that component as the
    oracle does: a single stage and two full steps (the second step's first
    stage damps that output) against the oracle."""
    prob = Problem1D(k=k, nc=3, flux=FLUX_EULER, bc=bc, n=300, xlo=0.0, xhi=1.0)
    uC, uD = _uniform_density_state(prob)
    tau = 0.15 * prob.h / ora.max_wavespeed1d(prob, uC, uD)
    hC, hD = ora.ssprk3_stage1d(prob, 0, tau, tau, uC, uD, uC, uD, oe=False)
    _, sig = ora.stats1d(prob, hC, hD)
    assert sig[0, 0] == 0.0 and sig[1, 0] == 0.0 and np.all(sig[:, 1:] > 0.0)
    print(f"[sigma0] bc={bc} k={k} stage 0", flush=True)
    with OECDG(prob, 0.15) as s:
        g = (to_device(uC), to_device(uD))
        oC, oD = s.stage(0, tau, tau, g[0], g[1])
    rC, rD = ora.ssprk3_stage1d(prob, 0, tau, tau, uC, uD, uC, uD)
    assert _rel(oC.cpu().numpy(), oD.cpu().numpy(), rC, rD) <= STAGE_TOL
    gC, gD, t, n = gpu_run(prob, uC, uD, 0.15, nsteps=2)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=2, cfl=0.15)
    assert n == rn == 2 and t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("seed", range(5))
def test_advection_sine_full_run(seed):
    """Linear advection, [0, 2pi] periodic, N = 256, P2, CFL 0.2, T = 1,
    sin(x + phi) with seeded phi."""
    phi = float(inputs.advection_phases(seed)[0])
    prob, uC, uD = inputs.advection_sine(256, 2, phase=phi)
    gC, gD, t, n = gpu_run(prob, uC, uD, 0.2, t_end=1.0)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=1.0, cfl=0.2)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k", [1, 2, 3])
def test_advection_square_wave_full_run(k):
    prob, uC, uD = inputs.advection_square(256, k)
    gC, gD, t, n = gpu_run(prob, uC, uD, 0.2, t_end=1.0)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=1.0, cfl=0.2)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("n", [1000, 2053])
def test_euler_riemann_run(k, n):
    """1D Euler Riemann workload states (seed 0), outflow, CFL 0.15, to T = 0.01."""
    prob, uC, uD = inputs.euler_riemann(n, k, inputs.riemann_states(0))
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.15, t_end=0.01)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.01, cfl=0.15)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("k", [1, 2, 3])
def test_euler_riemann_full_size_steps(k):
    """Full workload size N = 16384 for 12 steps (all tiles, ragged dual tail)."""
    prob, uC, uD = inputs.euler_riemann(16384, k, inputs.riemann_states(1))
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.15, nsteps=12)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=12, cfl=0.15)
    assert ns == rn == 12
    assert t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_burgers_fixed_step_full_size():
    """Burgers, [0, 2pi] periodic, N = 16384, P2, seeded Fourier modes, fixed
    tau = 0.3 h / max|u0|, 10 steps."""
    prob, uC, uD, _ = inputs.burgers_fourier(16384, 2, seed=0)
    dt = 0.3 * prob.h / np.abs(uC[0, 0]).max()
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.3, nsteps=10, dt_fixed=dt)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=10, dt_fixed=dt)
    assert ns == rn == 10
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_burgers_to_shock():
    """Burgers P2 N = 256 through shock formation (t = 2.2, sin x + 0.5)."""
    prob, uC, uD = inputs.burgers_sine(256, 2)
    gC, gD, t, ns = gpu_run(prob, uC, uD, 0.3, t_end=2.2)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=2.2, cfl=0.3)
    assert (ns, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


def test_plain_cdg_without_oe():
    prob, uC, uD = inputs.advection_square(256, 2)
    gC, gD, t, n = gpu_run(prob, uC, uD, 0.2, oe=False, t_end=0.5)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.5, cfl=0.2, oe=False)
    assert (n, t) == (rn, rt)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL


@pytest.mark.parametrize("tile", [32, 64, 128])
def test_execution_modes_bitwise_identical(tile):
    """Eager launches, the captured graph and the persistent cooperative
    launch run the same tiles with the same reduction order: identical bits."""
    prob, uC, uD = inputs.euler_riemann(3000, 2, inputs.riemann_states(2))
    outs = [gpu_run(prob, uC, uD, 0.15, mode=m, tile=tile, t_end=0.004)
            for m in (_lib.MODE_EAGER, _lib.MODE_GRAPH, _lib.MODE_PERSISTENT)]
    for o in outs[1:]:
        assert o[2] == outs[0][2] and o[3] == outs[0][3]
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, t_end=0.004, cfl=0.15)
    assert outs[0][3] == rn
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


@pytest.mark.parametrize("nsteps", [1, 30, 256])
def test_short_run_graph_matches_eager_bitwise(nsteps):
    """Runs of at most 256 steps replay one captured graph whose first stage
    reads the caller's arrays in place (no copy of the initial data); eager
    launches copy them first.  Same bits, same steps and time, and the
    oracle's result; the graph is replayed on the same arrays a second time."""
    prob, uC, uD = inputs.euler_riemann(2500, 2, inputs.riemann_states(6))
    ref = gpu_run(prob, uC, uD, 0.15, mode=_lib.MODE_EAGER, nsteps=nsteps)
    with OECDG(prob, 0.15) as s:
        gC, gD = to_device(uC), to_device(uD)
        for rep in range(2):
            gC.copy_(to_device(uC))
            gD.copy_(to_device(uD))
            t, n = s.run(gC, gD, nsteps=nsteps)
            oC, oD = gC.cpu().numpy().reshape(uC.shape), gD.cpu().numpy().reshape(uD.shape)
            assert (t, n) == (ref[2], ref[3]) and n == nsteps
            assert np.array_equal(oC, ref[0]) and np.array_equal(oD, ref[1]), rep
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=nsteps, cfl=0.15)
    assert rn == nsteps and _rel(ref[0], ref[1], rC, rD) <= RUN_TOL


@pytest.mark.parametrize("mode", [_lib.MODE_EAGER, _lib.MODE_GRAPH])
def test_zero_steps_leave_the_state_unchanged(mode):
    """nsteps = 0: no stage runs, so no OE is applied either (the initial data
    are u_sigma^0); the arrays come back bitwise, at t = 0 and no steps."""
    prob, uC, uD = inputs.euler_riemann(700, 3, inputs.riemann_states(8))
    oC, oD, t, n = gpu_run(prob, uC, uD, 0.15, mode=mode, nsteps=0, t_end=0.1)
    assert (t, n) == (0.0, 0)
    assert np.array_equal(oC, uC) and np.array_equal(oD, uD)


def test_repeat_runs_are_deterministic():
    prob, uC, uD = inputs.euler_riemann(4096, 3, inputs.riemann_states(3))
    a = gpu_run(prob, uC, uD, 0.15, nsteps=40)
    b = gpu_run(prob, uC, uD, 0.15, nsteps=40)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_dt_matches_oracle():
    prob, uC, uD = inputs.euler_riemann(777, 2, inputs.riemann_states(4))
    with OECDG(prob, 0.15) as s:
        dt = s.dt(to_device(uC), to_device(uD))
    ref = 0.15 * prob.h / ora.max_wavespeed1d(prob, uC, uD)
    assert dt == pytest.approx(ref, rel=1e-14)


def test_batched_instances_match_their_own_runs():
    """Several independent instances of uneven N and k advanced together:
    each matches the oracle run of that instance alone (each with its own
    CFL time step), for a fixed number of steps."""
    specs = inputs.batch_instances(seed=5, count=6, nmin=100, nmax=700)
    probs, states = [], []
    for n, k, st in specs:
        p, uC, uD = inputs.euler_riemann(n, k, st)
        probs.append(p)
        states.append((uC, uD))
    with OECDG(probs, 0.15) as s:
        gC = torch.cat([to_device(u[0]) for u in states])
        gD = torch.cat([to_device(u[1]) for u in states])
        print("[batched] 6 instances, 25 steps", flush=True)
        s.run(gC, gD, nsteps=25)
        offC, offD = s.off_primal, s.off_dual
        gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    for b, (p, (uC, uD)) in enumerate(zip(probs, states)):
        rC, rD, _, rn = ora.run1d(p, uC, uD, nsteps=25, cfl=0.15)
        bC = gC[offC[b]:offC[b + 1]].reshape(rC.shape)
        bD = gD[offD[b]:offD[b + 1]].reshape(rD.shape)
        assert _rel(bC, bD, rC, rD) <= RUN_TOL, b


def test_nonphysical_state_is_reported():
    prob, uC, uD = inputs.euler_riemann(64, 1, (1.0, 1.0, 0.5, 0.5))
    uC = uC.copy()
    uC[2, 0, 10] = -1.0
    with pytest.raises(_lib.OECDGError) as e:
        gpu_run(prob, uC, uD, 0.15, nsteps=2)
    assert e.value.code == _lib.ENONPHYSICAL


def test_many_handles_create_and_destroy():
    """Handles release what they own: creating, running and destroying many
    (1D single, 1D batch, 2D, with graph capture and the adjoint's second
    stream) leaves device memory where it was and every call succeeds."""
    import gc
    prob1, uC1, uD1 = inputs.euler_riemann(20000, 2, inputs.riemann_states(0))   # ~10 MB of handle memory
    prob2, uC2, uD2, _ = inputs.euler2d_quadrants(64, 2, seed=0)
    probb, uCb, uDb, _ = inputs.burgers_fourier(64, 2, seed=0)
    tau = 0.3 * probb.h / np.abs(uCb[0, 0]).max()

    def cycle():
        with OECDG(prob1, 0.15) as s:
            s.run(to_device(uC1), to_device(uD1), nsteps=70)          # graph capture (64-step chunks)
        with OECDG([prob1, prob1], 0.15) as s:
            s.run(torch.cat([to_device(uC1)] * 2), torch.cat([to_device(uD1)] * 2), nsteps=5)
        with OECDG(prob2, 0.3) as s:
            s.run(to_device(uC2), to_device(uD2), nsteps=3)
        with OECDG(probb, 0.3) as s:
            s.adjoint(to_device(uCb), to_device(uDb), 9, tau, to_device(uCb), to_device(uDb), 4)

    cycle()
    torch.cuda.synchronize()
    gc.collect()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        cycle()
    torch.cuda.synchronize()
    gc.collect()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < 16 << 20, (free0, free1)          # a leak would be >= 200 MB here


def test_nonfinite_input_is_reported():
    """A NaN in a higher mode of one cell (the wave speeds, from averages, stay
    finite): the run stops with ENONFINITE instead of returning NaNs."""
    prob, uC, uD = inputs.euler_riemann(64, 2, (1.0, 1.0, 0.5, 0.5))
    uC = uC.copy()
    uC[1, 2, 20] = float("nan")
    with pytest.raises(_lib.OECDGError) as e:
        gpu_run(prob, uC, uD, 0.15, nsteps=3)
    assert e.value.code == _lib.ENONFINITE


def test_adjoint_rejects_what_it_does_not_cover():
    """oecdg_adjoint: scalar flux on a periodic mesh, one instance, valid
    arguments; anything else is refused before any work."""
    rng = np.random.default_rng(0)
    prob, uC, uD, _ = inputs.burgers_fourier(64, 2, seed=0)
    g = (to_device(rng.normal(size=uC.shape)), to_device(rng.normal(size=uD.shape)))
    with OECDG(prob, 0.3) as s:
        for nsteps, dt, ck in ((-1, 0.01, 4), (5, 0.0, 4), (5, 0.01, 0)):
            with pytest.raises(_lib.OECDGError) as e:
                s.adjoint(to_device(uC), to_device(uD), nsteps, dt, g[0], g[1], ck)
            assert e.value.code == _lib.EINVAL
    pe, eC, eD = inputs.euler_riemann(64, 2, (1.0, 1.0, 0.5, 0.5))
    with OECDG(pe, 0.15) as s:
        with pytest.raises(_lib.OECDGError) as e:
            s.adjoint(to_device(eC), to_device(eD), 3, 0.001, to_device(eC), to_device(eD), 2)
        assert e.value.code == _lib.EUNSUPPORTED
    with OECDG([prob, prob], 0.3) as s:
        two = (torch.cat([to_device(uC)] * 2), torch.cat([to_device(uD)] * 2))
        with pytest.raises(_lib.OECDGError) as e:
            s.adjoint(two[0], two[1], 3, 0.01, two[0], two[1], 2)
        assert e.value.code == _lib.EUNSUPPORTED


def test_execution_modes_bitwise_identical_with_tail_tile():
    """N = 16384 outflow with tiles of 64: dual cell 16384 is carried by the
    last tile's extra wave (256 workgroups instead of 257).  Eager, graph and
    persistent launches give the same bits; the run matches the oracle."""
    prob, uC, uD = inputs.euler_riemann(16384, 2, inputs.riemann_states(4))
    outs = [gpu_run(prob, uC, uD, 0.15, mode=m, tile=64, nsteps=30)
            for m in (_lib.MODE_EAGER, _lib.MODE_GRAPH, _lib.MODE_PERSISTENT)]
    for o in outs[1:]:
        assert o[2] == outs[0][2] and o[3] == outs[0][3]
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    rC, rD, _, rn = ora.run1d(prob, uC, uD, nsteps=30, cfl=0.15)
    assert outs[0][3] == rn == 30
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


def test_tail_tile_gives_the_bits_of_the_separate_tile():
    """N = 8192 outflow with tiles of 32: run alone, dual cell 8192 rides on the
    last tile's extra wave (256 workgroups); in a batch it has a tile of its
    own.  Its statistics keep their own column either way: identical bits."""
    prob, uC, uD = inputs.euler_riemann(8192, 2, inputs.riemann_states(3))
    other, oC, oD = inputs.euler_riemann(300, 1, inputs.riemann_states(1))
    solo = gpu_run(prob, uC, uD, 0.15, tile=32, nsteps=40)
    with OECDG([prob, other], 0.15) as s:
        s.set_option(_lib.OPT_TILE, 32)
        gC = torch.cat([to_device(uC), to_device(oC)])
        gD = torch.cat([to_device(uD), to_device(oD)])
        print("[tail] batch of 2, 40 steps", flush=True)
        s.run(gC, gD, nsteps=40)
        offC, offD = s.off_primal, s.off_dual
        bC = gC.cpu().numpy()[offC[0]:offC[1]].reshape(uC.shape)
        bD = gD.cpu().numpy()[offD[0]:offD[1]].reshape(uD.shape)
    assert np.array_equal(solo[0], bC) and np.array_equal(solo[1], bD)


def test_single_stage_and_dt_with_tail_tile():
    """N = 16384 outflow (tail tile): oecdg_dt reads the wave speeds of all
    partial columns, oecdg_stage computes every SSP-RK3 stage, against the oracle."""
    prob, uC, uD = inputs.euler_riemann(16384, 2, inputs.riemann_states(2))
    rng = np.random.default_rng(11)
    lC = uC * (1.0 + 0.01 * rng.standard_normal(uC.shape))
    lD = uD * (1.0 + 0.01 * rng.standard_normal(uD.shape))
    with OECDG(prob, 0.15) as s:
        dt = s.dt(to_device(uC), to_device(uD))
        assert dt == pytest.approx(0.15 * prob.h / ora.max_wavespeed1d(prob, uC, uD), rel=1e-14)
        tau = 0.9 * dt
        for l in range(3):
            print(f"[tail stage] l={l}", flush=True)
            ulC, ulD = (uC, uD) if l == 0 else (lC, lD)
            o = s.stage(l, tau, dt, to_device(uC), to_device(uD), to_device(ulC), to_device(ulD))
            rC, rD = ora.ssprk3_stage1d(prob, l, tau, dt, uC, uD, ulC, ulD)
            gC, gD = o[0].cpu().numpy().reshape(rC.shape), o[1].cpu().numpy().reshape(rD.shape)
            assert _rel(gC, gD, rC, rD) <= STAGE_TOL, l


@pytest.mark.parametrize("n,k", [(16384, 2), (1000, 3), (130, 1)])
def test_statistics_fold_modes_give_the_same_bits(n, k):
    """The global statistics reduced inside every stage workgroup (1) or by a
    separate per-instance kernel (2) follow one fixed order: identical results,
    eager and graph launches (N = 16384 uses the extra-wave tail tiles, where
    mode 2 reduces in-kernel)."""
    prob, uC, uD = inputs.euler_riemann(n, k, inputs.riemann_states(2))
    outs = []
    for fold in (1, 2):
        for mode in (_lib.MODE_EAGER, _lib.MODE_GRAPH):
            print(f"[fold] n={n} k={k} fold={fold} mode={mode}", flush=True)
            with OECDG(prob, 0.15) as s:
                s.set_option(_lib.OPT_FOLD, fold)
                s.set_option(_lib.OPT_MODE, mode)
                a, b = to_device(uC), to_device(uD)
                t, ns = s.run(a, b, nsteps=300)
                outs.append((a.cpu().numpy(), b.cpu().numpy(), t, ns))
    for o in outs[1:]:
        assert o[2:] == outs[0][2:]
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=40, cfl=0.15) if n <= 1000 else (None, None, None, None)
    if rC is not None:
        with OECDG(prob, 0.15) as s:
            s.set_option(_lib.OPT_FOLD, 2)
            a, b = to_device(uC), to_device(uD)
            s.run(a, b, nsteps=40)
            assert _rel(a.cpu().numpy(), b.cpu().numpy(), rC, rD) <= RUN_TOL


def test_large_mesh_folds_its_statistics():
    """N = 80000 (1251 tiles of 64): the library folds the statistics with the
    per-instance kernel (more than 1024 tiles) and gives the bits of the
    in-kernel reduction, and the oracle's result to the run bar."""
    prob, uC, uD = inputs.euler_riemann(80000, 2, inputs.riemann_states(4))
    outs = []
    for fold in (0, 1):
        print(f"[large] n=80000 fold={fold}", flush=True)
        with OECDG(prob, 0.15) as s:
            if fold:
                s.set_option(_lib.OPT_FOLD, fold)
            a, b = to_device(uC), to_device(uD)
            t, ns = s.run(a, b, nsteps=8)
            outs.append((a.cpu().numpy(), b.cpu().numpy(), t, ns))
    assert outs[0][2:] == outs[1][2:]
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=8, cfl=0.15)
    # tau comes from the largest wave speed at a cell average, which both sides
    # evaluate on states that agree to rounding: the time agrees to rounding
    assert outs[0][3] == rn and abs(outs[0][2] - rt) <= 1e-12 * rt
    assert _rel(outs[0][0], outs[0][1], rC, rD) <= RUN_TOL


@pytest.mark.parametrize("ntiles", range(9, 17))
def test_every_tile_count_mod_8(ntiles):
    """Workgroups are mapped to tiles in one band of consecutive tiles per XCD
    (8 bands, the first n mod 8 of them one tile longer): tile counts 9..16
    cover every residue mod 8.  Euler, outflow, P2, N = 64 ntiles - 5 (the last
    tile ragged on both meshes), 4 steps against the oracle."""
    prob, uC, uD = inputs.euler_riemann(64 * ntiles - 5, 2, inputs.riemann_states(ntiles))
    gC, gD, t, n = gpu_run(prob, uC, uD, 0.15, tile=64, nsteps=4)
    rC, rD, rt, rn = ora.run1d(prob, uC, uD, nsteps=4, cfl=0.15)
    assert n == rn == 4 and t == pytest.approx(rt, rel=1e-14)
    assert _rel(gC, gD, rC, rD) <= RUN_TOL
