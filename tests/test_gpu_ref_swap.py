"""The same sequences of C-interface calls on the HIP library (oecdg_*, device
arrays) and on the oracle's mirror (oecdg_ref_*, host arrays), compared: runs
(single instance, a mixed batch, inflow, 2D in both spaces, a non-uniform
mesh), single stages in 1D and 2D, the allocation-free run, and oecdg_dt.
Bars as in the other parity tests: 1e-10 relative per component after a run
(equal step counts and times), 1e-12 for a single stage."""
import numpy as np
import pytest

from paper_2503_12473_amd import inputs
from tests import abi_swap

pytestmark = pytest.mark.gpu


def _comp_err(a, b):
    """Largest relative difference per component (first axis)."""
    a, b = np.asarray(a), np.asarray(b)
    return max(float(np.abs(a[q] - b[q]).max() / max(np.abs(b[q]).max(), 1e-300)) for q in range(a.shape[0]))


def _both(fn, *args, **kw):
    print(f"[ref-swap] {fn.__name__} {kw}", flush=True)
    return fn(abi_swap.Impl("hip"), *args, **kw), fn(abi_swap.Impl("ref"), *args, **kw)


def _check_run(g, r, bar=1e-10):
    assert g["steps"] == r["steps"]
    assert g["t"] == pytest.approx(r["t"], rel=1e-13)
    assert g["dt"] == pytest.approx(r["dt"], rel=1e-13)
    assert g["offP"] == r["offP"] and g["offD"] == r["offD"]
    for (gC, gD), (rC, rD) in zip(g["out"], r["out"]):
        assert _comp_err(gC, rC) <= bar and _comp_err(gD, rD) <= bar


def test_single_instance_run():
    prob, uC, uD = inputs.euler_riemann(256, 2, inputs.riemann_states(3))
    g, r = _both(abi_swap.run, [prob], [(uC, uD)], 0.15, t_end=0.04)
    assert r["steps"] > 20
    _check_run(g, r)


def test_batch_runs():
    """Batches of one flux: Euler with mixed degrees, sizes and boundaries
    (outflow, inflow, walls), and Burgers with mixed degrees; both
    implementations refuse a batch of two fluxes."""
    euler = [inputs.euler_riemann(64, 2, inputs.riemann_states(4)), inputs.euler_shu_osher(90, 3),
             inputs.euler_blast_waves(70, 1, pressures=(100.0, 1.0, 10.0)), inputs.euler_riemann(33, 1, inputs.riemann_states(7))]
    burgers = [inputs.burgers_fourier(100, 1, 3)[:3], inputs.burgers_fourier(61, 3, 4)[:3], inputs.burgers_sine(40, 2)]
    for cases in (euler, burgers):
        probs = [c[0] for c in cases]
        states = [(c[1], c[2]) for c in cases]
        g, r = _both(abi_swap.run, probs, states, 0.2, nsteps=40)
        _check_run(g, r)
    mixed = abi_swap._descs([euler[0][0], burgers[0][0]], 0.2, True, 3)
    for kind in ("hip", "ref"):
        impl = abi_swap.Impl(kind)
        h = abi_swap.C.c_void_p()
        assert impl.f("init")(mixed, 2, None, abi_swap.C.byref(h)) == -6


@pytest.mark.parametrize("space", [0, 1])
def test_2d_run(space):
    prob, uC, uD = inputs.advection2d_sine(12, 2, space=space)
    g, r = _both(abi_swap.run, [prob], [(uC, uD)], 0.3, nsteps=6)
    _check_run(g, r)


def test_2d_euler_run():
    prob, uC, uD, _ = inputs.euler2d_quadrants(16, 1, 0)
    g, r = _both(abi_swap.run, [prob], [(uC, uD)], 0.3, nsteps=4)
    _check_run(g, r)


def test_nonuniform_run():
    edges = inputs.quasi_uniform_edges(300, 0.0, 1.0, seed=2)
    prob, uC, uD = inputs.advection_sine_edges(edges, 2)
    g, r = _both(abi_swap.run, [prob], [(uC, uD)], 0.3, nsteps=30, edges=edges)
    _check_run(g, r)


@pytest.mark.parametrize("dim", [1, 2])
def test_single_stage(dim):
    if dim == 1:
        prob, uC, uD = inputs.euler_riemann(200, 2, inputs.riemann_states(5))
    else:
        prob, uC, uD = inputs.advection2d_sine(10, 2)
    ul = (uC * 1.001, uD * 0.999)
    for l in range(3):
        g, r = _both(abi_swap.stage, prob, 0.2, 3, l, 1e-3, 2e-3, (uC, uD), ul)
        assert _comp_err(g[0], r[0]) <= 1e-12 and _comp_err(g[1], r[1]) <= 1e-12


def test_noalloc_run():
    prob, uC, uD = inputs.euler_riemann(128, 1, inputs.riemann_states(6))
    (g, gt, gn), (r, rt, rn) = _both(abi_swap.run_noalloc, prob, 0.2, (uC, uD), nsteps=25)
    assert gn == rn == 25 and gt == pytest.approx(rt, rel=1e-13)
    assert _comp_err(g[0], r[0]) <= 1e-10 and _comp_err(g[1], r[1]) <= 1e-10
