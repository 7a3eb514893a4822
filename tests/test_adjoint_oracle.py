"""Pins of the discrete-adjoint oracle (CPU): its forward equals the C
oracle's, and its gradient matches central finite differences of the C
oracle's fixed-step run."""
import numpy as np
import pytest

from oracle import ora, adjoint_torch as adj
from paper_2503_12473_amd import inputs


def _setup(n=64, k=2, seed=0, steps=60):
    prob, uC, uD, _ = inputs.burgers_fourier(n, k, seed=seed)
    tau = 0.3 * prob.h / np.abs(uC[0, 0]).max()
    _, tC, tD, _ = inputs.burgers_fourier(n, k, seed=seed + 1)
    return prob, uC, uD, tC, tD, tau, steps


@pytest.mark.parametrize("k", [1, 2, 3])
def test_torch_forward_equals_c_oracle(k):
    prob, uC, uD, _, _, tau, steps = _setup(k=k)
    a, b = adj.forward(prob, uC, uD, steps, tau)
    rC, rD, _, _ = ora.run1d(prob, uC, uD, nsteps=steps, dt_fixed=tau)
    scale = max(np.abs(rC).max(), np.abs(rD).max())
    assert max(np.abs(a - rC).max(), np.abs(b - rD).max()) <= 1e-13 * scale


@pytest.mark.parametrize("k", [1, 2])
def test_gradient_matches_central_differences(k):
    """<dJ/du0, v> against (J(u0 + eps v) - J(u0 - eps v)) / (2 eps) of the C
    oracle, random directions on both meshes; best of three eps within 1e-6."""
    prob, uC, uD, tC, tD, tau, steps = _setup(k=k, steps=40)
    oC, oD, _, _ = ora.run1d(prob, uC, uD, nsteps=steps, dt_fixed=tau)
    _, gC, gD = adj.misfit_loss_grad(prob, oC, oD, tC, tD)
    dC, dD = adj.gradient(prob, uC, uD, steps, tau, gC, gD, checkpoint_every=8)
    rng = np.random.default_rng(7)
    for _ in range(3):
        vC = rng.normal(size=uC.shape) * (0.3 ** np.arange(k + 1))[None, :, None]
        vD = rng.normal(size=uD.shape) * (0.3 ** np.arange(k + 1))[None, :, None]
        exact = float((dC * vC).sum() + (dD * vD).sum())
        errs = []
        for eps in (1e-5, 1e-6, 1e-7, 1e-8):
            Jp = adj.misfit_loss_grad(prob, *ora.run1d(prob, uC + eps * vC, uD + eps * vD, nsteps=steps,
                                                        dt_fixed=tau)[:2], tC, tD)[0]
            Jm = adj.misfit_loss_grad(prob, *ora.run1d(prob, uC - eps * vC, uD - eps * vD, nsteps=steps,
                                                        dt_fixed=tau)[:2], tC, tD)[0]
            errs.append(abs((Jp - Jm) / (2 * eps) - exact) / abs(exact))
        assert min(errs) <= 1e-6, errs


def test_checkpointing_does_not_change_the_gradient():
    prob, uC, uD, tC, tD, tau, steps = _setup(n=48, steps=30)
    oC, oD, _, _ = ora.run1d(prob, uC, uD, nsteps=steps, dt_fixed=tau)
    _, gC, gD = adj.misfit_loss_grad(prob, oC, oD, tC, tD)
    a = adj.gradient(prob, uC, uD, steps, tau, gC, gD, checkpoint_every=0)
    b = adj.gradient(prob, uC, uD, steps, tau, gC, gD, checkpoint_every=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("flux", ["burgers", "advection"])
def test_tangent_linear_and_adjoint_are_transposes(flux):
    """Dot-product test: <J v, w> with J v from forward-mode differentiation of
    the run equals <v, J^T w> from the checkpointed reverse sweep, to 1e-12
    (exact transposition; only the summation order differs).  30 steps at
    n = 48 run well past the Burgers shock onset (about 4 steps here)."""
    import torch
    import torch.autograd.forward_ad as fwAD
    prob, uC, uD, _, _, tau, steps = _setup(n=48, k=2, steps=30)
    if flux == "advection":
        prob, uC, uD = inputs.advection_sine(48, 2, phase=1.3)
        tau = 0.2 * prob.h
    rng = np.random.default_rng(11)
    vC, vD, wC, wD = (rng.normal(size=uC.shape) for _ in range(4))
    s = adj.Scalar1D(prob)
    t = lambda x: torch.tensor(x[0], dtype=torch.float64)
    with fwAD.dual_level():
        oC, oD = s.run(fwAD.make_dual(t(uC), t(vC)), fwAD.make_dual(t(uD), t(vD)), steps, tau)
        tl = float((fwAD.unpack_dual(oC).tangent * t(wC)).sum() + (fwAD.unpack_dual(oD).tangent * t(wD)).sum())
    gC, gD = adj.gradient(prob, uC, uD, steps, tau, wC, wD, checkpoint_every=7)
    ad = float((gC * vC).sum() + (gD * vD).sum())
    assert abs(tl - ad) <= 1e-12 * max(abs(tl), abs(ad)), (tl, ad)


def test_plain_cdg_forward_and_gradient():
    """oe=False (plain CDG, the adjoint's mode without OE): the forward equals
    the C oracle's plain run and the gradient matches central differences."""
    prob, uC, uD, tC, tD, tau, steps = _setup(k=2, steps=25)
    s = adj.Scalar1D(prob)
    import torch
    with torch.no_grad():
        a, b = s.run(torch.tensor(uC[0]), torch.tensor(uD[0]), steps, tau, oe=False)
    rC, rD, _, _ = ora.run1d(prob, uC, uD, nsteps=steps, dt_fixed=tau, oe=False)
    scale = max(np.abs(rC).max(), np.abs(rD).max())
    assert max(np.abs(a.numpy() - rC[0]).max(), np.abs(b.numpy() - rD[0]).max()) <= 1e-13 * scale
    _, gC, gD = adj.misfit_loss_grad(prob, rC, rD, tC, tD)
    dC, dD = adj.gradient(prob, uC, uD, steps, tau, gC, gD, checkpoint_every=6, oe=False)
    rng = np.random.default_rng(8)
    vC, vD = rng.normal(size=uC.shape), rng.normal(size=uD.shape)
    exact = float((dC * vC).sum() + (dD * vD).sum())
    errs = []
    for eps in (1e-5, 1e-6, 1e-7):
        J = lambda sgn: adj.misfit_loss_grad(prob, *ora.run1d(prob, uC + sgn * eps * vC, uD + sgn * eps * vD,
                                                               nsteps=steps, dt_fixed=tau, oe=False)[:2], tC, tD)[0]
        errs.append(abs((J(1) - J(-1)) / (2 * eps) - exact) / abs(exact))
    assert min(errs) <= 1e-6, errs
