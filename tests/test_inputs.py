"""Input generators: the factorised projection of the 2D quadrant data equals
the generic point-value projection (same Gauss rule, different summation)."""
import numpy as np
import pytest

from paper_2503_12473_amd import inputs


@pytest.mark.parametrize("n", [8, 12])
def test_quadrant_projection_fast_equals_generic(n):
    _, a, b, qa = inputs.euler2d_quadrants(n, 2, seed=5, fast=True)
    _, c, d, qc = inputs.euler2d_quadrants(n, 2, seed=5, fast=False)
    assert np.array_equal(qa, qc)
    assert np.abs(a - c).max() <= 1e-13 and np.abs(b - d).max() <= 1e-13


def test_quadrant_states_follow_the_seeded_draw():
    _, _, _, q = inputs.euler2d_quadrants(4, 2, seed=0)
    rng = np.random.default_rng(0)
    for row in q:
        rq, pq = rng.uniform(0.2, 1.0, size=2)
        uq, vq = rng.uniform(-0.5, 0.5, size=2)
        assert np.array_equal(row, [rq, pq, uq, vq])


def test_nonuniform_mesh_generators():
    e = inputs.quasi_uniform_edges(500, -1.0, 2.0, 1.5, seed=3)
    w = np.diff(e)
    assert e[0] == -1.0 and e[-1] == 2.0 and np.all(w > 0)
    assert w.max() / w.min() <= 1.5 + 1e-12
    assert np.array_equal(e, inputs.quasi_uniform_edges(500, -1.0, 2.0, 1.5, seed=3))
    g = inputs.smooth_graded_edges(64, 0.0, 1.0, 0.3)
    wg = np.diff(g)
    assert g[0] == 0.0 and g[-1] == 1.0 and np.all(wg > 0)
    assert wg.max() <= 1.3 / 64 + 1e-12 and wg.min() >= 0.7 / 64 - 1e-12


def test_project_1d_edges_reproduces_polynomials():
    """A polynomial of degree <= k is reproduced exactly on every primal and
    dual cell (dual cell j = [x_{j-1}, x_j], dual 0 reaching below xlo)."""
    from numpy.polynomial import legendre as L
    k = 3
    e = inputs.quasi_uniform_edges(9, 0.0, 1.0, 1.5, seed=1)
    p = np.polynomial.Polynomial([0.2, -0.7, 1.1, 0.4])
    uC, uD = inputs.project_1d_edges(lambda x: p(x)[None], 1, k, e)
    c = 0.5 * (e[:-1] + e[1:])
    cm1 = np.concatenate([[c[-1] - 1.0], c[:-1]])
    for lo, hi, u in ((e[:-1], e[1:], uC), (cm1, c, uD)):
        for i in range(len(lo)):
            xi = np.linspace(-1, 1, 7)
            x = 0.5 * (lo[i] + hi[i]) + 0.5 * (hi[i] - lo[i]) * xi
            np.testing.assert_allclose(L.legval(xi, u[0, :, i]), p(x), rtol=0, atol=1e-13)
