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
