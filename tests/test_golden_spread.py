"""The rounding floor of the full-horizon Riemann parity bar (CPU only).

tests/golden/make_riemann_spread.py runs the 1D Euler Riemann workload of the
headline benchmark (N = 16384, P_k, CFL 0.15, to T = 0.2, ~33k steps) through
test-only builds of the oracle that round differently but equally validly
(oracle/build.py VARIANTS: FMA contraction; the domain mean summed pairwise;
both with the damping exponential in long double) and stores the same cells as
the plain oracle's golden file.  Their distance to that file is how far
last-bit differences grow over the run; the GPU parity bar at this horizon
(tests/test_gpu_golden.py, 1e-10 per component) rests on it.  Every variant
takes the same steps to the same final time, and stays within the bar."""
import os

import numpy as np
import pytest

from tests.parity import rel_per_component

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BAR = 1e-10


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_riemann_spread.py, about an hour of CPU)")
    return np.load(path)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("variant", ["fma", "pairwise", "mixed"])
def test_oracle_rounding_spread_at_full_horizon(k, variant):
    g = _load(f"riemann_seed0_N16384_k{k}_T0.2.npz")
    x = _load(f"riemann_seed0_N16384_k{k}_T0.2_{variant}.npz")
    assert int(x["steps"]) == int(g["steps"]) and float(x["t"]) == float(g["t"])
    assert int(x["stride"]) == int(g["stride"])
    per = rel_per_component(x["uC"], x["uD"], g["uC"], g["uD"])
    print(f"k={k} {variant}: per-component spread {per}")
    assert per.max() > 0.0          # a different rounding indeed (not the same build)
    assert per.max() <= BAR
