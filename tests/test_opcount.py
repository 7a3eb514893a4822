"""The oracle's operation counter (oracle/opcount): it builds, and its counts
are consistent with the structure of an SSP-RK3 step (CPU only)."""
import shutil

import pytest

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def test_step_counts_are_three_stages():
    from oracle.opcount.run import counts
    c = counts()
    for dim in ("1d_euler_p2", "2d_euler_q2"):
        op, oe, step = (c[f"{dim}.{x}"]["flops_per_dof"] for x in ("operator", "oe", "step"))
        assert op > 0 and oe > 0
        # a step is three operator evaluations, three OE steps and the RK combinations
        assert 3 * (op + oe) < step < 3 * (op + oe) + 40
        assert c[f"{dim}.step"]["exp"] == pytest.approx(3 * c[f"{dim}.oe"]["exp"], abs=2e-3)
