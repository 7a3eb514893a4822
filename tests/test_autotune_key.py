"""The autotuner's cache key separates batches that run different kernels or
stage sequences (host logic only)."""
from paper_2503_12473_amd import autotune, inputs


def test_key_separates_rk_methods_walls_and_degrees():
    out = [inputs.euler_riemann(300, 2, inputs.riemann_states(0))[0]] * 4
    walls = [inputs.euler_blast_waves(300, 2)[0]] * 4
    mixed = [inputs.euler_riemann(300, k, inputs.riemann_states(0))[0] for k in (1, 2, 3, 2)]
    keys = {autotune._key(out), autotune._key(out, 4), autotune._key(walls), autotune._key(mixed)}
    assert len(keys) == 4
    assert autotune._key(out) == autotune._key(out, 3)
