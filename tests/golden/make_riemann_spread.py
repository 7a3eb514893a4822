"""Write the full-horizon result of a test-only oracle build variant for the
1D Euler Riemann workload (the same workload and stored cells as
make_riemann_golden.py).

The variants (oracle/build.py VARIANTS) evaluate the same scheme with other,
equally valid FP64 rounding: FMA contraction, the domain mean summed in
pairwise order, or both with the damping exponential taken in long double.  Their distance to the plain oracle's stored result on the same
cells measures how far last-bit differences grow over the ~33k steps of the
run, which is what the full-horizon parity bar of the HIP path rests on.
Calls only the CPU oracle; about an hour of serial CPU per degree for T = 0.2.

    python tests/golden/make_riemann_spread.py VARIANT K [T]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ora  # noqa: E402
from paper_2503_12473_amd import inputs  # noqa: E402

N, CFL, SEED, STRIDE = 16384, 0.15, 0, 8


def main(variant: str, k: int, T: float = 0.2):
    ora.use_variant(variant)
    states = inputs.riemann_states(SEED)
    prob, uC, uD = inputs.euler_riemann(N, k, states)
    t0 = time.time()
    oC, oD, t, steps = ora.run1d(prob, uC, uD, t_end=T, cfl=CFL)
    wall = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"riemann_seed{SEED}_N{N}_k{k}_T{T:g}_{variant}.npz")
    np.savez_compressed(out, uC=oC[:, :, ::STRIDE], uD=oD[:, :, ::STRIDE], t=t, steps=steps, stride=STRIDE,
                        n=N, k=k, cfl=CFL, seed=SEED, variant=variant, oracle_seconds=wall)
    print(out, steps, t, wall)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), float(sys.argv[3]) if len(sys.argv) > 3 else 0.2)
