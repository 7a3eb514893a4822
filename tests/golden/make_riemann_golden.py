"""Write the oracle's full-horizon result for the 1D Euler Riemann workload.

1D Euler, gamma = 1.4, [0, 1], outflow, N = 16384 primal cells, seeded states
(seed 0), CFL 0.15, run to T (default 0.2) with SSP-RK3 + OE.  Calls only the
CPU oracle; stores every 8th cell of both meshes (all components and modes)
plus the final time and step count.  About an hour of serial CPU per degree
for T = 0.2 (the cost is proportional to T).

    python tests/golden/make_riemann_golden.py K [T]
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


def main(k: int, T: float = 0.2):
    states = inputs.riemann_states(SEED)
    prob, uC, uD = inputs.euler_riemann(N, k, states)
    t0 = time.time()
    oC, oD, t, steps = ora.run1d(prob, uC, uD, t_end=T, cfl=CFL)
    wall = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"riemann_seed{SEED}_N{N}_k{k}_T{T:g}.npz")
    np.savez_compressed(out, uC=oC[:, :, ::STRIDE], uD=oD[:, :, ::STRIDE], t=t, steps=steps, stride=STRIDE,
                        n=N, k=k, cfl=CFL, seed=SEED, oracle_seconds=wall)
    print(out, steps, t, wall)


if __name__ == "__main__":
    main(int(sys.argv[1]), float(sys.argv[2]) if len(sys.argv) > 2 else 0.2)
