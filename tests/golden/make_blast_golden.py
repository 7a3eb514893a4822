"""Write the oracle's result for the paper's two-blast-wave example.

1D Euler, gamma = 1.4, [0, 1] between reflective walls, rho = 1, v = 0 and
p = 1000 (x < 0.1), 0.01 (0.1 < x < 0.9), 100 (x > 0.9); P2, 960 cells,
CFL 0.3, SSP-RK3 + OE to t = 0.038 (Sec. 4, the two-blast-wave example).  A
cell average next to the weaker blast carries a small non-positive pressure
for a few hundred steps, which the problem tolerates (the wave speed takes
|p|).  Calls only the CPU oracle (a few minutes); stores every 4th cell of
both meshes plus the final time and step count, and the full primal cell
averages of the density.

    python tests/golden/make_blast_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ora  # noqa: E402
from paper_2503_12473_amd import inputs  # noqa: E402

N, K, CFL, T, STRIDE = 960, 2, 0.3, 0.038, 4


def main():
    prob, uC, uD = inputs.euler_blast_waves(N, K)
    t0 = time.time()
    oC, oD, t, steps = ora.run1d(prob, uC, uD, t_end=T, cfl=CFL)
    wall = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"blast_waves_N{N}_k{K}_T{T:g}.npz")
    np.savez_compressed(out, uC=oC[:, :, ::STRIDE], uD=oD[:, :, ::STRIDE], rho=oC[0, 0], t=t, steps=steps,
                        stride=STRIDE, n=N, k=K, cfl=CFL, oracle_seconds=wall)
    print(out, steps, t, wall)


if __name__ == "__main__":
    main()
