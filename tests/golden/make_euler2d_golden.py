"""Write the 2D oracle's results for the 2D Euler quadrant workload.

2D Euler, gamma = 1.4, [0,1]^2 periodic, tensor Q2, seeded quadrant states
(seed 0) plus 0.2 sin(2 pi (x+y)) in the density, CFL 0.3, SSP-RK3 + OE.
Calls only the CPU oracle; stores every `stride`-th cell in each direction of
both meshes (all components and modes) plus the final time and step count.

    python tests/golden/make_euler2d_golden.py N STEPS STRIDE [SPACE]
(the committed files: 128 500 4 and 1024 3 32, about an hour of serial CPU
each; with SPACE = 1 the total-degree space P^2: 128 200 4)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ora  # noqa: E402
from paper_2503_12473_amd import inputs  # noqa: E402

SEED, CFL = 0, 0.3


def main(n: int, steps: int, stride: int, space: int = 0):
    prob, uC, uD, _ = inputs.euler2d_quadrants(n, 2, seed=SEED, space=space)
    t0 = time.time()
    oC, oD, t, done = ora.run2d(prob, uC, uD, nsteps=steps, cfl=CFL)
    wall = time.time() - t0
    tag = "_p2" if space == 1 else ""
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"euler2d{tag}_seed{SEED}_N{n}_{steps}steps.npz")
    np.savez_compressed(out, uC=oC[..., ::stride, ::stride], uD=oD[..., ::stride, ::stride], t=t, steps=done,
                        stride=stride, n=n, cfl=CFL, seed=SEED, oracle_seconds=wall)
    print(out, done, t, wall)


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]) if len(sys.argv) > 4 else 0)
