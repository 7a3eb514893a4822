"""Write the oracle's result for 2D linear advection in the P^k space.

u_t + u_x + u_y = 0 on [0, 1]^2 periodic, u0 = sin^2(pi (x + y)), P^2
(total degree), SSP-RK3 with OE, CFL 0.33, to t = 1.1: the setting of Table
2Dlinear_accuracy (Sec. 4).  Calls only the CPU oracle; stores every 4th cell
in each direction of both meshes, the l1 / l2 / l-infinity errors of the
primal solution against the exact one (8 x 8 Gauss points per cell, area
weighted), the final time and the step count.  About 40 minutes of serial CPU
at N = 128.

    python tests/golden/make_pk_advection_golden.py [N]
"""
import os
import sys
import time

import numpy as np
from numpy.polynomial import legendre as npleg

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ora  # noqa: E402
from paper_2503_12473_amd import inputs  # noqa: E402

K, CFL, T, STRIDE = 2, 0.33, 1.1, 4


def error_norms(prob, u, t):
    """l1, l2, l-infinity of the primal polynomial minus sin^2(pi (x + y - 2t))."""
    s, w = npleg.leggauss(8)
    P = np.stack([npleg.legval(s, [0.0] * m + [1.0]) for m in range(prob.k + 1)])
    vals = np.einsum("abyx,ag,bh->yxgh", u[0], P, P)
    xc = prob.xlo + (np.arange(prob.nx) + 0.5) * prob.hx
    yc = prob.ylo + (np.arange(prob.ny) + 0.5) * prob.hy
    X = xc[None, :, None, None] + 0.5 * prob.hx * s[None, None, :, None]
    Y = yc[:, None, None, None] + 0.5 * prob.hy * s[None, None, None, :]
    e = vals - np.sin(np.pi * (X + Y - 2.0 * t)) ** 2
    W = w[:, None] * w[None, :] / 4.0
    cells = prob.nx * prob.ny
    return (np.abs(e) * W).sum() / cells, np.sqrt((e ** 2 * W).sum() / cells), np.abs(e).max()


def main(n: int = 128):
    prob, uC, uD = inputs.advection2d_sine(n, K, space=1)
    t0 = time.time()
    oC, oD, t, steps = ora.run2d(prob, uC, uD, t_end=T, cfl=CFL, rk=3)
    wall = time.time() - t0
    l1, l2, linf = error_norms(prob, oC, t)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"advection2d_p{K}_N{n}_T{T:g}.npz")
    np.savez_compressed(out, uC=oC[..., ::STRIDE, ::STRIDE], uD=oD[..., ::STRIDE, ::STRIDE], t=t, steps=steps,
                        stride=STRIDE, n=n, k=K, cfl=CFL, l1=l1, l2=l2, linf=linf, oracle_seconds=wall)
    print(out, steps, t, wall, l1, l2, linf)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 128)
