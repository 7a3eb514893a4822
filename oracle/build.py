"""Build the C oracle library with the host compiler (plain FP64, no contraction).

Three test-only variants evaluate the same oracle with different, equally valid
FP64 rounding, to measure how far last-bit differences grow over a long run:
"fma" lets the compiler contract a*b+c into fused multiply-adds, "pairwise"
sums the cell averages of the domain mean in pairwise order, "mixed" does both
and evaluates the damping exponential in long double before rounding it.  The
product never loads any of these libraries.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oecdg_oracle.c", "oecdg_oracle_2d.c", "oecdg_oracle_nu.c", "oecdg_ref.c"]
LIB = os.path.join(HERE, "liboecdg_oracle.so")
VARIANTS = {
    "fma": ["-ffp-contract=fast", "-mfma"],
    "pairwise": ["-ffp-contract=off", "-DORA_PAIRWISE_MEAN"],
    "mixed": ["-ffp-contract=fast", "-mfma", "-DORA_PAIRWISE_MEAN", "-DORA_EXP_LONG_DOUBLE"],
}


def lib_path(variant: str | None = None) -> str:
    return LIB if variant is None else os.path.join(HERE, f"liboecdg_oracle_{variant}.so")


def build(verbose: bool = False, variant: str | None = None) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    out = lib_path(variant)
    tmp = out + ".tmp"
    fp = ["-ffp-contract=off"] if variant is None else VARIANTS[variant]
    cmd = ["gcc", "-O2"] + fp + ["-fno-fast-math", "-fPIC", "-shared", "-std=c11",
                                 "-D_DEFAULT_SOURCE", "-Wall", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
