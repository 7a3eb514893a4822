"""Build and run the oracle's operation counter (test infrastructure).

The oracle's C sources are compiled as C++ with `double` replaced by a type
that counts every + - * / and library call (ora_real.hpp); the drivers run one
operator evaluation, one OE step and one SSP-RK3 step (three stages, OE after
each) of 1D Euler P2 (256 cells, outflow) and 2D Euler Q2 (32^2, periodic) on
smooth data, and report operations per DOF of both meshes.  A step's count per
DOF is the operation count per DOF-update of the oracle's plain evaluation of
the method.

    python oracle/opcount/run.py [OUT.json]
"""
import json
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def counts():
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in ("count_1d.cpp", "count_2d.cpp", "main.cpp"):
            obj = os.path.join(d, src + ".o")
            subprocess.run(["g++", "-O1", "-std=c++17", "-fpermissive", "-w", "-c", os.path.join(HERE, src), "-o", obj],
                           check=True)
            objs.append(obj)
        exe = os.path.join(d, "opcount")
        subprocess.run(["g++", "-o", exe] + objs, check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {r["phase"]: r for r in (json.loads(line) for line in out.splitlines() if line.strip())}


if __name__ == "__main__":
    res = counts()
    text = json.dumps(res, indent=1)
    if len(sys.argv) > 1:
        open(sys.argv[1], "w").write(text + "\n")
    print(text)
