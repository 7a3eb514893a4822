"""Tile-size autotuner for the 1D stage kernels.

A workgroup owns T primal + T dual cells, one thread per cell, plus one wave
for the cells next to the tile.  Small tiles give more workgroups (good for
small meshes and latency), large tiles fewer partial statistics to reduce and a
smaller share of neighbour cells (good for large meshes).  The tuner times
a few RK steps of the real batch for each candidate T on scratch copies of
the state and keeps the fastest; results are cached per batch shape (flux,
degrees, mesh-size bucket, batch-size bucket, GPU architecture), in memory and
optionally in a JSON file named by $OECDG_AUTOTUNE_CACHE.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import _lib

CANDIDATES = (32, 64, 128)
_memory: dict = {}


def _key(probs, rk: int = 3) -> str:
    ns = [p.n for p in probs]
    ks = sorted({p.k for p in probs})
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "none"
    nb = int(round(math.log2(max(1.0, sum(ns) / len(ns)))))
    bb = int(round(math.log2(len(probs))))
    walls = "|walls" if any(getattr(p, "bc", 0) == 2 for p in probs) else ""
    return f"{arch}|flux{probs[0].flux}{walls}|rk{rk}|k{''.join(map(str, ks))}|n2^{nb}|b2^{bb}"


def _load_file():
    path = os.environ.get("OECDG_AUTOTUNE_CACHE")
    if path and os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            return {}
    return {}


def _store_file(cache):
    path = os.environ.get("OECDG_AUTOTUNE_CACHE")
    if path:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)


def tune_tile(solver, uC: torch.Tensor, uD: torch.Tensor, steps: int = 12, candidates=CANDIDATES,
              t_end: float = math.inf) -> int:
    """Pick the fastest tile size for `solver` (an api.OECDG handle) on this
    state, set it on the handle and return it.  The state is not modified."""
    key = _key(solver.probs, getattr(solver, "rk", 3))
    cache = _memory or _load_file()
    _memory.update(cache)
    if key in _memory:
        solver.set_option(_lib.OPT_TILE, _memory[key]["tile"])
        return _memory[key]["tile"]
    stream = solver.stream
    best, timings = None, {}
    for tile in candidates:
        solver.set_option(_lib.OPT_TILE, tile)
        a, b = uC.clone(), uD.clone()
        solver.run(a, b, t_end=t_end, nsteps=steps)          # warm-up: code load, graph capture
        a.copy_(uC)
        b.copy_(uD)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.run(a, b, t_end=t_end, nsteps=steps)
        e1.record(stream)
        torch.cuda.synchronize()
        timings[tile] = e0.elapsed_time(e1)
        if best is None or timings[tile] < timings[best]:
            best = tile
    solver.set_option(_lib.OPT_TILE, best)
    _memory[key] = {"tile": best, "ms": timings}
    _store_file(_memory)
    return best
