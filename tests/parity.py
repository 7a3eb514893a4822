"""Parity measure of the GPU path against the oracle.

The bar is applied per component: for component q, max |gpu - oracle| over
both meshes, every mode and every cell, divided by max |oracle| over the same
entries of that component.  For the Euler systems this keeps the momentum (and
the small higher modes it carries) to the same relative bar as the energy,
whose magnitude would otherwise set the scale for all components.  Arrays are
in the modal layouts of the library (component first); device-shaped flat
arrays are reshaped to the oracle's shapes.
"""
import math

import numpy as np


def rel_per_component(gC, gD, rC, rD):
    rC, rD = np.asarray(rC), np.asarray(rD)
    gC = np.asarray(gC).reshape(rC.shape)
    gD = np.asarray(gD).reshape(rD.shape)
    out = []
    for q in range(rC.shape[0]):
        num = max(np.abs(gC[q] - rC[q]).max(), np.abs(gD[q] - rD[q]).max())
        den = max(np.abs(rC[q]).max(), np.abs(rD[q]).max())
        out.append(num / den if den > 0 else (0.0 if num == 0 else math.inf))
    return np.array(out)


def rel(gC, gD, rC, rD):
    """Largest per-component relative L-infinity error."""
    return float(rel_per_component(gC, gD, rC, rD).max())
