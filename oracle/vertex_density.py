"""Per-vertex density estimate -- TEST INFRASTRUCTURE (oracle).

Section 4, "Calculation of the acceleration": the density at vertex j is
the total mass of the simplices incident to j divided by their total
volume (area in 2D),

    rho_j = sum_{i incident to j} M_i / sum_{i incident to j} |V_i|.

Volumes are unsigned (a shell-crossed, inverted simplex still covers its
region) and measured after unwrapping each simplex's corners to the minimum
image of its first corner on periodic axes.  Plain FP64 numpy, one step per
line of the definition.  Vertices with no incident volume get 0.
"""
from __future__ import annotations

import math

import numpy as np


def vertex_density(xyz, simplices, mass, extent=(1.0, 1.0, 1.0), periodic=(True, True, True)) -> np.ndarray:
    """xyz [n_vert][D], simplices [n_simplex][D+1], mass [n_simplex] (or a
    scalar for equal masses).  Returns rho [n_vert] (float64)."""
    X = np.asarray(xyz, dtype=np.float64)
    S = np.asarray(simplices, dtype=np.int64)
    n_vert, D = X.shape
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (S.shape[0],))
    corners = X[S]                                  # [n][D+1][D]
    edges = corners[:, 1:, :] - corners[:, :1, :]   # corner a minus corner 0
    for d in range(D):
        if periodic[d]:
            L = float(extent[d])
            edges[:, :, d] -= L * np.rint(edges[:, :, d] / L)
    vol = np.abs(np.linalg.det(edges)) / math.factorial(D)
    num = np.zeros(n_vert)
    den = np.zeros(n_vert)
    for a in range(D + 1):
        np.add.at(num, S[:, a], m)
        np.add.at(den, S[:, a], vol)
    out = np.zeros(n_vert)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out
