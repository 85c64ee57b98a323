"""Two-stage (adaptive-resolution) projection -- TEST INFRASTRUCTURE (oracle).

Section 4, "Calculation of the acceleration": the density is projected
exactly onto an adaptive grid whose cells are no larger than the smallest
height of the simplices they meet, and the adaptive grid is then gathered
onto the uniform grid by donor cell (each coarse cell's mass spread evenly
over the fine cells it covers).  Reading used here (per simplex rather than
per region): a simplex whose smallest height is h fine cells is projected
exactly onto the grid coarsened by 2^l along every axis, l = floor(log2 h)
clamped to [0, max_level]; the coarse grids are then donor-cell gathered
onto the fine grid and summed.  Heights are measured in fine-cell units
after the minimum-image unwrap, in FP64: the smallest height of a
tetrahedron is 3 V / (largest face area).

Plain numpy on top of the FP64 projection oracle, one step per line of the
definition.
"""
from __future__ import annotations

import math

import numpy as np

from . import project as _project


def smallest_heights(prob) -> np.ndarray:
    """Smallest height of every tetrahedron, in fine-cell units."""
    X = np.asarray(prob["xyz"], dtype=np.float64)
    S = np.asarray(prob["simplices"], dtype=np.int64)
    dims = np.asarray(prob["dims"], dtype=np.float64)[:3]
    ext = np.asarray(prob["extent"], dtype=np.float64)[:3]
    P = X[S]                                    # [n][4][3]
    E = P[:, 1:, :] - P[:, :1, :]               # edges from corner 0
    for d in range(3):
        if prob["periodic"][d]:
            E[:, :, d] -= ext[d] * np.rint(E[:, :, d] / ext[d])
    E = E * (dims / ext)                        # cell units
    V = np.abs(np.einsum("ni,ni->n", E[:, 0], np.cross(E[:, 1], E[:, 2]))) / 6.0
    # faces: (0,1,2), (0,1,3), (0,2,3) from corner 0, and (1,2,3)
    a = [np.linalg.norm(np.cross(E[:, 0], E[:, 1]), axis=1),
         np.linalg.norm(np.cross(E[:, 0], E[:, 2]), axis=1),
         np.linalg.norm(np.cross(E[:, 1], E[:, 2]), axis=1),
         np.linalg.norm(np.cross(E[:, 1] - E[:, 0], E[:, 2] - E[:, 0]), axis=1)]
    amax = np.max(np.stack(a, axis=1), axis=1) / 2.0
    h = np.zeros_like(V)
    ok = amax > 0
    h[ok] = 3.0 * V[ok] / amax[ok]
    return h


def levels(prob, max_level: int) -> np.ndarray:
    h = smallest_heights(prob)
    lv = np.zeros(h.shape[0], dtype=np.int64)
    pos = h >= 1.0
    lv[pos] = np.floor(np.log2(h[pos])).astype(np.int64)
    return np.clip(lv, 0, max_level)


def donor_cell(coarse: np.ndarray, level: int) -> np.ndarray:
    """Spread each coarse cell's mass evenly over its 2^(3 level) fine cells."""
    f = 2 ** level
    fine = coarse
    for axis in range(coarse.ndim):
        fine = np.repeat(fine, f, axis=axis)
    return fine / float(f ** coarse.ndim)


def project(prob, max_level: int) -> dict:
    """Masses [dims2][dims1][dims0] of the two-stage projection, and the
    level of every simplex."""
    lv = levels(prob, max_level)
    dims = np.asarray(prob["dims"], dtype=np.int64)
    total = np.zeros(tuple(int(d) for d in dims[::-1]))
    for l in range(max_level + 1):
        sel = np.nonzero(lv == l)[0]
        if sel.size == 0:
            continue
        sub = dict(prob, simplices=np.ascontiguousarray(np.asarray(prob["simplices"])[sel]),
                   dims=dims // (2 ** l))
        if prob["rho_per_corner"]:
            sub["rho"] = np.ascontiguousarray(np.asarray(prob["rho"])[sel])
        coarse = _project(sub, coverage=False)["mass"]
        total += donor_cell(coarse, l)
    return dict(mass=total, levels=lv)
