"""Adaptive-grid projection with a donor-cell gather -- TEST INFRASTRUCTURE
(oracle).

Section 4, "Calculation of the acceleration": an adaptive (octree) grid is
refined, region by region, as long as its cells are larger than the smallest
perpendicular height of any simplex intersecting them, or until the finest
level (the uniform Poisson grid) is reached; the density is projected exactly
onto that adaptive grid, which is then gathered onto the uniform grid by donor
cell.  Written out here step by step:

1. levels: the smallest height h_i of every tetrahedron (3 V / largest face
   area, in cells of the uniform grid, after the minimum-image unwrap, FP64)
   gives l_i = floor(log2 h_i) clamped to [0, max_level] (0 when h_i < 1): a
   cell of side 2^l is no larger than h_i exactly when l <= l_i;
2. marks: a block of side 2^(l_i + 1) that tetrahedron i intersects (with a
   positive volume) is too large for it; every such block is marked, tested
   against every block of that size in i's bounding box by the separating
   axis test below (a block of any larger side that i intersects contains
   one of them);
3. refinement, top down: a block of side 2^l (l >= 1) is refined when it, or
   one of the smaller blocks inside it, is marked; the leaf holding a cell of
   the uniform grid is the largest block around it that is not refined, of
   level lev(c) (at most max_level, at least 0);
4. exact projection onto the adaptive grid: the mass of a leaf is the
   integral of the density over it, the sum of the exact projection onto the
   uniform grid over the leaf's cells (projection is additive over cells);
5. donor cell: every cell of the uniform grid receives its leaf's mass spread
   evenly, mass(leaf) / 8^lev.

Intersection (step 2) is taken between interiors, so a tetrahedron that only
touches a block along its boundary does not refine it.  Two convex polytopes
have disjoint interiors exactly when some plane separates them weakly; for a
tetrahedron and a box the candidate normals are the three axes, the four face
normals of the tetrahedron and the cross products of its six edges with the
three axes.  The normals come from FP64 differences of the corners, the
projections from FP64 corners relative to the block's lower corner, summed in
the order written, so that another implementation taking the same FP64 steps
reaches the same decisions.

Plain numpy on top of the FP64 projection oracle; no blocking or reordering
beyond what the definition states.
"""
from __future__ import annotations

import numpy as np

from . import project as _project


def _unwrapped_cells(prob) -> np.ndarray:
    """Corner positions [n][4][3] in cells of the uniform grid: each simplex
    unwrapped to the minimum image of its first corner on periodic axes
    (box units, FP64), then (x - origin) * dims / extent."""
    X = np.asarray(prob["xyz"], dtype=np.float64)
    S = np.asarray(prob["simplices"], dtype=np.int64)
    dims = np.asarray(prob["dims"], dtype=np.float64)[:3]
    ext = np.asarray(prob["extent"], dtype=np.float64)[:3]
    org = np.asarray(prob["origin"], dtype=np.float64)[:3]
    P = X[S].copy()                             # [n][4][3]
    for d in range(3):
        if prob["periodic"][d]:
            P[:, :, d] = P[:, :, d] - ext[d] * np.rint((P[:, :, d] - P[:, :1, d]) / ext[d])
    return (P - org) * (dims / ext)


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
    """Step 1: the largest level whose cells are no larger than the simplex's
    smallest height."""
    h = smallest_heights(prob)
    lv = np.zeros(h.shape[0], dtype=np.int64)
    pos = h >= 1.0
    lv[pos] = np.floor(np.log2(h[pos])).astype(np.int64)
    return np.clip(lv, 0, max_level)


def _axes(P: np.ndarray) -> np.ndarray:
    """The 25 candidate separating axes of a tetrahedron (corners [4][3], cell
    units) and an axis-aligned box: the three axes, the four face normals
    (cross products of two edges from a face's first corner) and each of the
    six edges crossed with each axis.  Differences of the corners in FP64."""
    axes = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]
    for (i, j, k) in ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)):
        e1 = P[j] - P[i]
        e2 = P[k] - P[i]
        axes.append([e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]])
    for (i, j) in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        e = P[j] - P[i]
        axes.append([0.0, e[2], -e[1]])   # e x (1, 0, 0)
        axes.append([-e[2], 0.0, e[0]])   # e x (0, 1, 0)
        axes.append([e[1], -e[0], 0.0])   # e x (0, 0, 1)
    return np.array(axes, dtype=np.float64)


def meets(P: np.ndarray, lo: np.ndarray, size: float) -> np.ndarray:
    """For each box lo[m] + [0, size]^3 (lo [m][3], cell units): do its
    interior and the tetrahedron's (corners P [4][3]) intersect?  Separating
    axis test, strict: on every candidate axis with a non-zero normal the
    open intervals of the two projections must overlap.  Projections of the
    corners relative to the box's lower corner, summed x + y, then + z."""
    n = _axes(P)                                        # [25][3]
    rel = P[None, :, :] - lo[:, None, :]                # [m][4][3]
    t = (n[None, :, None, 0] * rel[:, None, :, 0] + n[None, :, None, 1] * rel[:, None, :, 1]) \
        + n[None, :, None, 2] * rel[:, None, :, 2]      # [m][25][4]
    tmin, tmax = t.min(axis=2), t.max(axis=2)
    ns = n * size
    bmin = (np.minimum(0.0, ns[:, 0]) + np.minimum(0.0, ns[:, 1])) + np.minimum(0.0, ns[:, 2])
    bmax = (np.maximum(0.0, ns[:, 0]) + np.maximum(0.0, ns[:, 1])) + np.maximum(0.0, ns[:, 2])
    overlap = (tmin < bmax[None, :]) & (bmin[None, :] < tmax)
    zero = np.all(n == 0.0, axis=1)
    return np.all(overlap | zero[None, :], axis=1)


def marks(prob, max_level: int, lv=None):
    """Step 2: for each level l in 1..max_level, a boolean grid over the
    blocks of side 2^l, True where a tetrahedron of level l - 1 intersects
    the block."""
    if lv is None:
        lv = levels(prob, max_level)
    dims = [int(d) for d in prob["dims"][:3]]
    P = _unwrapped_cells(prob)
    out = {l: np.zeros(tuple(d >> l for d in reversed(dims)), dtype=bool) for l in range(1, max_level + 1)}
    for i in np.nonzero(lv < max_level)[0]:
        l = int(lv[i]) + 1
        size = float(1 << l)
        nb = [d >> l for d in dims]
        blo = [int(np.floor(P[i, :, d].min() / size)) for d in range(3)]
        bhi = [int(np.floor(P[i, :, d].max() / size)) for d in range(3)]
        bz, by, bx = np.meshgrid(*[np.arange(blo[d], bhi[d] + 1) for d in (2, 1, 0)], indexing="ij")
        B = np.stack([bx.ravel(), by.ravel(), bz.ravel()], axis=1)          # block indices [m][3]
        keep = np.ones(B.shape[0], dtype=bool)
        W = B.copy()
        for d in range(3):
            if prob["periodic"][d]:
                W[:, d] = np.mod(B[:, d], nb[d])
            else:
                keep &= (B[:, d] >= 0) & (B[:, d] < nb[d])
        hit = keep & meets(P[i], B.astype(np.float64) * size, size)
        out[l][W[hit, 2], W[hit, 1], W[hit, 0]] = True
    return out


def _expand(r: np.ndarray, l: int) -> np.ndarray:
    """A grid over blocks of side 2^l repeated onto the uniform grid."""
    for axis in range(3):
        r = np.repeat(r, 1 << l, axis=axis)
    return r


def leaf_levels(prob, max_level: int, mk=None) -> np.ndarray:
    """Step 3: the leaf level of every cell of the uniform grid, shape
    [dims2][dims1][dims0]."""
    if mk is None:
        mk = marks(prob, max_level)
    dims = [int(d) for d in prob["dims"][:3]]
    # refined[l]: a block of side 2^l is refined (it or a smaller block
    # inside it is marked); blocks of side 1 are never refined
    refined = {0: np.zeros(tuple(reversed(dims)), dtype=bool)}
    for l in range(1, max_level + 1):
        child = refined[l - 1]
        nz, ny, nx = child.shape
        up = child.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).any(axis=(1, 3, 5))
        refined[l] = mk[l] | up
    # top down: start from the largest blocks, descend while refined
    lev = np.full(tuple(reversed(dims)), max_level, dtype=np.int64)
    descending = _expand(refined[max_level], max_level)
    for l in range(max_level - 1, -1, -1):
        lev = np.where(descending, l, lev)
        descending = descending & _expand(refined[l], l)
    return lev


def donor_cell(coarse: np.ndarray, level: int) -> np.ndarray:
    """Spread each coarse cell's mass evenly over its 2^(3 level) fine cells."""
    f = 2 ** level
    fine = coarse
    for axis in range(coarse.ndim):
        fine = np.repeat(fine, f, axis=axis)
    return fine / float(f ** coarse.ndim)


def block_sums(fine: np.ndarray, level: int) -> np.ndarray:
    """Sum of a fine grid over the blocks of side 2^level."""
    f = 1 << level
    nz, ny, nx = fine.shape
    return fine.reshape(nz // f, f, ny // f, f, nx // f, f).sum(axis=(1, 3, 5))


def project(prob, max_level: int) -> dict:
    """Masses [dims2][dims1][dims0] of the adaptive-grid projection gathered
    onto the uniform grid (steps 1-5), with the simplex levels, the block
    marks and the leaf level of every cell."""
    lv = levels(prob, max_level)
    mk = marks(prob, max_level, lv)
    lev = leaf_levels(prob, max_level, mk)
    fine = _project(prob, coverage=False)["mass"]
    out = np.where(lev == 0, fine, 0.0)
    for l in range(1, max_level + 1):
        spread = donor_cell(block_sums(fine, l), l)
        out = np.where(lev == l, spread, out)
    return dict(mass=out, levels=lv, marks=mk, leaf=lev)
