"""Work counts of the exact projection's slab recursion -- TEST
INFRASTRUCTURE (oracle).

The projection of a simplex onto the grid (Section 3, eq. eq_firstOrder)
cuts it into its pieces S cap G_j and integrates each (Appendix C: cones
from an apex over the facets, each facet fanned into triangles).  Its
arithmetic is counted here on a plain CPU model of the recursion the pieces
come from, with the simplex's axes ordered by cell span (smallest first):

    remainder --cut at the next plane of axis 0--> slab + remainder
    slab      --cut at the next plane of axis 1--> column + rest of the slab
    column    --cut at the next plane of axis 2--> piece + rest of the column

every cut made once (the last slab, column and piece need none).  Three
quantities are counted:

* classifications N_cls: one per polytope vertex per cut (which side of the
  plane it lies on);
* intersection points N_int: one per edge a cut crosses (a new vertex, shared
  by both sides);
* fan tetrahedra N_fan: per piece, its facets not containing the apex, each
  fanned into (vertices - 2) triangles; the apex is a vertex of the cut that
  closes the piece from above (its first new vertex), else of the cut below
  it, else the simplex's first corner, so that the facets through it add
  nothing.

Priced as 10 flops per intersection point (a division and four fused
multiply-adds: three coordinates and the density), 2 per classification and
20 per fan tetrahedron (a determinant and a mean of four densities).

Polytopes are vertex lists with their facets as vertex loops, counter-
clockwise seen from outside; a cut splits every facet it crosses and closes
each side with a cap loop built from the split facets' new edges.  A vertex
on the plane counts as above it (the half-open cells of Section 3.3).  FP64
throughout; plain Python, for samples of a few thousand simplices.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

FLOPS_INT, FLOPS_CLS, FLOPS_FAN = 10, 2, 20


class Poly:
    """A convex polytope: points (list of [x, y, z]) and facets (lists of
    point indices, counter-clockwise seen from outside)."""

    def __init__(self, pts, faces):
        self.pts = pts
        self.faces = faces

    def used(self):
        s = set()
        for f in self.faces:
            s.update(f)
        return sorted(s)


def tet(P) -> Poly:
    """A tetrahedron with corners P [4][3]; oriented so its facets face out."""
    P = [list(map(float, p)) for p in P]
    d = np.linalg.det(np.array([np.subtract(P[k], P[0]) for k in (1, 2, 3)]))
    if d < 0:
        P[1], P[2] = P[2], P[1]
    # facet opposite corner k, counter-clockwise seen from outside
    faces = [[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]]
    return Poly(P, faces)


def cut(poly: Poly, ax: int, c: float, cnt: Dict[str, int]):
    """Split poly by the plane x_ax = c into (below, above, first new point);
    either side may be None.  Counts classifications and intersections."""
    used = poly.used()
    cnt["cls"] += len(used)
    below = {v: poly.pts[v][ax] < c for v in used}
    if all(below.values()):
        return poly, None, None
    if not any(below.values()):
        return None, poly, None
    pts = [list(p) for p in poly.pts]
    cross: Dict[Tuple[int, int], int] = {}

    def point(a, b):
        key = (min(a, b), max(a, b))
        if key not in cross:
            lo, hi = (a, b) if below[a] else (b, a)
            pa, pb = pts[lo], pts[hi]
            t = (c - pa[ax]) / (pb[ax] - pa[ax])
            q = [pa[k] + t * (pb[k] - pa[k]) for k in range(3)]
            q[ax] = c
            pts.append(q)
            cross[key] = len(pts) - 1
            cnt["int"] += 1
        return cross[key]

    low_faces, up_faces = [], []
    cap_low: Dict[int, int] = {}   # next point of the lower part's cap loop
    cap_up: Dict[int, int] = {}
    for f in poly.faces:
        n = len(f)
        lo_loop, up_loop = [], []
        f_exit = f_entry = None  # where the loop leaves / re-enters the lower side
        for i in range(n):
            a, b = f[i], f[(i + 1) % n]
            if below[a]:
                lo_loop.append(a)
            else:
                up_loop.append(a)
            if below[a] != below[b]:
                q = point(a, b)
                lo_loop.append(q)
                up_loop.append(q)
                if below[a]:
                    f_exit = q
                else:
                    f_entry = q
        if len(lo_loop) >= 3:
            low_faces.append(lo_loop)
        if len(up_loop) >= 3:
            up_faces.append(up_loop)
        if f_exit is not None:
            # the facet's edge (exit -> entry) on the lower side, (entry ->
            # exit) on the upper side; each cap runs it the other way
            cap_low[f_entry] = f_exit
            cap_up[f_exit] = f_entry
    caps = []
    for nxt in (cap_low, cap_up):
        start = next(iter(nxt))
        loop, v = [start], nxt[start]
        while v != start:
            loop.append(v)
            v = nxt[v]
        caps.append(loop)
    first = min(cross.values())
    return Poly(pts, low_faces + [caps[0]]), Poly(pts, up_faces + [caps[1]]), first


def volume(poly: Poly, apex=None) -> float:
    """Volume by cones from the apex over the facets, each fanned."""
    P = poly.pts
    A = np.array(P[poly.faces[0][0]] if apex is None else P[apex])
    v = 0.0
    for f in poly.faces:
        p0 = np.array(P[f[0]]) - A
        for i in range(1, len(f) - 1):
            v += np.linalg.det(np.array([p0, np.array(P[f[i]]) - A, np.array(P[f[i + 1]]) - A])) / 6.0
    return v


def fan_count(poly: Poly, apex: int) -> int:
    return sum(len(f) - 2 for f in poly.faces if apex not in f)


def simplex_counts(P, cnt: Dict[str, int], pieces: Optional[list] = None) -> None:
    """Sweep one simplex (corners P [4][3] in cell units, unwrapped) and add
    its counts to cnt; with pieces given, append (cell, volume) per piece."""
    P = np.asarray(P, dtype=np.float64)
    lo = np.floor(P.min(axis=0)).astype(int)
    hi = np.floor(P.max(axis=0)).astype(int)
    span = hi - lo + 1
    order = sorted(range(3), key=lambda d: (span[d], d))  # smallest span outermost
    rest = tet(P)
    for i0 in range(lo[order[0]], hi[order[0]] + 1):
        if rest is None:
            break
        if i0 < hi[order[0]]:
            slab, rest, _ = cut(rest, order[0], float(i0 + 1), cnt)
        else:
            slab, rest = rest, None
        rest_s = slab
        for i1 in range(lo[order[1]], hi[order[1]] + 1):
            if rest_s is None:
                break
            if i1 < hi[order[1]]:
                col, rest_s, _ = cut(rest_s, order[1], float(i1 + 1), cnt)
            else:
                col, rest_s = rest_s, None
            rest_c = col
            below_apex = None
            for i2 in range(lo[order[2]], hi[order[2]] + 1):
                if rest_c is None:
                    break
                if i2 < hi[order[2]]:
                    piece, rest_c, top = cut(rest_c, order[2], float(i2 + 1), cnt)
                else:
                    piece, rest_c, top = rest_c, None, None
                if piece is not None:
                    apex = top if top is not None else (below_apex if below_apex is not None else piece.used()[0])
                    cnt["fan"] += fan_count(piece, apex)
                    cnt["pieces"] += 1
                    if pieces is not None:
                        cell = [0, 0, 0]
                        cell[order[0]], cell[order[1]], cell[order[2]] = i0, i1, i2
                        pieces.append((tuple(cell), volume(piece, apex)))
                below_apex = top
    return None


def cell_corners(prob) -> np.ndarray:
    """Corners [n][4][3] of a problem's simplices in cells of its grid, each
    unwrapped to the minimum image of its first corner on periodic axes."""
    X = np.asarray(prob["xyz"], dtype=np.float64)
    S = np.asarray(prob["simplices"], dtype=np.int64)
    dims = np.asarray(prob["dims"], dtype=np.float64)[:3]
    ext = np.asarray(prob["extent"], dtype=np.float64)[:3]
    org = np.asarray(prob["origin"], dtype=np.float64)[:3]
    P = X[S].copy()
    for d in range(3):
        if prob["periodic"][d]:
            P[:, :, d] = P[:, :, d] - ext[d] * np.rint((P[:, :, d] - P[:, :1, d]) / ext[d])
    return (P - org) * (dims / ext)


def counts(corners) -> Dict[str, float]:
    """Counts over simplices with corners [n][4][3] (cell units, unwrapped),
    with the flops they are priced at, in total and per piece."""
    cnt = {"pieces": 0, "cls": 0, "int": 0, "fan": 0}
    for P in corners:
        simplex_counts(P, cnt)
    flops = FLOPS_INT * cnt["int"] + FLOPS_CLS * cnt["cls"] + FLOPS_FAN * cnt["fan"]
    out = dict(cnt)
    out["flops"] = flops
    out["flops_per_piece"] = flops / max(cnt["pieces"], 1)
    return out
