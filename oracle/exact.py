"""Exact-rational projection for tiny inputs -- TEST INFRASTRUCTURE.

Computes P_j = sum_i int_{S_i cap G_j} rho_i (Section 3, eq. eq_firstOrder)
in exact rational arithmetic (``fractions.Fraction``), so the result has no
rounding error at all for rational inputs.  The construction differs on
purpose from the C oracle: here the simplex is clipped in sequence by the
2*dim closed half-spaces of the cell, each cut closing the polytope with a cap
facet, and the final polytope is integrated by cones from the mean of its
vertices (Appendix C), each cone cut into tetrahedra along a fan of its facet.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from typing import Dict, List, Sequence, Tuple

Point = Tuple[Fr, ...]  # (x, y, [z,] rho)


def _clip_faces3(faces: List[List[Point]], d: int, c: Fr, keep_ge: bool) -> List[List[Point]]:
    """Clip a closed convex polytope, given as its facet polygons, by the
    half-space x_d >= c (keep_ge) or x_d <= c; add the cap facet."""

    def s(p):
        return (p[d] - c) if keep_ge else (c - p[d])

    out = []
    cap = []
    face_on_plane = False
    for f in faces:
        n = len(f)
        g = []
        for i in range(n):
            a, b = f[i], f[(i + 1) % n]
            sa, sb = s(a), s(b)
            if sa >= 0:
                g.append(a)
            if (sa >= 0) != (sb >= 0):
                t = sa / (sa - sb)
                g.append(tuple(a[k] + t * (b[k] - a[k]) for k in range(len(a))))
        # drop consecutive duplicates
        h = []
        for p in g:
            if not h or h[-1] != p:
                h.append(p)
        while len(h) > 1 and h[0] == h[-1]:
            h.pop()
        if len(h) >= 3:
            out.append(h)
            if all(s(p) == 0 for p in h):
                # a facet lying in the cutting plane already closes the cut
                face_on_plane = True
        for p in h:
            if s(p) == 0:
                cap.append(p)
    # cap facet: distinct on-plane points, ordered around their centroid in
    # the plane (exact angular comparison)
    uniq = []
    for p in cap:
        if p not in uniq:
            uniq.append(p)
    if len(uniq) >= 3 and not face_on_plane:
        ax = [k for k in range(3) if k != d]
        cx = sum(p[ax[0]] for p in uniq) / len(uniq)
        cy = sum(p[ax[1]] for p in uniq) / len(uniq)

        def half(p):
            x, y = p[ax[0]] - cx, p[ax[1]] - cy
            return 0 if (y > 0 or (y == 0 and x > 0)) else 1

        import functools

        def cmp(p, q):
            hp, hq = half(p), half(q)
            if hp != hq:
                return -1 if hp < hq else 1
            xp, yp = p[ax[0]] - cx, p[ax[1]] - cy
            xq, yq = q[ax[0]] - cx, q[ax[1]] - cy
            cr = xp * yq - yp * xq
            return -1 if cr > 0 else (1 if cr < 0 else 0)

        uniq.sort(key=functools.cmp_to_key(cmp))
        out.append(uniq)
    return out


def _det3(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def piece3(tet: Sequence[Point], cell: Tuple[int, int, int]) -> Tuple[Fr, Fr]:
    """(volume, integral of rho) of tet cap closed cell, exactly."""
    faces = [[tet[1], tet[2], tet[3]], [tet[0], tet[2], tet[3]], [tet[0], tet[1], tet[3]], [tet[0], tet[1], tet[2]]]
    for d in range(3):
        faces = _clip_faces3(faces, d, Fr(cell[d]), True)
        if not faces:
            return Fr(0), Fr(0)
        faces = _clip_faces3(faces, d, Fr(cell[d] + 1), False)
        if not faces:
            return Fr(0), Fr(0)
    verts = []
    for f in faces:
        for p in f:
            if p not in verts:
                verts.append(p)
    if len(verts) < 4:
        return Fr(0), Fr(0)
    O = tuple(sum(p[k] for p in verts) / len(verts) for k in range(4))
    vol = Fr(0)
    mass = Fr(0)
    for f in faces:
        for i in range(1, len(f) - 1):
            a, b, c = f[0], f[i], f[i + 1]
            v6 = abs(_det3([a[k] - O[k] for k in range(3)], [b[k] - O[k] for k in range(3)],
                           [c[k] - O[k] for k in range(3)]))
            vol += v6 / 6
            mass += v6 / 6 * (O[3] + a[3] + b[3] + c[3]) / 4
    return vol, mass


def _clip_poly2(poly: List[Point], d: int, c: Fr, keep_ge: bool) -> List[Point]:
    def s(p):
        return (p[d] - c) if keep_ge else (c - p[d])

    g = []
    n = len(poly)
    for i in range(n):
        a, b = poly[i], poly[(i + 1) % n]
        sa, sb = s(a), s(b)
        if sa >= 0:
            g.append(a)
        if (sa >= 0) != (sb >= 0):
            t = sa / (sa - sb)
            g.append(tuple(a[k] + t * (b[k] - a[k]) for k in range(len(a))))
    h = []
    for p in g:
        if not h or h[-1] != p:
            h.append(p)
    while len(h) > 1 and h[0] == h[-1]:
        h.pop()
    return h


def piece2(tri: Sequence[Point], cell: Tuple[int, int]) -> Tuple[Fr, Fr]:
    poly = list(tri)
    for d in range(2):
        poly = _clip_poly2(poly, d, Fr(cell[d]), True)
        if len(poly) < 3:
            return Fr(0), Fr(0)
        poly = _clip_poly2(poly, d, Fr(cell[d] + 1), False)
        if len(poly) < 3:
            return Fr(0), Fr(0)
    O = tuple(sum(p[k] for p in poly) / len(poly) for k in range(3))
    area = Fr(0)
    mass = Fr(0)
    n = len(poly)
    for i in range(n):
        a, b = poly[i], poly[(i + 1) % n]
        A2 = abs((a[0] - O[0]) * (b[1] - O[1]) - (a[1] - O[1]) * (b[0] - O[0]))
        area += A2 / 2
        mass += A2 / 2 * (O[2] + a[2] + b[2]) / 3
    return area, mass


def project(dim: int, simplices_xyz: Sequence[Sequence[Sequence[Fr]]], simplices_rho: Sequence[Sequence[Fr]],
            dims: Sequence[int]) -> Dict[Tuple[int, ...], Fr]:
    """Exact projection of simplices given directly in cell units (no
    periodic wrap): returns {cell index tuple: mass}, mass in cell-volume
    units.  Simplices of either orientation are accepted."""
    out: Dict[Tuple[int, ...], Fr] = {}
    for X, R in zip(simplices_xyz, simplices_rho):
        pts = [tuple(Fr(v) for v in x) + (Fr(r),) for x, r in zip(X, R)]
        lo = [math.floor(min(p[d] for p in pts)) for d in range(dim)]
        hi = [math.floor(max(p[d] for p in pts)) for d in range(dim)]
        if dim == 3:
            cells = [(i, j, k) for k in range(lo[2], hi[2] + 1) for j in range(lo[1], hi[1] + 1)
                     for i in range(lo[0], hi[0] + 1)]
        else:
            cells = [(i, j) for j in range(lo[1], hi[1] + 1) for i in range(lo[0], hi[0] + 1)]
        for c in cells:
            vol, m = (piece3 if dim == 3 else piece2)(pts, c)
            if vol > 0:
                key = tuple(int(c[d]) % int(dims[d]) for d in range(dim))
                out[key] = out.get(key, Fr(0)) + m
    return out


def polytope_faces(tet: Sequence[Point], cell: Tuple[int, int, int]) -> List[List[Point]]:
    """Facet polygons of tet cap closed cell (exact), for the corner-sum
    cross-check."""
    faces = [[tet[1], tet[2], tet[3]], [tet[0], tet[2], tet[3]], [tet[0], tet[1], tet[3]], [tet[0], tet[1], tet[2]]]
    for d in range(3):
        faces = _clip_faces3(faces, d, Fr(cell[d]), True)
        if not faces:
            return []
        faces = _clip_faces3(faces, d, Fr(cell[d] + 1), False)
        if not faces:
            return []
    return faces
