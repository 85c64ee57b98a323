"""Franklin's first-order corner sum (Section 3.1) -- TEST INFRASTRUCTURE.

For a polyhedron given by its facet polygons, every (vertex v, incident edge
e, incident facet f) triple defines unit vectors
  T  along e, leaving v;
  N  in the plane of f, orthogonal to T, pointing into f;
  B  normal to f, pointing into the polyhedron;
and, with P the position of v,
  E0 = -1/6 (P.T)(P.N)(P.B),   E1 = 1/4 ((P.T) T + 2 (P.N) N + 3 (P.B) B)
(eq. eq:E03D, eq:E13D).  The integral of the linear function
rho(X) = rho0 + grad.X over the polyhedron is the sum of E0 (rho0 + E1.grad)
over all triples (eq. eq_firstOrder, eq_contrib); with grad = 0 and rho0 = 1
it is the volume (eq. eq_vol).  In 2D the triples are (vertex, edge) with
E0 = 1/2 (P.T)(P.N), E1 = 1/3 ((P.T) T + 2 (P.N) N) (eq. eq:E02D, eq:E12D).

This is an independent formula for the same integrals the oracle computes by
cone decomposition, used only to cross-check it.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def _unit(v):
    n = np.linalg.norm(v)
    return v / n if n > 0 else v


def integral3(faces: Sequence[Sequence[Sequence[float]]], rho0: float, grad: Sequence[float]) -> float:
    """Integral of rho0 + grad.X over the polyhedron with the given facet
    polygons (each a cyclic list of 3D points, any orientation)."""
    F = [np.asarray(f, dtype=np.float64)[:, :3] for f in faces]
    allv = np.concatenate(F, axis=0)
    inside = allv.mean(axis=0)
    g = np.asarray(grad, dtype=np.float64)
    total = 0.0
    for f in F:
        c = f.mean(axis=0)
        # facet normal (Newell) oriented toward the interior
        n = np.zeros(3)
        m = len(f)
        for i in range(m):
            a, b = f[i], f[(i + 1) % m]
            n += np.cross(a, b)
        B = _unit(n)
        if np.dot(B, inside - c) < 0:
            B = -B
        for i in range(m):
            P = f[i]
            for j in ((i + 1) % m, (i - 1) % m):
                e = f[j] - P
                if np.linalg.norm(e) == 0:
                    continue
                T = _unit(e)
                N = _unit(np.cross(B, T))
                if np.dot(N, c - P) < 0:
                    N = -N
                pt, pn, pb = np.dot(P, T), np.dot(P, N), np.dot(P, B)
                E0 = -pt * pn * pb / 6.0
                E1 = 0.25 * (pt * T + 2 * pn * N + 3 * pb * B)
                total += E0 * (rho0 + np.dot(E1, g))
    return float(total)


def integral2(poly: Sequence[Sequence[float]], rho0: float, grad: Sequence[float]) -> float:
    """Integral of rho0 + grad.X over the convex polygon (cyclic list of 2D
    points, any orientation)."""
    p = np.asarray(poly, dtype=np.float64)[:, :2]
    c = p.mean(axis=0)
    g = np.asarray(grad, dtype=np.float64)[:2]
    m = len(p)
    total = 0.0
    for i in range(m):
        P = p[i]
        for j in ((i + 1) % m, (i - 1) % m):
            e = p[j] - P
            if np.linalg.norm(e) == 0:
                continue
            T = _unit(e)
            N = np.array([-T[1], T[0]])
            if np.dot(N, c - P) < 0:
                N = -N
            pt, pn = np.dot(P, T), np.dot(P, N)
            E0 = 0.5 * pt * pn
            E1 = (pt * T + 2 * pn * N) / 3.0
            total += E0 * (rho0 + np.dot(E1, g))
    return float(total)
