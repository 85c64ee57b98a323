"""Pins of the work-count model of the slab recursion (oracle/work.py): the
arithmetic of the exact projection (Section 3, eq. eq_firstOrder; Appendix C)
counted as intersection points, classifications and fan tetrahedra.

PW1 a simplex inside one cell needs no cut and one fan triangle; PW2 one cut
through a tetrahedron, counted by hand (one corner below: four
classifications, three new points, 1 + 3 fan triangles); PW3 the pieces of
the recursion have the exact rational volumes of S cap G_j cell by cell
(oracle.exact, dyadic corners), so every piece is the true piece; PW4 the
number of pieces equals the brute-force C oracle's count of positive-volume
pieces on a deformed lattice; PW5 counts do not change under a shift by whole
cells."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import exact, work
from paper_1509_07720_amd import synth


def _cnt():
    return {"pieces": 0, "cls": 0, "int": 0, "fan": 0}


def test_pw1_single_cell():
    c = _cnt()
    work.simplex_counts([[0.1, 0.2, 0.3], [0.9, 0.1, 0.2], [0.2, 0.8, 0.4], [0.3, 0.3, 0.9]], c)
    assert c == {"pieces": 1, "cls": 0, "int": 0, "fan": 1}


def test_pw2_one_cut_by_hand():
    # corner 0 alone below x = 1: the cut classifies the 4 corners and crosses
    # the 3 edges from corner 0; the small tetrahedron below has one facet
    # away from its apex (a new point), the prism above three (its apex is a
    # new point on its bottom cap: the other quad and the top triangle)
    c = _cnt()
    pieces = []
    P = [[0.5, 0.25, 0.25], [1.75, 0.3, 0.4], [1.3, 0.6, 0.5], [1.4, 0.35, 0.7]]
    work.simplex_counts(P, c, pieces)
    assert c == {"pieces": 2, "cls": 4, "int": 3, "fan": 1 + 3}
    vol = abs(np.linalg.det(np.subtract(P[1:], P[0]))) / 6.0
    assert abs(sum(v for _, v in pieces) - vol) <= 1e-14


def _exact_cells(P):
    pts = [tuple(Fr(x) for x in p) + (Fr(1),) for p in P]
    lo = np.floor(np.min(P, axis=0)).astype(int)
    hi = np.floor(np.max(P, axis=0)).astype(int)
    out = {}
    for k in range(lo[2], hi[2] + 1):
        for j in range(lo[1], hi[1] + 1):
            for i in range(lo[0], hi[0] + 1):
                v, _ = exact.piece3(pts, (i, j, k))
                if v > 0:
                    out[(i, j, k)] = float(v)
    return out


def test_pw3_piece_volumes_are_exact():
    rng = np.random.default_rng(11)
    n = 0
    for t in range(12):
        s = [0.7, 1.6, 2.5][t % 3]
        c = rng.uniform(2.0, 6.0, 3)
        P = np.round((c + rng.uniform(-s, s, (4, 3))) * 16) / 16
        if abs(np.linalg.det(P[1:] - P[0])) < 1e-6:
            continue
        pieces = []
        work.simplex_counts(P, _cnt(), pieces)
        got = {}
        for cell, v in pieces:
            got[cell] = got.get(cell, 0.0) + v
        ref = _exact_cells(P)
        for cell in set(got) | set(ref):
            assert abs(got.get(cell, 0.0) - ref.get(cell, 0.0)) <= 1e-12 * max(1.0, abs(ref.get(cell, 0.0))), (t, cell)
        n += len(ref)
    assert n > 100


def test_pw4_piece_count_matches_brute_force():
    p = synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=3)
    r = oracle.project(p)
    assert r["stats"]["n_bad_span"] == 0  # both sides see every simplex
    c = work.counts(work.cell_corners(p))
    assert c["pieces"] == r["stats"]["n_pieces"]
    assert c["cls"] > 0 and c["int"] > 0 and c["fan"] >= c["pieces"]


def test_pw5_shift_by_whole_cells():
    P = np.array([[0.3, 0.4, 0.2], [2.6, 0.9, 1.3], [0.7, 3.1, 0.6], [1.1, 1.2, 2.8]])
    a, b = _cnt(), _cnt()
    work.simplex_counts(P, a)
    work.simplex_counts(P + np.array([5.0, -3.0, 7.0]), b)
    assert a == b and a["pieces"] > 5
