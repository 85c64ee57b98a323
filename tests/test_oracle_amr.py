"""Pins of the adaptive-grid projection oracle (Section 4, "Calculation of
the acceleration": an adaptive grid refined region by region until its cells
are no larger than the smallest height of any simplex intersecting them,
exact projection onto it, donor-cell gather onto the uniform grid).

P14a the smallest height of a Kuhn tetrahedron of side s is s/sqrt(2);
P14b that of a regular tetrahedron of edge a is a sqrt(2/3), and its level
floor(log2 h); P14c with max_level 0 the result is the plain projection;
P14d mass is conserved; P14e a uniform density stays uniform whatever the
levels; P14f donor cell spreads a coarse cell evenly; P14g a thin simplex
inside a large one makes the large one's contribution resolved at the fine
level around the thin one (the per-region rule, not a per-simplex level);
P14h the intersection test agrees with exact rational clipping, touching
contacts included; P14i brute force on exact pieces: every leaf is no larger
than the smallest height of every simplex meeting it, and every refined block
is met by a simplex too thin for it (the grid is the coarsest that obeys the
rule); leaves are uniform blocks."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import amr, exact
from paper_1509_07720_amd import synth


def test_p14a_kuhn_heights():
    p = synth.zeldovich_3d(n=8, grid=32, sigma_cells=0.0, seed=1)
    h = amr.smallest_heights(p)
    assert np.allclose(h, 4.0 / math.sqrt(2.0), rtol=1e-12)
    assert np.all(amr.levels(p, 5) == 1)


def test_p14b_regular_tetrahedron():
    a = 5.0
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    v = v / np.linalg.norm(v[0] - v[1]) * a + 20.0
    prob = dict(dim=3, xyz=v, simplices=np.array([[0, 1, 2, 3]], np.int32), rho=np.ones(4), rho_per_corner=False,
                origin=np.zeros(3), extent=np.full(3, 64.0), dims=np.array([64, 64, 64]),
                periodic=(False, False, False))
    h = amr.smallest_heights(prob)[0]
    assert abs(h - a * math.sqrt(2.0 / 3.0)) <= 1e-12 * h
    assert amr.levels(prob, 9)[0] == int(math.floor(math.log2(a * math.sqrt(2.0 / 3.0))))


def test_p14c_level_zero_is_the_plain_projection():
    p = synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=3)
    a = amr.project(p, 0)["mass"]
    b = oracle.project(p, coverage=False)["mass"]
    assert np.array_equal(a, b)


def test_p14d_mass_is_conserved():
    p = synth.zeldovich_3d(n=8, grid=64, sigma_cells=1.5, seed=4)
    r = amr.project(p, 3)
    assert set(np.unique(r["leaf"])) - {0} != set()  # coarse leaves in use
    tot = oracle.simplex_mass(p).sum()
    assert abs(r["mass"].sum() - tot) <= 1e-12 * tot


def test_p14e_uniform_density_stays_uniform():
    p = synth.zeldovich_3d(n=8, grid=32, sigma_cells=0.0, seed=1)
    p = dict(p, rho=np.ones_like(np.asarray(p["rho"])))
    r = amr.project(p, 3)
    assert np.all(r["leaf"] == 1)  # side-4 Kuhn tets: height 2.83, level 1 everywhere
    assert np.allclose(r["mass"], 1.0 / 32 ** 3, rtol=1e-12)


def test_p14f_donor_cell():
    c = np.zeros((2, 2, 2))
    c[1, 0, 1] = 8.0
    f = amr.donor_cell(c, 1)
    assert f.shape == (4, 4, 4)
    assert np.allclose(f[2:4, 0:2, 2:4], 1.0) and f.sum() == 8.0


def _tets(X, R, dims, periodic=False):
    """A problem holding tetrahedra with corners X [n][4][3] in cell units."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    dims = np.asarray(dims)
    return dict(dim=3, xyz=X.reshape(-1, 3) / dims, simplices=np.arange(4 * n, dtype=np.int32).reshape(n, 4),
                rho=np.asarray(R, dtype=np.float64).reshape(-1), rho_per_corner=True, origin=np.zeros(3),
                extent=np.ones(3), dims=dims, periodic=(periodic,) * 3)


def test_p14g_thin_simplex_refines_the_large_one_around_it():
    """A large tetrahedron (smallest height ~11 cells: level 3) with a thin
    one (height < 1: level 0) inside it.  Around the thin one the grid is
    refined to single cells, so there the result is the exact projection of
    both -- the large one included, although on its own it would be spread
    over blocks of 8 cells.  Away from the thin one the large one alone sets
    the resolution (blocks of side 8)."""
    big = [[2.0, 2.0, 2.0], [30.0, 3.0, 4.0], [4.0, 29.0, 3.5], [3.0, 5.0, 30.0]]
    thin = [[9.3, 9.2, 9.1], [12.7, 9.6, 9.4], [9.5, 12.6, 9.3], [10.2, 10.1, 9.45]]
    R = [[1.0, 2.0, 0.5, 1.5], [3.0, 1.0, 2.0, 2.0]]
    prob = _tets([big, thin], R, [32, 32, 32])
    lv = amr.levels(prob, 3)
    assert list(lv) == [3, 0]
    r = amr.project(prob, 3)
    fine = oracle.project(prob, coverage=False)["mass"]
    leaf = r["leaf"]
    # the cells the thin tetrahedron meets are leaves of side 1 and hold the
    # exact projection of both tetrahedra
    thin_only = _tets([thin], [R[1]], [32, 32, 32])
    near = oracle.project(thin_only, coverage=False)["mass"] > 0
    assert near.sum() >= 8
    assert np.all(leaf[near] == 0)
    assert np.array_equal(r["mass"][leaf == 0], fine[leaf == 0])
    # the large tetrahedron covers them too, and its own contribution there
    # is not its level-3 average: the per-simplex reading differs there
    big_only = _tets([big], [R[0]], [32, 32, 32])
    fine_big = oracle.project(big_only, coverage=False)["mass"]
    assert np.all(fine_big[near] > 0)
    per_simplex_big = amr.donor_cell(amr.block_sums(fine_big, 3), 3)
    assert np.max(np.abs(fine_big[near] - per_simplex_big[near])) > 1e-3 * np.max(fine_big)
    # around them blocks grow back through sides 2 and 4 to 8
    assert set(np.unique(leaf).tolist()) == {0, 1, 2, 3}
    # far from the thin one, blocks of side 8 (inside the large one and
    # outside both)
    assert np.all(leaf[0:8, 0:8, 16:24] == 3) and fine_big[0:8, 0:8, 16:24].sum() > 0
    assert np.all(leaf[24:32, 24:32, 24:32] == 3)
    assert abs(r["mass"].sum() - fine.sum()) <= 1e-13 * fine.sum()


def _exact_meets(P, lo, size):
    """Positive volume of tet cap box, exactly: in units of the box side the
    box is a unit cell, whose exact rational piece is taken (corners are
    dyadic, so the scaling is exact too)."""
    pts = [tuple(Fr(v) / size for v in p) + (Fr(1),) for p in P]
    v, _ = exact.piece3(pts, tuple(int(lo[d]) // size for d in range(3)))
    return v > 0


def test_p14h_intersection_test_matches_exact_clipping():
    rng = np.random.default_rng(5)
    cases = 0
    for t in range(60):
        size = 2 if t % 2 else 4
        P = np.round(rng.uniform(0.0, 10.0, (4, 3)) * 4) / 4
        if t % 3 == 0:
            P[:3, t % 3] = np.round(P[0, t % 3] / size) * size  # a facet on a block plane
        if t % 5 == 0:
            P[1] = np.round(P[1] / size) * size                 # a corner on a block corner
        if abs(np.linalg.det(P[1:] - P[0])) < 1e-9:
            continue
        blo = np.floor(P.min(axis=0) / size).astype(int) - 1
        bhi = np.floor(P.max(axis=0) / size).astype(int) + 1
        lows = np.array([[i, j, k] for k in range(blo[2], bhi[2] + 1) for j in range(blo[1], bhi[1] + 1)
                         for i in range(blo[0], bhi[0] + 1)], dtype=np.float64) * size
        got = amr.meets(P, lows, float(size))
        for m in range(lows.shape[0]):
            assert got[m] == _exact_meets(P, lows[m], size), (t, P, lows[m])
            cases += 1
    assert cases > 1000


def test_p14i_brute_force_grid_rule():
    """Twelve dyadic tetrahedra of assorted sizes on a 16^3 grid, max level 2.
    With the cells each simplex meets taken from exact rational clipping:
    (a) every simplex meeting a leaf of side 2^l has level >= l; (b) every
    block of side 2^l > 1 that is refined is met by a simplex of level < l;
    (c) the leaf level is constant over each leaf block."""
    rng = np.random.default_rng(9)
    X, R = [], []
    for i in range(12):
        s = [0.6, 1.5, 3.0, 6.0][i % 4]
        c = rng.uniform(2.0, 14.0, 3)
        P = c + rng.uniform(-s, s, (4, 3))
        X.append(np.round(P * 8) / 8)
        R.append(rng.uniform(0.5, 2.0, 4))
    prob = _tets(X, R, [16, 16, 16], periodic=True)
    ML = 2
    lv = amr.levels(prob, ML)
    r = amr.project(prob, ML)
    leaf = r["leaf"]
    P = amr._unwrapped_cells(prob)
    met = []  # cells (x, y, z) with a positive exact piece, per simplex
    for i in range(P.shape[0]):
        pts = [tuple(Fr(v) for v in p) + (Fr(1),) for p in P[i]]
        lo = np.floor(P[i].min(axis=0)).astype(int)
        hi = np.floor(P[i].max(axis=0)).astype(int)
        cells = set()
        for k in range(lo[2], hi[2] + 1):
            for j in range(lo[1], hi[1] + 1):
                for q in range(lo[0], hi[0] + 1):
                    v, _ = exact.piece3(pts, (q, j, k))
                    if v > 0:
                        cells.add((q % 16, j % 16, k % 16))
        met.append(cells)
    assert len(set(lv.tolist())) >= 2
    # (c) uniform leaves
    for (z, y, x), l in np.ndenumerate(leaf):
        f = 1 << l
        blk = leaf[z // f * f:(z // f + 1) * f, y // f * f:(y // f + 1) * f, x // f * f:(x // f + 1) * f]
        assert np.all(blk == l)
    # (a) every simplex meeting a leaf is thick enough for it
    for i, cells in enumerate(met):
        for (x, y, z) in cells:
            assert lv[i] >= leaf[z, y, x], (i, (x, y, z))
    # (b) every refined block (its cells' leaves are smaller) is met by a
    # simplex too thin for it
    for l in range(1, ML + 1):
        f = 1 << l
        for bz in range(16 // f):
            for by in range(16 // f):
                for bx in range(16 // f):
                    blk = leaf[bz * f:(bz + 1) * f, by * f:(by + 1) * f, bx * f:(bx + 1) * f]
                    if np.all(blk >= l):
                        continue
                    inside = {(x, y, z) for z in range(bz * f, (bz + 1) * f) for y in range(by * f, (by + 1) * f)
                              for x in range(bx * f, (bx + 1) * f)}
                    assert any(lv[i] < l and (met[i] & inside) for i in range(len(met))), (l, bx, by, bz)
