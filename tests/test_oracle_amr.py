"""Pins of the two-stage (adaptive-resolution + donor-cell) projection
oracle (Section 4, "Calculation of the acceleration").

P14a the smallest height of a Kuhn tetrahedron of side s is s/sqrt(2);
P14b that of a regular tetrahedron of edge a is a sqrt(2/3), and its level
floor(log2 h); P14c with max_level 0 the result is the plain projection;
P14d donor-cell conserves mass, so the total equals the plain projection's;
P14e a uniform density stays uniform whatever the levels; P14f a single
coarse cell spreads evenly over its fine cells."""
import math

import numpy as np

import oracle
from oracle import amr
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
    assert set(np.unique(r["levels"])) - {0} != set()  # some coarse levels in use
    tot = oracle.simplex_mass(p).sum()
    assert abs(r["mass"].sum() - tot) <= 1e-12 * tot


def test_p14e_uniform_density_stays_uniform():
    p = synth.zeldovich_3d(n=8, grid=32, sigma_cells=0.0, seed=1)
    p = dict(p, rho=np.ones_like(np.asarray(p["rho"])))
    m = amr.project(p, 3)["mass"]
    assert np.allclose(m, 1.0 / 32 ** 3, rtol=1e-12)


def test_p14f_donor_cell():
    c = np.zeros((2, 2, 2))
    c[1, 0, 1] = 8.0
    f = amr.donor_cell(c, 1)
    assert f.shape == (4, 4, 4)
    assert np.allclose(f[2:4, 0:2, 2:4], 1.0) and f.sum() == 8.0
