"""Pins of the per-vertex density oracle (Section 4, "Calculation of the
acceleration": rho_j = sum of incident masses / sum of incident volumes).

P13a a hand-worked pair of triangles (golden fixture); P13b undisplaced
periodic lattices in 2D and 3D with equal masses give the closed form
rho = M / V everywhere; P13c an integer shear of the torus preserves every
volume, so rho stays uniform while the corners wrap across the box; P13d a
uniform scaling of the box by s divides rho by s^D; P13e inverted simplices
count with their unsigned volume; P13f masses enter linearly."""
import os

import numpy as np

from oracle.vertex_density import vertex_density
from paper_1509_07720_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_p13a_two_triangles_by_hand():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "vertex_density_two_triangles.txt"))
            if l.strip() and not l.startswith("#")]
    xy = np.array([[float(r[1]), float(r[2])] for r in rows])
    want = np.array([float(r[3]) for r in rows])
    tris = np.array([[0, 1, 2], [1, 3, 2]])
    got = vertex_density(xy, tris, 1.0, extent=(10.0, 10.0), periodic=(False, False))
    assert np.allclose(got, want, rtol=1e-15, atol=0)


def test_p13b_undisplaced_lattices_closed_form():
    for n in (3, 8):
        q, tets = synth.lattice_tets(n)
        got = vertex_density(q, tets, 1.0 / tets.shape[0])
        assert np.allclose(got, 1.0, rtol=1e-13)
        q2, tris = synth.lattice_tris(n)
        got2 = vertex_density(q2, tris, 3.0 / tris.shape[0], periodic=(True, True))
        assert np.allclose(got2, 3.0, rtol=1e-13)


def test_p13c_integer_shear_of_the_torus():
    n = 6
    q, tets = synth.lattice_tets(n)
    x = q.copy()
    x[:, 0] = np.mod(q[:, 0] + q[:, 1], 1.0)  # det 1, maps the lattice to itself
    P = synth.unwrapped_corners(x, tets, np.ones(3), (True, True, True))
    assert (np.ptp(P[:, :, 0], axis=1) > 1.5 / n).any()  # the shear really stretches the tets
    raw = x[tets]
    assert (np.ptp(raw[:, :, 0], axis=1) > 0.5).any()      # and some corners wrap across the box
    got = vertex_density(x, tets, 1.0 / tets.shape[0])
    assert np.allclose(got, 1.0, rtol=1e-12)


def test_p13d_scaling():
    s = 2.5
    q, tets = synth.lattice_tets(4)
    got = vertex_density(q * s, tets, 1.0 / tets.shape[0], extent=(s, s, s))
    assert np.allclose(got, 1.0 / s ** 3, rtol=1e-13)


def test_p13e_inverted_simplices_count_unsigned():
    prob = synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.5, seed=11)
    x, tets = prob["xyz"], prob["simplices"]
    rng = np.random.default_rng(1)
    m = rng.uniform(0.5, 2.0, tets.shape[0])
    a = vertex_density(x, tets, m)
    flipped = tets.copy()
    sel = rng.random(tets.shape[0]) < 0.5
    flipped[sel, 1], flipped[sel, 2] = tets[sel, 2], tets[sel, 1]
    b = vertex_density(x, flipped, m)
    assert np.allclose(a, b, rtol=1e-14)
    assert (a > 0).all()


def test_p13f_linear_in_the_masses():
    prob = synth.zeldovich_3d(n=6, grid=12, sigma_cells=1.0, seed=12)
    x, tets = prob["xyz"], prob["simplices"]
    rng = np.random.default_rng(2)
    m1, m2 = rng.random(tets.shape[0]), rng.random(tets.shape[0])
    r1, r2 = vertex_density(x, tets, m1), vertex_density(x, tets, m2)
    r12 = vertex_density(x, tets, 2.0 * m1 + 3.0 * m2)
    assert np.allclose(r12, 2.0 * r1 + 3.0 * r2, rtol=1e-13)
    # an isolated vertex (no incident simplex) gets 0
    xx = np.vstack([x, [[0.5, 0.5, 0.5]]])
    assert vertex_density(xx, tets, m1)[-1] == 0.0
