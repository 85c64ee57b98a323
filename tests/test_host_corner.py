"""The corner-sum projection (the header the corner kernel uses) compiled
for the host with g++ and compared with the oracle on the CPU: meshes in
general position, and degenerate ones -- corners on grid planes, lines and
points, edges and facets through grid lines and points -- which simulation
of simplicity resolves (Section 3.3, eq. eq_sos), all to 1e-12 per cell;
and the same with the fused facet contributions of App. D (eq.
eq_contribFused): the terms that two simplices sharing a facet contribute at
the same piece vertex summed once."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Corner sums are signed and cancel within a cell: per cell relative to the
# coverage scale, and of the total (the same bar as the FP64 clipping path).
TOL_CELL, TOL_MASS = 1e-12, 1e-12


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("corner") / "corner_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I",
                           os.path.join(ROOT, "paper_1509_07720_amd", "csrc"), "-o", so,
                           os.path.join(ROOT, "tests", "host", "corner_host.cpp")])
    L = ctypes.CDLL(so)
    V = ctypes.c_void_p
    L.corner_host.argtypes = [V, ctypes.c_int64, V, ctypes.c_int64, V, ctypes.c_int, V, V, V, V]
    L.corner_host_fused.argtypes = L.corner_host.argtypes
    return L


def corner(lib, prob, fused=False):
    x = np.ascontiguousarray(prob["xyz"], np.float64)
    s = np.ascontiguousarray(prob["simplices"], np.int32)
    r = np.ascontiguousarray(prob["rho"], np.float64)
    dims = np.asarray(prob["dims"], np.int32)
    per = np.asarray([1 if p else 0 for p in prob["periodic"]], np.int32)
    out = np.zeros(int(np.prod(dims)), np.float64)
    st = np.zeros(6, np.int64)
    (lib.corner_host_fused if fused else lib.corner_host)(x.ctypes.data, x.shape[0], s.ctypes.data, s.shape[0], r.ctypes.data, int(prob["rho_per_corner"]),
                    dims.ctypes.data, per.ctypes.data, out.ctypes.data, st.ctypes.data)
    return out.reshape(tuple(dims[::-1])), st


def snapped(prob, k):
    """Positions rounded to 1/k of a cell (unit box); simplices that become
    flat are dropped."""
    dims = np.asarray(prob["dims"], np.float64)
    x = np.round(np.asarray(prob["xyz"]) * dims * k) / (dims * k)
    x = np.mod(x, 1.0)
    S = np.asarray(prob["simplices"])
    P = synth.unwrapped_corners(x, S, np.ones(3), prob["periodic"])
    keep = np.abs(synth.signed_volumes(P)) > 1e-12
    return dict(prob, xyz=x, simplices=S[keep], rho=np.asarray(prob["rho"])[keep] if prob["rho_per_corner"]
                else prob["rho"])


def half_cell_soup(n, grid, seed):
    """n tetrahedra with corners on the half-cell lattice of a periodic grid
    (each within two cells of its first corner), per-corner densities."""
    rng = np.random.default_rng(seed)
    X, R = [], []
    while len(X) < n:
        c = rng.integers(0, 2 * grid, 3)
        P = (c + rng.integers(-4, 5, (4, 3))) / 2.0
        if abs(np.linalg.det(P[1:] - P[0])) < 1e-9:
            continue
        X.append(np.mod(P, grid) / grid)
        R.append(rng.uniform(0.5, 2.0, 4))
    return dict(dim=3, xyz=np.concatenate(X), simplices=np.arange(4 * n, dtype=np.int32).reshape(n, 4),
                rho=np.concatenate(R), rho_per_corner=True, origin=np.zeros(3), extent=np.ones(3),
                dims=np.array([grid] * 3), periodic=(True, True, True))


def stretched(prob):
    return dict(prob, xyz=np.asarray(prob["xyz"]) * 1.3 - 0.15, periodic=(False,) * 3)


PROBLEMS = {
    "lattice_3d": lambda: synth.zeldovich_3d(n=12, grid=24, sigma_cells=1.5, seed=2),
    "lattice_per_corner": lambda: synth.zeldovich_3d(n=8, grid=20, sigma_cells=1.0, seed=6, per_corner=True),
    "soup": lambda: synth.tet_soup(n_tets=3000, grid=32, seed=5),
    "refined": lambda: synth.refined_3d(n=6, grid=32, sigma_cells=1.0, seed=5),
    # FP32 coordinates on a grid of 48: some corners fall exactly on grid planes
    "soup_on_planes": lambda: synth.tet_soup(n_tets=20000, grid=48, seed=5),
    # every corner on a grid point
    "undisplaced_lattice": lambda: synth.zeldovich_3d(n=8, grid=16, sigma_cells=0.0, seed=1),
    # positions snapped to quarter cells: corners on grid planes, lines and
    # points, edges and facets through grid lines and points
    "quarter_cell_lattice": lambda: snapped(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=4), 4),
    # tetrahedra with every corner on the half-cell lattice
    "half_cell_soup": lambda: half_cell_soup(400, 12, seed=7),
    # a lattice stretched over a non-periodic box: wrapped simplices span it,
    # parts fall outside and are dropped
    "non_periodic": lambda: stretched(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=8)),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_corner_sums_match_oracle(lib, name):
    prob = PROBLEMS[name]()
    got, st = corner(lib, prob)
    assert st[2] == 0  # every simplex summed
    err = oracle.cell_error(got, oracle.project(prob))
    assert err["e_cell"] <= TOL_CELL, err
    assert err["e_mass"] <= TOL_MASS, err


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_fused_corner_sums_match_oracle(lib, name):
    prob = PROBLEMS[name]()
    got, st = corner(lib, prob, fused=True)
    assert st[2] == 0
    if name in ("lattice_3d", "lattice_per_corner", "refined", "undisplaced_lattice"):
        # a periodic lattice: every facet of a summed simplex is shared, but
        # for those of and next to a simplex skipped at set-up (flat ones) or
        # left out of the fusion (slivers)
        assert st[4] * 2 >= 4 * st[1] - 8 * (st[0] + st[5]), st
        assert st[5] * 100 < st[1], st
    if name == "quarter_cell_lattice":
        assert st[4] * 2 > 3 * st[1]  # (snapping flattened and dropped a few)
    if name in ("soup", "soup_on_planes", "half_cell_soup"):
        assert st[4] == 0  # independent simplices share no facet
    err = oracle.cell_error(got, oracle.project(prob))
    assert err["e_cell"] <= TOL_CELL, err
    assert err["e_mass"] <= TOL_MASS, err


def test_fused_terms_are_fewer_and_folds_are_paired(lib):
    """On a shell-crossed sheet some facets have both of their simplices on
    one side (sigma = +1); the fused sum still matches the oracle, and fewer
    terms are deposited than without fusion."""
    prob = synth.zeldovich_3d(n=12, grid=24, sigma_cells=3.0, seed=9)
    P = synth.unwrapped_corners(np.asarray(prob["xyz"]), np.asarray(prob["simplices"]), np.ones(3), prob["periodic"])
    assert (synth.signed_volumes(P) < 0).any()  # inverted simplices: folds
    got, st = corner(lib, prob, fused=True)
    plain, st0 = corner(lib, prob)
    assert st[3] < st0[3]
    err = oracle.cell_error(got, oracle.project(prob))
    assert err["e_cell"] <= TOL_CELL, err
    assert err["e_mass"] <= TOL_MASS, err
