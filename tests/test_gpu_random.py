"""Seeded random problems against the oracle: tetrahedron soups and random
triangle soups on random grids (anisotropic cells, offset origins, mixed
periodic and non-periodic axes, per-vertex or per-corner densities, some
negative), both precisions.  A broad net for the cases the structured tests
do not hit."""
import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402

TOL = {"fp64": (1e-12, 1e-12), "fp32c": (1e-5, 1e-7)}


@pytest.fixture(scope="module")
def ctx():
    c = simproj.Context(0)
    yield c
    c.close()


def random_problem(seed):
    rng = np.random.default_rng(1000 + seed)
    dim = 3 if seed % 3 else 2
    dims = rng.integers(10, 40, size=dim)
    extent = rng.uniform(0.5, 3.0, size=dim)
    origin = rng.uniform(-2.0, 2.0, size=dim)
    periodic = tuple(bool(b) for b in rng.integers(0, 2, size=dim))
    n = int(rng.integers(200, 1500))
    # simplices around random centres, sizes from a tenth of a cell to a few cells
    cell = extent / dims
    centre = origin + rng.uniform(0.0, 1.0, size=(n, dim)) * extent
    top = min(3.0, dims.min() / 15.0)
    size = np.exp(rng.uniform(np.log(0.1), np.log(top), size=(n, 1))) * cell
    corners = centre[:, None, :] + rng.normal(size=(n, dim + 1, dim)) * size[:, None, :]
    # no simplex near half a periodic box (its minimum image would be a
    # rounding-dependent choice)
    ext = corners.max(axis=1) - corners.min(axis=1)
    keep = np.all(ext < 0.4 * extent, axis=1)
    corners, n = corners[keep], int(keep.sum())
    # keep the minimum image well defined on periodic axes
    for d in range(dim):
        if periodic[d]:
            corners[:, :, d] = origin[d] + np.mod(corners[:, :, d] - origin[d], extent[d])
    xyz = corners.reshape(-1, dim)
    simp = np.arange(n * (dim + 1), dtype=np.int32).reshape(n, dim + 1)
    per_corner = bool(seed % 2)
    if per_corner:
        rho = rng.uniform(-0.5, 2.0, size=(n, dim + 1))
    else:
        rho = rng.uniform(-0.5, 2.0, size=n * (dim + 1))
    o3, e3, d3 = np.zeros(3), np.ones(3), np.ones(3, np.int64)
    o3[:dim], e3[:dim], d3[:dim] = origin, extent, dims
    per3 = tuple(list(periodic) + [True] * (3 - dim))
    return dict(dim=dim, xyz=xyz, simplices=simp, rho=rho, rho_per_corner=per_corner, origin=o3, extent=e3,
                dims=d3, periodic=per3, meta=dict(recipe="random soup", seed=seed))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("seed", range(12))
def test_random_problem(ctx, seed, prec):
    prob = random_problem(seed)
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    ref = oracle.project(prob)
    D = prob["dim"]
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=dt, device=d)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=d)
    r = torch.tensor(prob["rho"], dtype=dt, device=d)
    g, total = ctx.project(x, s, r, list(prob["dims"][:D]), origin=list(prob["origin"][:D]),
                           extent=list(prob["extent"][:D]), periodic=prob["periodic"][:D], precision=prec,
                           rho_per_corner=prob["rho_per_corner"], out_mass=True, validate=False)
    got = g.double().cpu().numpy()
    err = oracle.cell_error(got, ref)
    tc, tm = TOL[prec]
    scale = np.abs(ref["mass"]).sum()
    assert err["e_cell"] <= tc, (seed, err, ref["stats"])
    assert abs(got.sum() - ref["mass"].sum()) <= tm * scale, (seed, err)
    assert abs(float(total.cpu()[0]) - ref["mass"].sum()) <= tm * scale
