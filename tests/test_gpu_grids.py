"""Grid descriptions beyond the unit cube: anisotropic cells, offset
origins, non-power-of-two resolutions (the FP32 cell split then needs its
error-free product), 2D and 3D, and a grid of more than 2^32 cells."""
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


def _run(ctx, prob, prec, out_mass=True):
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    D = prob["dim"]
    x = torch.tensor(np.asarray(prob["xyz"]), dtype=dt, device=d)
    s = torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=d)
    r = torch.tensor(np.asarray(prob["rho"]), dtype=dt, device=d)
    g, total = ctx.project(x, s, r, list(prob["dims"][:D]), origin=list(prob["origin"][:D]),
                           extent=list(prob["extent"][:D]), periodic=prob["periodic"][:D], precision=prec,
                           rho_per_corner=prob["rho_per_corner"], out_mass=out_mass, validate=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    return g, float(total.cpu()[0])


def _placed(prob, origin, extent, dims):
    D = prob["dim"]
    o = np.zeros(3)
    e = np.ones(3)
    o[:D], e[:D] = origin, extent
    d3 = np.ones(3, np.int64)
    d3[:D] = dims
    return dict(prob, xyz=o[:D] + np.asarray(prob["xyz"]) * e[:D], origin=o, extent=e, dims=d3)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_anisotropic_offset_grid_3d(ctx, prec):
    base = synth.zeldovich_3d(n=12, grid=32, sigma_cells=1.5, seed=31)
    prob = _placed(base, (-0.3, 0.1, 0.7), (2.0, 1.0, 0.5), (24, 40, 12))
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    ref = oracle.project(prob)
    g, total = _run(ctx, prob, prec)
    err = oracle.cell_error(g.double().cpu().numpy(), ref)
    tc, tm = TOL[prec]
    assert err["e_cell"] <= tc and err["e_mass"] <= tm, err
    assert abs(total - ref["mass"].sum()) <= tm * ref["mass"].sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_anisotropic_offset_grid_2d(ctx, prec):
    base = synth.two_sine_2d(n=24, grid=48, seed=32, per_corner=True)
    prob = _placed(base, (1.25, -0.6), (3.0, 0.75), (60, 22))
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    ref = oracle.project(prob)
    g, total = _run(ctx, prob, prec)
    err = oracle.cell_error(g.double().cpu().numpy(), ref)
    tc, tm = TOL[prec]
    assert err["e_cell"] <= tc and err["e_mass"] <= tm, err


def test_grid_of_more_than_2_32_cells(ctx):
    """2048 x 2048 x 1040 cells (4.36e9 > 2^32) in FP64, with a displaced
    lattice block near the far corner: the block's cells must equal the
    oracle's projection of the same block translated next to the origin
    (cell-aligned dyadic translation, exact in FP64), and every other cell
    must be zero."""
    base = synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=33)
    q = np.round(np.asarray(base["xyz"]) * 2.0 ** 30) / 2.0 ** 30
    dims = (2048, 2048, 1040)
    off = np.array([2020.0, 2020.0, 1010.0])
    far = dict(base, xyz=q * 16.0 + off, origin=np.zeros(3), extent=np.array(dims, float),
               dims=np.array(dims), periodic=(False, False, False))
    near = dict(base, xyz=q * 16.0 + 2.0, origin=np.zeros(3), extent=np.full(3, 24.0), dims=np.array([24] * 3),
                periodic=(False, False, False))
    ref = oracle.project(near)
    assert ref["stats"]["n_bad_span"] == 0
    g, total = _run(ctx, far, "fp64")
    assert g.shape == (1040, 2048, 2048)
    lo = (off - 2.0).astype(int)  # cell (0,0,0) of the small grid
    block = g[lo[2]:lo[2] + 24, lo[1]:lo[1] + 24, lo[0]:lo[0] + 24].cpu().numpy()
    err = oracle.cell_error(block, ref)
    assert err["e_cell"] <= 1e-12 and err["e_mass"] <= 1e-12, err
    assert abs(float(g.sum()) - ref["mass"].sum()) <= 1e-12 * ref["mass"].sum()
    assert abs(total - ref["mass"].sum()) <= 1e-12 * ref["mass"].sum()
    del g
    torch.cuda.empty_cache()
