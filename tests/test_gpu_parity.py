"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (per-cell error normalised by max(|R_j|, C_j), C_j the cell's
coverage scale; total-mass error relative):
  FP64 mode   e_cell <= 1e-12, e_mass <= 1e-12
  FP32C mode  e_cell <= 1e-5,  e_mass <= 1e-7
The FP32C oracle run sees the same float32-rounded inputs as the GPU.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402  (fails loudly if the library is missing)

TOL = {"fp64": (1e-12, 1e-12), "fp32c": (1e-5, 1e-7)}


@pytest.fixture(scope="module")
def ctx():
    c = simproj.Context(0)
    yield c
    c.close()


def _dev(prob, prec):
    dt = torch.float32 if prec == "fp32c" else torch.float64
    dev = torch.device("cuda:0")
    xyz = torch.tensor(np.asarray(prob["xyz"]), dtype=dt, device=dev).contiguous()
    simp = torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=dev).contiguous()
    rho = torch.tensor(np.asarray(prob["rho"]), dtype=dt, device=dev).contiguous()
    return xyz, simp, rho


def run(ctx, prob, prec, out_mass=True, validate=True, **kw):
    xyz, simp, rho = _dev(prob, prec)
    dim = prob["dim"]
    g, total = ctx.project(xyz, simp, rho, prob["dims"][:dim], origin=prob["origin"][:dim],
                           extent=prob["extent"][:dim], periodic=prob["periodic"][:dim], precision=prec,
                           rho_per_corner=prob["rho_per_corner"], out_mass=out_mass, validate=validate, **kw)
    st = ctx.sync_status()
    assert st == simproj.SP_OK, simproj.sp_last_error()
    return g.cpu().numpy().astype(np.float64), float(total.cpu()[0])


def check(ctx, prob, prec):
    ref_in = synth.as_float32(prob) if prec == "fp32c" else prob
    ref = oracle.project(ref_in)
    assert ref["stats"]["n_bad_span"] == 0
    got, total = run(ctx, ref_in, prec)
    err = oracle.cell_error(got, ref)
    tc, tm = TOL[prec]
    print(prec, prob["meta"].get("recipe"), err, flush=True)
    assert err["e_cell"] <= tc, err
    assert err["e_mass"] <= tm, err
    assert err["stray"] <= tc * max(ref["cov"].max(), 1e-300)
    assert abs(total - ref["mass"].sum()) <= tm * abs(ref["mass"].sum())
    return err


PROBLEMS = {
    "2d_two_sine": lambda: synth.two_sine_2d(n=32, grid=64, seed=1),
    "2d_two_sine_corner": lambda: synth.two_sine_2d(n=32, grid=64, seed=1, per_corner=True),
    "3d_zeldovich": lambda: synth.zeldovich_3d(n=16, grid=32, sigma_cells=1.5, seed=2),
    "3d_soup": lambda: synth.tet_soup(n_tets=20000, grid=256, seed=3),
    "3d_refined": lambda: synth.refined_3d(n=8, grid=48, sigma_cells=0.75, seed=5),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_parity(ctx, name, prec):
    check(ctx, PROBLEMS[name](), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_full_size_lattice_config(ctx, prec):
    """The 64^3-lattice Zel'dovich workload onto 128^3 at full size."""
    check(ctx, synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2), prec)


def test_full_size_soup_sampled_cells(ctx):
    """The 10M-tet soup onto 256^3 at full size, in the benchmark's launch
    configuration: every cell of a random sample against the oracle, and the
    total against the exact simplex masses."""
    prob = synth.tet_soup(n_tets=10_000_000, grid=256, seed=3)
    got, total = run(ctx, prob, "fp32c")
    rng = np.random.default_rng(0)
    mask = np.zeros(256 ** 3, dtype=np.uint8)
    # cells with mass (most of them) and a few arbitrary ones
    nz = np.flatnonzero(got.ravel() != 0)
    mask[rng.choice(nz, 3000, replace=False)] = 1
    mask[rng.integers(0, 256 ** 3, 500)] = 1
    ref = oracle.project(prob, cell_mask=mask)
    sel = mask.reshape(got.shape).astype(bool)
    err = oracle.cell_error(np.where(sel, got, 0.0), dict(mass=np.where(sel, ref["mass"], 0.0), cov=ref["cov"]))
    print("soup sampled", err, flush=True)
    assert err["e_cell"] <= 1e-5
    exact = oracle.simplex_mass(prob).sum()
    assert abs(got.sum() - exact) <= 1e-7 * exact
    assert abs(total - exact) <= 1e-7 * exact


@pytest.fixture(scope="module")
def refined_full():
    """The 50M-tet two-level refined lattice (128^3 coarse cubes, rms
    displacement 4 coarse cells) onto 512^3, float32-rounded."""
    return synth.as_float32(synth.refined_3d(n=128, grid=512, sigma_cells=4.0, seed=5))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_full_size_refined_subset(ctx, refined_full, prec):
    """Every 64th tetrahedron of the 50M-tet refined mesh onto the full 512^3
    grid (projection is additive over simplices): every cell against the
    oracle."""
    sub = synth.subset(refined_full, 64)
    ref = oracle.project(sub)
    assert ref["stats"]["n_bad_span"] == 0
    got, total = run(ctx, sub, prec)
    err = oracle.cell_error(got, ref)
    print("refined subset", prec, err, flush=True)
    tc, tm = TOL[prec]
    assert err["e_cell"] <= tc, err
    assert err["e_mass"] <= tm, err
    assert abs(total - ref["mass"].sum()) <= tm * ref["mass"].sum()


def test_full_size_refined_total(ctx, refined_full):
    """All 50M tetrahedra onto 512^3 in FP32C: the deposited total against
    the exact simplex masses, and no cell below rounding level of zero (all
    densities are positive)."""
    got, total = run(ctx, refined_full, "fp32c")
    exact = oracle.simplex_mass(refined_full).sum()
    print("refined total", total, exact, flush=True)
    assert abs(total - exact) <= 1e-7 * exact
    assert abs(got.sum() - exact) <= 1e-7 * exact
    assert got.min() >= -1e-6 * got.max()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_signed_coverage_full_size(ctx, prec):
    """Per-corner rho = sign(V) on the displaced periodic lattice covers every
    cell exactly once (the sheet is a degree-one map of the torus)."""
    prob = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2)
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    P = synth.unwrapped_corners(prob["xyz"], prob["simplices"], prob["extent"], prob["periodic"])
    sgn = np.sign(synth.signed_volumes(P))
    assert (sgn < 0).any()
    p = dict(prob, rho=np.repeat(sgn[:, None], 4, axis=1), rho_per_corner=True)
    got, _ = run(ctx, p, prec, out_mass=False)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.abs(got - 1.0).max() <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_lattice_aligned_degenerate(ctx, prec):
    """Undisplaced Kuhn lattice: every vertex and many facets lie exactly on
    grid planes; rho = 1 must give density 1 everywhere."""
    for n, grid in ((8, 16), (16, 16), (8, 32)):
        q, tets = synth.lattice_tets(n)
        prob = dict(dim=3, xyz=q, simplices=tets, rho=np.ones(q.shape[0]), rho_per_corner=False,
                    origin=np.zeros(3), extent=np.ones(3), dims=np.array([grid] * 3), periodic=(True,) * 3,
                    meta={})
        got, _ = run(ctx, prob, prec, out_mass=False)
        assert np.abs(got - 1.0).max() <= (1e-13 if prec == "fp64" else 1e-6), (n, grid)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_inside_one_cell_and_empty(ctx, prec):
    rng = np.random.default_rng(3)
    X = (rng.uniform(0.05, 0.95, (50, 4, 3)) + np.array([3, 4, 5])) / 8.0
    R = rng.uniform(0.5, 2.0, (50, 4))
    prob = dict(dim=3, xyz=X.reshape(-1, 3), simplices=np.arange(200, dtype=np.int32).reshape(50, 4),
                rho=R, rho_per_corner=True, origin=np.zeros(3), extent=np.ones(3), dims=np.array([8, 8, 8]),
                periodic=(True,) * 3, meta={})
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    ref = oracle.project(prob)
    got, _ = run(ctx, prob, prec)
    assert got[5, 4, 3] == pytest.approx(ref["mass"][5, 4, 3], rel=TOL[prec][1])
    got[5, 4, 3] = 0
    assert np.all(got == 0)
    empty = dict(prob, simplices=np.zeros((0, 4), dtype=np.int32), rho=np.zeros((0, 4)))
    got, total = run(ctx, empty, prec)
    assert np.all(got == 0) and total == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_dense_mesh_single_cell_merge(ctx, prec):
    """A 32^3 lattice onto 8^3 (384 tets per cell): most tetrahedra lie in one
    cell and are merged per cell and block before they reach the grid; the
    result must still match the oracle cell by cell, with signed densities
    as well (one simplex in ten negative)."""
    prob = synth.zeldovich_3d(n=32, grid=8, sigma_cells=0.2, seed=12, per_corner=True)
    rng = np.random.default_rng(12)
    prob["rho"] = prob["rho"] * np.where(rng.uniform(size=prob["rho"].shape[0]) < 0.1, -1.0, 1.0)[:, None]
    check(ctx, prob, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_non_periodic_drops_outside(ctx, prec):
    prob = synth.zeldovich_3d(n=16, grid=24, sigma_cells=1.0, seed=8)
    # shift and shrink so the mesh sticks out of a non-periodic box
    p = dict(prob, xyz=prob["xyz"] * 1.3 - 0.15, periodic=(False, False, False))
    if prec == "fp32c":
        p = synth.as_float32(p)
    ref = oracle.project(p)
    got, total = run(ctx, p, prec)
    err = oracle.cell_error(got, ref)
    assert err["e_cell"] <= TOL[prec][0] and err["e_mass"] <= TOL[prec][1], err


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_folded_flat_simplices(ctx, prec):
    """A stretched periodic lattice in a non-periodic box with every
    coordinate beyond the far face folded back to 0: huge, flat and nearly
    flat simplices (a nearly flat simplex has a huge density gradient across
    it), parts outside the box."""
    prob = synth.zeldovich_3d(n=16, grid=24, sigma_cells=1.0, seed=8)
    x = np.asarray(prob["xyz"]) * 1.3 - 0.15
    x = np.where(x.astype(np.float32) >= np.float32(1.0), 0.0, x)
    p = dict(prob, xyz=x, periodic=(False, False, False))
    if prec == "fp32c":
        p = synth.as_float32(p)
    ref = oracle.project(p)
    assert ref["stats"]["n_zero_volume"] > 0
    got, total = run(ctx, p, prec)
    err = oracle.cell_error(got, ref)
    assert err["e_cell"] <= TOL[prec][0] and err["e_mass"] <= TOL[prec][1], err


def test_accumulate_and_out_lo(ctx):
    prob = synth.as_float32(synth.zeldovich_3d(n=16, grid=32, sigma_cells=1.5, seed=2))
    ref = oracle.project(prob)
    xyz, simp, rho = _dev(prob, "fp32c")
    hi = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda:0")
    lo = torch.zeros_like(hi)
    half = simp.shape[0] // 2
    for part in (simp[:half].contiguous(), simp[half:].contiguous()):
        ctx.project(xyz, part, rho, [32] * 3, precision="fp32c", out=hi, out_lo=lo, out_mass=True, accumulate=True)
    assert ctx.sync_status() == simproj.SP_OK
    got = hi.cpu().numpy().astype(np.float64) + lo.cpu().numpy().astype(np.float64)
    err = oracle.cell_error(got, ref)
    assert err["e_cell"] <= 1e-5 and err["e_mass"] <= 1e-7, err


def test_validate_reports_bad_input(ctx):
    prob = synth.as_float32(synth.zeldovich_3d(n=8, grid=16, sigma_cells=0.5, seed=2))
    simp = prob["simplices"].copy()
    simp[3, 2] = prob["xyz"].shape[0] + 5  # out of range
    xyz = prob["xyz"].copy()
    xyz[simp[10, 0], 1] = np.nan
    p = dict(prob, simplices=simp, xyz=xyz)
    xyz_d, simp_d, rho_d = _dev(p, "fp32c")
    ctx.project(xyz_d, simp_d, rho_d, [16] * 3, precision="fp32c", validate=True)
    st = ctx.sync_status()
    assert st in (simproj.SP_E_OUT_OF_RANGE, simproj.SP_E_NONFINITE)
    assert "bad index" in simproj.sp_last_error()
    assert ctx.sync_status() == simproj.SP_OK  # cleared
    # without SP_VALIDATE the bad simplices are skipped silently
    ctx.project(xyz_d, simp_d, rho_d, [16] * 3, precision="fp32c", validate=False)
    assert ctx.sync_status() == simproj.SP_OK
