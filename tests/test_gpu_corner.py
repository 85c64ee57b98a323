"""The corner-sum projection (sp_project_tets_corners, FP64), and the same
with the fused facet contributions of App. D (sp_project_tets_corners_fused),
against the oracle, against the FP64 clipping projection at full size, and
their device-side input checks, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402
from test_host_corner import half_cell_soup, snapped  # noqa: E402  (input builders only)

# signed corner terms cancel within a cell: per cell relative to the
# coverage scale, and of the total (the clipping path holds 1e-12 for both)
TOL_CELL, TOL_MASS = 1e-12, 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = simproj.Context(0)
    yield c
    c.close()


def _dev(prob):
    d = torch.device("cuda:0")
    x = torch.tensor(np.asarray(prob["xyz"]), dtype=torch.float64, device=d)
    s = torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=d)
    r = torch.tensor(np.asarray(prob["rho"]), dtype=torch.float64, device=d)
    return x, s, r


def stretched(prob):
    return dict(prob, xyz=np.asarray(prob["xyz"]) * 1.3 - 0.15, periodic=(False,) * 3)


CASES = {
    "lattice_3d": lambda: synth.zeldovich_3d(n=12, grid=24, sigma_cells=1.5, seed=2),
    "lattice_per_corner": lambda: synth.zeldovich_3d(n=8, grid=20, sigma_cells=1.0, seed=6, per_corner=True),
    "soup": lambda: synth.tet_soup(n_tets=20000, grid=48, seed=5),
    "refined": lambda: synth.refined_3d(n=8, grid=48, sigma_cells=1.0, seed=5),
    "undisplaced_lattice": lambda: synth.zeldovich_3d(n=8, grid=16, sigma_cells=0.0, seed=1),
    # stretched over a non-periodic box: wrapped simplices span it, parts fall outside
    "non_periodic": lambda: stretched(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=8)),
    # degenerate positions resolved by simulation of simplicity
    "quarter_cell_lattice": lambda: snapped(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=4), 4),
    "half_cell_soup": lambda: half_cell_soup(400, 12, seed=7),
}


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_corners_match_oracle(ctx, name, fused):
    prob = CASES[name]()
    x, s, r = _dev(prob)
    g, total = ctx.project_corners(x, s, r, list(prob["dims"]), periodic=prob["periodic"],
                                   rho_per_corner=prob["rho_per_corner"], out_mass=True, fused=fused)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    ref = oracle.project(prob)
    err = oracle.cell_error(g.cpu().numpy(), ref)
    print(name, "fused" if fused else "plain", err, flush=True)
    assert err["e_cell"] <= TOL_CELL and err["e_mass"] <= TOL_MASS, err
    assert abs(float(total.cpu()[0]) - ref["mass"].sum()) <= TOL_MASS * ref["mass"].sum()


def test_corners_agree_with_clipping_at_full_size(ctx):
    """The 1.57M-tet lattice onto 128^3: the two FP64 algorithms on the GPU
    each match the oracle on every cell to the per-cell bar, and both totals
    match the exact sum of the simplex masses."""
    prob = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2)
    x, s, r = _dev(prob)
    gc, tc = ctx.project_corners(x, s, r, [128] * 3, out_mass=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    gf, tf = ctx.project_corners(x, s, r, [128] * 3, out_mass=True, fused=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    gp, tp = ctx.project(x, s, r, [128] * 3, precision="fp64", out_mass=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    ref = oracle.project(prob)
    # Each cell of this mesh takes the signed terms of many overlapping
    # simplices (heavy shell crossing): their rounding adds up, so the corner
    # sums are held to 1e-11 of the coverage scale here (1e-14 on the small
    # meshes above), the clipping path to its own 1e-12.  The worst cell
    # holds a sliver (volume 2.8e-7 cells, density gradient 7.8e6 per cell
    # against corner densities near 5): its terms are about 1e6 times its
    # pieces and cancel (the loss of bits of Section 3.4); the fused terms
    # of its neighbours' facets are formed on other vectors than their
    # unfused twins, and the fused sums are held to 2e-11 there
    for name, g, tol in (("corners", gc, 1e-11), ("fused corners", gf, 2e-11), ("clipping", gp, 1e-12)):
        err = oracle.cell_error(g.cpu().numpy(), ref)
        print(name, err, flush=True)
        assert err["e_cell"] <= tol and err["e_mass"] <= TOL_MASS, (name, err)
    exact = oracle.simplex_mass(prob).sum()
    assert abs(float(tc.cpu()[0]) - exact) <= TOL_MASS * exact
    assert abs(float(tf.cpu()[0]) - exact) <= TOL_MASS * exact
    assert abs(float(tp.cpu()[0]) - exact) <= 1e-12 * exact


def test_density_output_matches_clipping(ctx):
    prob = synth.zeldovich_3d(n=10, grid=16, sigma_cells=1.0, seed=8)
    x, s, r = _dev(prob)
    gc, _ = ctx.project_corners(x, s, r, [16] * 3)
    gp, _ = ctx.project(x, s, r, [16] * 3, precision="fp64")
    assert ctx.sync_status() == simproj.SP_OK
    assert float((gc - gp).abs().max() / gp.abs().max()) <= TOL_CELL


def test_validate_reports_bad_input(ctx):
    prob = synth.zeldovich_3d(n=4, grid=8, sigma_cells=0.0, seed=1)
    prob["simplices"] = np.array(prob["simplices"], copy=True)
    prob["simplices"][3, 2] = 10 ** 6  # index out of range: skipped, reported
    x, s, r = _dev(prob)
    ctx.project_corners(x, s, r, [8] * 3, out_mass=True, validate=True)
    assert ctx.sync_status() == simproj.SP_E_OUT_OF_RANGE
    assert "1 bad index" in simproj.sp_last_error()


def test_fused_on_a_folded_sheet_and_repeated_calls(ctx):
    """A strongly shell-crossed sheet (facets with both simplices on one
    side), projected twice in a row with the fused terms (the facet table is
    rebuilt each call), then a smaller mesh: each against the oracle."""
    big = synth.zeldovich_3d(n=16, grid=32, sigma_cells=3.0, seed=9)
    small = synth.zeldovich_3d(n=6, grid=12, sigma_cells=1.0, seed=3)
    for prob in (big, big, small):
        x, s, r = _dev(prob)
        g, _ = ctx.project_corners(x, s, r, list(prob["dims"]), out_mass=True, fused=True)
        assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
        err = oracle.cell_error(g.cpu().numpy(), oracle.project(prob))
        print("folded/fused", err, flush=True)
        assert err["e_cell"] <= TOL_CELL and err["e_mass"] <= TOL_MASS, err


def test_fused_terms_reach_the_grid_less_often(ctx):
    """The facet matching finds the shared facets on the device: with the
    pairs summed once, fewer vertices deposit terms than without fusion (a
    corner of the mesh whose three facets are all summed by neighbours of
    lower index deposits nothing); deposits counted in profiling mode 2."""
    prob = synth.zeldovich_3d(n=12, grid=24, sigma_cells=1.5, seed=2)
    x, s, r = _dev(prob)
    counts = []
    for fused in (False, True):
        assert simproj.sp_profile_enable(ctx.handle, 2) == simproj.SP_OK
        ctx.project_corners(x, s, r, [24] * 3, out_mass=True, fused=fused)
        assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
        st, prof = simproj.sp_profile_read(ctx.handle)
        assert st == simproj.SP_OK
        counts.append(int(prof.pieces))
        assert simproj.sp_profile_enable(ctx.handle, 0) == simproj.SP_OK
    print("deposits plain/fused", counts, flush=True)
    assert 0 < counts[1] < counts[0], counts
