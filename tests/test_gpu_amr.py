"""Adaptive-grid projection (sp_project_tets_amr) against its oracle
(oracle/amr.py: refined region by region until the cells are no larger than
the smallest height of any simplex intersecting them, exact projection onto
it, donor cell onto the uniform grid).  The grid must match FP64 to 1e-12
and FP32C to the usual per-cell and total bounds; every simplex is projected
at some level."""
import numpy as np
import pytest

import oracle
from oracle import amr
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


def _no_borderline(prob):
    h = amr.smallest_heights(prob)
    frac = np.log2(np.maximum(h, 1e-300))
    return np.all(np.abs(frac - np.rint(frac)) > 1e-9)


def _run(ctx, prob, prec, max_level):
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=dt, device=d)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=d)
    r = torch.tensor(prob["rho"], dtype=dt, device=d)
    dims = [int(v) for v in prob["dims"]]
    g, total, counts = ctx.project_amr(x, s, r, dims, max_level, precision=prec, extent=prob["extent"],
                                       periodic=prob["periodic"], rho_per_corner=prob["rho_per_corner"],
                                       out_mass=True, validate=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    return g.double().cpu().numpy(), float(total.cpu()[0]), counts


def _check(ctx, prob, prec, max_level):
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    assert _no_borderline(prob)
    ref = amr.project(prob, max_level)
    print(prec, "levels", np.bincount(ref["levels"]).tolist(), "leaves", np.bincount(ref["leaf"].ravel()).tolist(),
          flush=True)
    got, total, counts = _run(ctx, prob, prec, max_level)
    assert sum(counts) == prob["simplices"].shape[0]
    cov = oracle.project(prob)["cov"]
    err = oracle.cell_error(got, dict(mass=ref["mass"], cov=cov))
    tc, tm = TOL[prec]
    print(prec, err, "projection levels", counts, flush=True)
    assert err["e_cell"] <= tc and err["e_mass"] <= tm, err
    tot = oracle.simplex_mass(prob).sum()
    assert abs(total - tot) <= tm * tot
    return ref, counts


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("case", ["lattice", "corner"])
def test_amr_matches_oracle(ctx, prec, case):
    if case == "lattice":
        prob = synth.zeldovich_3d(n=10, grid=64, sigma_cells=1.0, seed=41)
    else:
        prob = synth.zeldovich_3d(n=12, grid=64, sigma_cells=1.5, seed=42, per_corner=True)
    ref, counts = _check(ctx, prob, prec, 3)
    assert len(set(ref["leaf"].ravel().tolist())) >= 3
    assert sum(counts[1:]) > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_amr_thin_inside_large(ctx, prec):
    """A large tetrahedron with thin ones inside it: around them the large
    one's contribution must be resolved at the finest level (leaves of one
    cell), away from them at its own level."""
    big = [[2.0, 2.0, 2.0], [30.0, 3.0, 4.0], [4.0, 29.0, 3.5], [3.0, 5.0, 30.0]]
    thin = [[9.3, 9.2, 9.1], [12.7, 9.6, 9.4], [9.5, 12.6, 9.3], [10.2, 10.1, 9.45]]
    thin2 = [[17.1, 5.3, 6.2], [19.6, 5.4, 6.3], [17.3, 7.7, 6.1], [18.2, 6.1, 7.9]]
    X = np.array([big, thin, thin2]) / 32.0
    prob = dict(dim=3, xyz=X.reshape(-1, 3), simplices=np.arange(12, dtype=np.int32).reshape(3, 4),
                rho=np.array([1.0, 2.0, 0.5, 1.5, 3.0, 1.0, 2.0, 2.0, 1.0, 1.0, 1.0, 2.0]), rho_per_corner=True,
                origin=np.zeros(3), extent=np.ones(3), dims=np.array([32, 32, 32]), periodic=(False, False, False))
    ref, counts = _check(ctx, prob, prec, 3)
    assert set(np.unique(ref["leaf"]).tolist()) == {0, 1, 2, 3}
    assert counts[0] == 3  # the large one meets single-cell leaves, so it is projected at level 0


def test_amr_level_zero_equals_plain(ctx):
    prob = synth.as_float32(synth.zeldovich_3d(n=10, grid=32, sigma_cells=1.0, seed=43))
    d = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=torch.float32, device=d)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=d)
    r = torch.tensor(prob["rho"], dtype=torch.float32, device=d)
    g, _, counts = ctx.project_amr(x, s, r, [32] * 3, 0, out_mass=True)
    plain, _ = ctx.project(x, s, r, [32] * 3, out_mass=True)
    assert counts == [s.shape[0]]
    ref = oracle.project(prob)
    for got in (g, plain):
        err = oracle.cell_error(got.double().cpu().numpy(), ref)
        assert err["e_cell"] <= 1e-5 and err["e_mass"] <= 1e-7


def test_amr_density_output(ctx):
    """Density output (the default) is the mass grid over the cell volume."""
    prob = synth.as_float32(synth.zeldovich_3d(n=8, grid=32, sigma_cells=1.0, seed=44))
    ref = amr.project(prob, 2)
    d = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=torch.float32, device=d)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=d)
    r = torch.tensor(prob["rho"], dtype=torch.float32, device=d)
    g, _, _ = ctx.project_amr(x, s, r, [32] * 3, 2)
    got = g.double().cpu().numpy() / 32 ** 3
    err = oracle.cell_error(got, dict(mass=ref["mass"], cov=oracle.project(prob)["cov"]))
    assert err["e_cell"] <= 1e-5 and err["e_mass"] <= 1e-7, err
