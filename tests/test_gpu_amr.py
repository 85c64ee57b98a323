"""Two-stage projection (sp_project_tets_amr) against its oracle
(oracle/amr.py): the same per-simplex levels, and the same grid, FP64 to
1e-12 and FP32C to the usual per-cell and total bounds."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("case", ["lattice", "corner"])
def test_amr_matches_oracle(ctx, prec, case):
    if case == "lattice":
        prob = synth.zeldovich_3d(n=10, grid=64, sigma_cells=1.0, seed=41)
    else:
        prob = synth.zeldovich_3d(n=12, grid=64, sigma_cells=1.5, seed=42, per_corner=True)
    if prec == "fp32c":
        prob = synth.as_float32(prob)
    assert _no_borderline(prob)
    ref = amr.project(prob, 3)
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=dt, device=d)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=d)
    r = torch.tensor(prob["rho"], dtype=dt, device=d)
    g, total, counts = ctx.project_amr(x, s, r, [64] * 3, 3, precision=prec, rho_per_corner=prob["rho_per_corner"],
                                       out_mass=True, validate=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    assert counts == [int((ref["levels"] == l).sum()) for l in range(4)]
    assert sum(c for c in counts[1:]) > 0
    got = g.double().cpu().numpy()
    cov = oracle.project(prob)["cov"]
    err = oracle.cell_error(got, dict(mass=ref["mass"], cov=cov))
    tc, tm = TOL[prec]
    assert err["e_cell"] <= tc and err["e_mass"] <= tm, err
    tot = oracle.simplex_mass(prob).sum()
    assert abs(float(total.cpu()[0]) - tot) <= tm * tot


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
