"""GPU per-vertex density estimate (sp_vertex_density, through the C ABI)
against the oracle: FP64 mode to 1e-12 relative per vertex; FP32C mode (float
inputs, FP64 sums and division, rounded once) to 2^-23 relative."""
import numpy as np
import pytest

from oracle.vertex_density import vertex_density
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402

TOL = {"fp64": 1e-12, "fp32c": 2.0 ** -23}


@pytest.fixture(scope="module")
def ctx():
    c = simproj.Context(0)
    yield c
    c.close()


def _gpu(ctx, x, simp, mass, prec, extent, periodic, mass_uniform=1.0):
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    xt = torch.tensor(np.asarray(x), dtype=dt, device=d).contiguous()
    st = torch.tensor(np.asarray(simp), dtype=torch.int32, device=d).contiguous()
    mt = None if mass is None else torch.tensor(np.asarray(mass), dtype=dt, device=d).contiguous()
    r = ctx.vertex_density(xt, st, mt, mass_uniform, extent, periodic, precision=prec)
    status = ctx.sync_status()
    return r.double().cpu().numpy(), status


def _inputs(prob, prec):
    x = np.asarray(prob["xyz"], dtype=np.float64)
    if prec == "fp32c":
        x = x.astype(np.float32).astype(np.float64)
    return x


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_lattice_meshes_match_oracle(ctx, prec):
    rng = np.random.default_rng(3)
    for prob in (synth.zeldovich_3d(n=32, grid=64, sigma_cells=1.5, seed=2),
                 synth.two_sine_2d(n=32, grid=64, seed=1),
                 synth.refined_3d(n=8, grid=32, sigma_cells=2.0, seed=5)):
        x = _inputs(prob, prec)
        S = prob["simplices"]
        D = prob["dim"]
        m = rng.uniform(0.5, 2.0, S.shape[0])
        if prec == "fp32c":
            m = m.astype(np.float32).astype(np.float64)
        per = prob["periodic"][:D]
        ext = prob["extent"][:D]
        want = vertex_density(x, S, m, ext, per)
        got, st = _gpu(ctx, x, S, m, prec, ext, per)
        assert st == simproj.SP_OK, simproj.sp_last_error()
        rel = np.abs(got - want) / np.abs(want).max()
        print(prec, prob["meta"]["recipe"], rel.max(), flush=True)
        assert rel.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_uniform_mass_and_generator_density(ctx, prec):
    """Equal masses passed as one number reproduce the density the workload
    generator attaches to the config-2 lattice, and the oracle's."""
    prob = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2)
    x = _inputs(prob, prec)
    S = prob["simplices"]
    m0 = 1.0 / S.shape[0]
    want = vertex_density(x, S, m0)
    got, st = _gpu(ctx, x, S, None, prec, (1.0, 1.0, 1.0), (True, True, True), mass_uniform=m0)
    assert st == simproj.SP_OK
    assert (np.abs(got - want) / want).max() <= TOL[prec]
    if prec == "fp64":
        assert np.allclose(got, prob["rho"], rtol=1e-12)


def test_isolated_vertices_empty_and_bad_index(ctx):
    q, tets = synth.lattice_tets(4)
    x = np.vstack([q, [[0.5, 0.5, 0.5]]])
    got, st = _gpu(ctx, x, tets, None, "fp64", (1.0, 1.0, 1.0), (True, True, True), mass_uniform=1.0 / 384)
    assert st == simproj.SP_OK
    assert np.allclose(got[:-1], 1.0, rtol=1e-13) and got[-1] == 0.0
    got, st = _gpu(ctx, q, np.zeros((0, 4), dtype=np.int32), None, "fp64", (1.0,) * 3, (True,) * 3)
    assert st == simproj.SP_OK and np.all(got == 0.0)
    bad = tets.copy()
    bad[5, 2] = 10_000
    got, st = _gpu(ctx, q, bad, None, "fp64", (1.0,) * 3, (True,) * 3, mass_uniform=1.0 / 384)
    assert st == simproj.SP_E_OUT_OF_RANGE
    assert "bad index" in simproj.sp_last_error()
