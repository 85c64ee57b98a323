"""sp_project_tets_noalloc (the entry point for callers that cannot allocate)
against sp_project_tets through the C ABI: two calls in a row on the same
GPU, the second with a smaller input, each equal to the allocating entry
point's result at the parity tolerances; a problem too large for the static
scratch is refused with SP_E_NO_MEMORY and nothing is enqueued."""
import numpy as np
import pytest

from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402

TOL = {"fp64": (1e-12, 1e-12), "fp32c": (1e-5, 1e-7)}


def _dev(prob, prec, keep_lo):
    dt = torch.float32 if prec == "fp32c" else torch.float64
    d = torch.device("cuda:0")
    t = dict(xyz=torch.tensor(np.asarray(prob["xyz"]), dtype=dt, device=d),
             simp=torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=d),
             rho=torch.tensor(np.asarray(prob["rho"]), dtype=dt, device=d))
    t["out"] = torch.full(tuple(reversed(prob["dims"])), 7.0, dtype=dt, device=d)  # stale values
    t["lo"] = torch.full_like(t["out"], 3.0, dtype=torch.float32) if keep_lo else None
    t["total"] = torch.zeros(1, dtype=torch.float64, device=d)
    t["rec"] = simproj.make_problem(t["xyz"], t["simp"], t["rho"], prob["dims"], prob["origin"], prob["extent"],
                                    prob["periodic"], prob["rho_per_corner"], t["out"], t["lo"], t["total"],
                                    out_mass=True, validate=True)
    return t


def _grid(t):
    g = t["out"].double()
    if t["lo"] is not None:
        g = g + t["lo"].double()
    return g


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("keep_lo", [False, True])
def test_noalloc_matches_allocating_call_twice(prec, keep_lo):
    if keep_lo and prec == "fp64":
        pytest.skip("out_lo is an FP32C buffer")
    ctx = simproj.Context(0)
    code = simproj.SP_PREC_FP32C if prec == "fp32c" else simproj.SP_PREC_FP64
    stream = simproj._stream_ptr(None)
    big = synth.zeldovich_3d(n=40, grid=96, sigma_cells=1.5, seed=31)
    small = synth.zeldovich_3d(n=20, grid=48, sigma_cells=1.5, seed=32)
    for name, prob in (("first (larger)", big), ("second (smaller)", small)):
        if prec == "fp32c":
            prob = synth.as_float32(prob)
        print(f"noalloc {prec} keep_lo={keep_lo}: {name}, {prob['simplices'].shape[0]} tets", flush=True)
        a = _dev(prob, prec, keep_lo)
        b = _dev(prob, prec, keep_lo)
        assert simproj.sp_project_tets_noalloc(ctx.handle, a["rec"], code, stream) == simproj.SP_OK, \
            simproj.sp_last_error()
        assert simproj.sp_project_tets(ctx.handle, b["rec"], code, stream) == simproj.SP_OK
        assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
        ga, gb = _grid(a), _grid(b)
        tc, tm = TOL[prec]
        scale = float(gb.abs().max())
        assert scale > 0
        assert float((ga - gb).abs().max()) <= tc * scale, name
        ta, tb = float(a["total"].cpu()[0]), float(b["total"].cpu()[0])
        assert abs(ta - tb) <= tm * abs(tb), name
    ctx.close()


def test_noalloc_refuses_a_problem_beyond_its_scratch():
    """About 780K tets fit with a caller-held low grid; 20M cannot (20M
    simplices need over 2 GB of work lists and set-up records; the check is
    on sizes alone, before anything is enqueued)."""
    ctx = simproj.Context(0)
    d = torch.device("cuda:0")
    xyz = torch.zeros((4, 3), dtype=torch.float32, device=d)
    simp = torch.zeros((1, 4), dtype=torch.int32, device=d)
    rho = torch.zeros(4, dtype=torch.float32, device=d)
    out = torch.full((8, 8, 8), 5.0, dtype=torch.float32, device=d)
    rec = simproj.make_problem(xyz, simp, rho, [8, 8, 8], out=out)
    rec.n_simplex = 20_000_000
    st = simproj.sp_project_tets_noalloc(ctx.handle, rec, simproj.SP_PREC_FP32C, simproj._stream_ptr(None))
    assert st == simproj.SP_E_NO_MEMORY
    assert "static scratch" in simproj.sp_last_error()
    torch.cuda.synchronize()
    assert float(out.min()) == 5.0 and float(out.max()) == 5.0  # nothing was enqueued
    ctx.close()
