"""Scratch memory of a context, through the C ABI.  SP_SCRATCH_CAP bounds
what a context may hold: a call that needs more fails with SP_E_NO_MEMORY
before it enqueues anything (its output keeps its old values) and the
context stays usable.  Growth is stream-ordered on the call's stream: one
context used on a side stream with problems of growing size gives the same
grids as fresh contexts on the default stream."""
import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402


def _dev(prob):
    d = torch.device("cuda:0")
    t = dict(xyz=torch.tensor(np.asarray(prob["xyz"]), dtype=torch.float32, device=d),
             simp=torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=d),
             rho=torch.tensor(np.asarray(prob["rho"]), dtype=torch.float32, device=d))
    t["out"] = torch.full(tuple(reversed(prob["dims"])), 7.0, dtype=torch.float32, device=d)
    t["lo"] = torch.zeros_like(t["out"])
    t["rec"] = simproj.make_problem(t["xyz"], t["simp"], t["rho"], prob["dims"], prob["origin"], prob["extent"],
                                    prob["periodic"], prob["rho_per_corner"], t["out"], t["lo"], out_mass=True)
    return t


def _grid(t):
    return t["out"].double() + t["lo"].double()


def _lattice(n, grid, seed):
    return synth.as_float32(synth.zeldovich_3d(n=n, grid=grid, sigma_cells=1.0, seed=seed))


def test_scratch_cap_refuses_a_call_and_the_context_stays_usable(monkeypatch):
    monkeypatch.setenv("SP_SCRATCH_CAP", "64M")
    ctx = simproj.Context(0)
    monkeypatch.delenv("SP_SCRATCH_CAP")
    stream = simproj._stream_ptr(None)
    small = _lattice(8, 16, 3)                # 3K tets: fits in 64 MiB
    big = _lattice(48, 64, 4)                 # 664K tets: about 90 MB of work lists
    ref = oracle.project(small)
    for step in ("before", "after"):
        print(f"scratch cap: small problem {step} the refused call", flush=True)
        t = _dev(small)
        assert simproj.sp_project_tets(ctx.handle, t["rec"], simproj.SP_PREC_FP32C, stream) == simproj.SP_OK, \
            simproj.sp_last_error()
        assert ctx.sync_status() == simproj.SP_OK
        err = oracle.cell_error(_grid(t).cpu().numpy(), ref)
        assert err["e_cell"] < 1e-5, err
        if step == "before":
            print("scratch cap: big problem, expect SP_E_NO_MEMORY", flush=True)
            tb = _dev(big)
            st = simproj.sp_project_tets(ctx.handle, tb["rec"], simproj.SP_PREC_FP32C, stream)
            assert st == simproj.SP_E_NO_MEMORY
            assert "SP_SCRATCH_CAP" in simproj.sp_last_error()
            torch.cuda.synchronize()
            assert float(tb["out"].min()) == 7.0 and float(tb["out"].max()) == 7.0  # nothing enqueued
    ctx.close()


def test_scratch_grows_in_order_on_a_side_stream():
    ctx = simproj.Context(0)
    side = torch.cuda.Stream()
    for n, grid, seed in ((8, 16, 5), (24, 48, 6), (40, 64, 7)):
        prob = _lattice(n, grid, seed)
        print(f"side stream: lattice {n}^3 onto {grid}^3", flush=True)
        a, b = _dev(prob), _dev(prob)
        torch.cuda.synchronize()
        assert simproj.sp_project_tets(ctx.handle, a["rec"], simproj.SP_PREC_FP32C, side.cuda_stream) == simproj.SP_OK
        fresh = simproj.Context(0)
        assert simproj.sp_project_tets(fresh.handle, b["rec"], simproj.SP_PREC_FP32C,
                                       simproj._stream_ptr(None)) == simproj.SP_OK
        side.synchronize()
        torch.cuda.synchronize()
        assert fresh.sync_status() == simproj.SP_OK
        fresh.close()
        ga, gb = _grid(a), _grid(b)
        assert float((ga - gb).abs().max()) <= 1e-6 * float(gb.abs().max())
    assert ctx.sync_status() == simproj.SP_OK
    ctx.close()
