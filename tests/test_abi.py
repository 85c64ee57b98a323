"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, the ctypes structures match the C layout, and
host-side argument validation returns the documented codes."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simproj.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sp_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sp_create", "sp_destroy", "sp_project_tets", "sp_project_tris", "sp_project_batch",
              "sp_sync_status", "sp_autotune", "sp_last_error", "sp_vertex_density", "sp_tuning_set",
              "sp_tuning_read", "sp_project_tets_accurate", "sp_project_tets_amr", "sp_project_tets_corners",
              "sp_project_tets_corners_fused"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1509_07720_amd import simproj

    lib = ctypes.CDLL(simproj.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", simproj.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sp_\w+)", out))
    assert set(_declared()) <= exported


def test_struct_layout_matches_c(tmp_path):
    from paper_1509_07720_amd import simproj

    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "simproj.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(sp_problem), offsetof(sp_problem,n_vert), offsetof(sp_problem,simplices),"
        "offsetof(sp_problem,rho), offsetof(sp_problem,grid), offsetof(sp_problem,out),"
        "offsetof(sp_problem,out_lo), offsetof(sp_problem,total_mass), sizeof(sp_grid),"
        "offsetof(sp_grid,dims), offsetof(sp_grid,flags)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P, G = simproj.sp_problem, simproj.sp_grid
    want = [ctypes.sizeof(P), P.n_vert.offset, P.simplices.offset, P.rho.offset, P.grid.offset, P.out.offset,
            P.out_lo.offset, P.total_mass.offset, ctypes.sizeof(G), G.dims.offset, G.flags.offset]
    assert got == want


def _prob(**kw):
    from paper_1509_07720_amd import simproj

    p = simproj.sp_problem()
    p.xyz = 0x1000
    p.n_vert = 4
    p.simplices = 0x2000
    p.n_simplex = 1
    p.rho = 0x3000
    p.out = 0x4000
    for d in range(3):
        p.grid.extent[d] = 1.0
        p.grid.dims[d] = 8
    p.grid.flags = 7
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("mutate, needle", [
    (lambda p: setattr(p.grid, "flags", 1 << 12), "unknown flag"),
    (lambda p: p.grid.dims.__setitem__(1, 0), "dims[1]"),
    (lambda p: p.grid.extent.__setitem__(2, -1.0), "extent[2]"),
    (lambda p: setattr(p, "n_simplex", 1 << 31), "n_simplex"),
    (lambda p: setattr(p, "n_vert", -1), "n_vert"),
    (lambda p: setattr(p, "out", None), "out is NULL"),
    (lambda p: setattr(p, "xyz", None), "must not be NULL"),
])
def test_host_validation_codes(mutate, needle):
    from paper_1509_07720_amd import simproj

    p = _prob()
    mutate(p)
    st = simproj.sp_project_tets(None, p, simproj.SP_PREC_FP32C)
    assert st == simproj.SP_E_INVALID_ARG
    assert needle in simproj.sp_last_error()


def test_host_validation_precision_and_ctx():
    from paper_1509_07720_amd import simproj

    p = _prob()
    assert simproj.sp_project_tets(None, p, 7) == simproj.SP_E_INVALID_ARG
    assert "precision" in simproj.sp_last_error()
    p.out_lo = 0x5000
    assert simproj.sp_project_tets(None, p, simproj.SP_PREC_FP64) == simproj.SP_E_INVALID_ARG
    assert "out_lo" in simproj.sp_last_error()
    p = _prob()
    assert simproj.sp_project_tets(None, p, simproj.SP_PREC_FP32C) == simproj.SP_E_INVALID_ARG
    assert "ctx is NULL" in simproj.sp_last_error()
    assert simproj.sp_project_tris(None, p, simproj.SP_PREC_FP32C) == simproj.SP_E_INVALID_ARG
    assert simproj.sp_sync_status(None) == simproj.SP_E_INVALID_ARG


def test_create_without_gpu_reports_device_error():
    code = ("import sys; sys.path.insert(0, %r); from paper_1509_07720_amd import simproj; "
            "st, h = simproj.sp_create(0); print(st)") % ROOT
    env = dict(os.environ)
    env["HIP_VISIBLE_DEVICES"] = "-1"  # hide any device, so the test means the same everywhere
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr
    assert int(out.stdout.strip().splitlines()[-1]) == 6  # SP_E_DEVICE


def test_vertex_density_host_validation():
    from paper_1509_07720_amd import simproj

    box = simproj.sp_grid()
    for d in range(3):
        box.extent[d] = 1.0
    box.flags = 7
    args = dict(dim=3, xyz=0x1000, n_vert=4, simplices=0x2000, n_simplex=1, mass=None, mass_uniform=1.0,
                box=box, rho_out=0x3000, prec=simproj.SP_PREC_FP64)

    def call(**kw):
        a = dict(args, **kw)
        return simproj.sp_vertex_density(None, a["dim"], a["xyz"], a["n_vert"], a["simplices"], a["n_simplex"],
                                         a["mass"], a["mass_uniform"], a["box"], a["rho_out"], a["prec"])

    assert call(dim=4) == simproj.SP_E_INVALID_ARG and "dim" in simproj.sp_last_error()
    assert call(prec=9) == simproj.SP_E_INVALID_ARG
    assert call(xyz=None) == simproj.SP_E_INVALID_ARG
    assert call(n_simplex=-1) == simproj.SP_E_INVALID_ARG
    assert call(mass_uniform=float("nan")) == simproj.SP_E_INVALID_ARG
    bad = simproj.sp_grid()
    bad.flags = simproj.SP_OUT_MASS
    for d in range(3):
        bad.extent[d] = 1.0
    assert call(box=bad) == simproj.SP_E_INVALID_ARG and "SP_PERIODIC" in simproj.sp_last_error()
    zero = simproj.sp_grid()
    zero.flags = 1
    assert call(box=zero) == simproj.SP_E_INVALID_ARG and "extent[0]" in simproj.sp_last_error()
    assert call() == simproj.SP_E_INVALID_ARG and "ctx is NULL" in simproj.sp_last_error()


def test_accurate_host_validation():
    from paper_1509_07720_amd import simproj

    p = _prob()
    st, _, _ = simproj.sp_project_tets_accurate(None, p, 10, 10)
    assert st == simproj.SP_E_INVALID_ARG and "ctx is NULL" in simproj.sp_last_error()
    for a, w, needle in ((0, 10, "accurate_bits"), (41, 10, "accurate_bits"), (10, -1, "wrong_bits"),
                         (10, 24, "wrong_bits")):
        st, _, _ = simproj.sp_project_tets_accurate(None, p, a, w)
        assert st == simproj.SP_E_INVALID_ARG and needle in simproj.sp_last_error()
    p.grid.flags |= simproj.SP_ACCUMULATE
    st, _, _ = simproj.sp_project_tets_accurate(None, p, 10, 10)
    assert st == simproj.SP_E_INVALID_ARG and "SP_ACCUMULATE" in simproj.sp_last_error()


def test_amr_host_validation():
    from paper_1509_07720_amd import simproj

    p = _prob()
    st, _ = simproj.sp_project_tets_amr(None, p, simproj.SP_PREC_FP32C, 2)
    assert st == simproj.SP_E_INVALID_ARG and "ctx is NULL" in simproj.sp_last_error()
    st, _ = simproj.sp_project_tets_amr(None, p, simproj.SP_PREC_FP32C, 11)
    assert st == simproj.SP_E_INVALID_ARG and "max_level" in simproj.sp_last_error()
    st, _ = simproj.sp_project_tets_amr(None, p, simproj.SP_PREC_FP32C, 4)  # dims 8 not a multiple of 16
    assert st == simproj.SP_E_INVALID_ARG and "multiple" in simproj.sp_last_error()


def test_corners_host_validation():
    from paper_1509_07720_amd import simproj

    p = _prob()
    assert simproj.sp_project_tets_corners(None, p) == simproj.SP_E_INVALID_ARG
    assert "ctx is NULL" in simproj.sp_last_error()
    p = _prob()
    p.grid.dims[1] = 0
    assert simproj.sp_project_tets_corners(None, p) == simproj.SP_E_INVALID_ARG
    assert "dims[1]" in simproj.sp_last_error()
    p = _prob()
    assert simproj.sp_project_tets_corners_fused(None, p) == simproj.SP_E_INVALID_ARG
    assert "ctx is NULL" in simproj.sp_last_error()
