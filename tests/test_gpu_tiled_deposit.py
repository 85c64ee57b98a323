"""The opt-in deposit tile of the FP32 clip kernel (chosen by
SIMPROJ_TILED_DEPOSIT=1 when the context is created: each wave merges
pieces of one cell in a 64-cell LDS tile before one compensated grid
deposit) against the oracle on the FP32C 3D workloads, through the C ABI,
with the default kernel's tolerances (1e-5 of the coverage scale per cell,
1e-7 of the total).  The lattices put many pieces of neighbouring simplices
into one cell, which is where the tile merges; the soup and the needles
evict on nearly every piece."""
import numpy as np
import pytest

from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07720_amd import simproj  # noqa: E402
from test_gpu_parity import _needles, check, run  # noqa: E402  (the parity check itself)


@pytest.fixture(scope="module")
def tctx():
    mp = pytest.MonkeyPatch()
    mp.setenv("SIMPROJ_TILED_DEPOSIT", "1")
    c = simproj.Context(0)
    mp.undo()
    yield c
    c.close()


CASES = {
    "3d_zeldovich": lambda: synth.zeldovich_3d(n=16, grid=32, sigma_cells=1.5, seed=2),
    "3d_zeldovich_dense": lambda: synth.zeldovich_3d(n=16, grid=12, sigma_cells=0.5, seed=4),
    "3d_soup": lambda: synth.tet_soup(n_tets=20000, grid=256, seed=3),
    "3d_refined": lambda: synth.refined_3d(n=8, grid=48, sigma_cells=0.75, seed=5),
    "needles": lambda: _needles(400, 256, seed=12, lmin=20.0, lmax=90.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_deposit_matches_oracle(tctx, name):
    print(f"tiled deposit: {name}", flush=True)
    check(tctx, CASES[name](), "fp32c")


def test_tiled_deposit_matches_default_kernel(tctx):
    """Same problem through the tiled and the default kernel, several calls in
    a row on the tiled context: every call agrees with the default kernel to
    the compensated sums' rounding, cell by cell and in the total."""
    print("tiled deposit: against the default kernel", flush=True)
    prob = synth.as_float32(synth.zeldovich_3d(n=32, grid=64, sigma_cells=1.0, seed=21))
    dctx = simproj.Context(0)
    try:
        ref, ref_total = run(dctx, prob, "fp32c")
    finally:
        dctx.close()
    scale = float(np.abs(ref).max())
    for _ in range(3):
        got, total = run(tctx, prob, "fp32c")
        assert np.abs(got - ref).max() <= 1e-6 * scale
        assert abs(total - ref_total) <= 1e-7 * abs(ref_total)
