"""Process exit with live contexts: the module-level helpers keep a default
context per device, closed at interpreter exit; a Context the caller never
closed is released by the process end.  Each case runs in a child process
that ends normally (no os._exit), and must exit with status 0 after printing
its result, which is checked against the FP64 oracle in the parent."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1509_07720_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import torch
from paper_1509_07720_amd import simproj, synth
prob = synth.as_float32(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=2))
dev = torch.device("cuda:0")
xyz = torch.tensor(prob["xyz"], dtype=torch.float32, device=dev)
simp = torch.tensor(prob["simplices"], dtype=torch.int32, device=dev)
rho = torch.tensor(prob["rho"], dtype=torch.float32, device=dev)
mode = {mode!r}
if mode == "default":
    grid, total = simproj.project(xyz, simp, rho, prob["dims"], out_mass=True)
else:
    ctx = simproj.Context(0)  # never closed by the caller
    grid, total = ctx.project(xyz, simp, rho, prob["dims"], out_mass=True)
torch.cuda.synchronize()
print("TOTAL %.17g" % float(total.cpu()[0]), flush=True)
"""


@pytest.mark.parametrize("mode", ["default", "unclosed"])
def test_child_process_exits_cleanly(mode):
    print(f"teardown child: mode {mode}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, mode=mode)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    line = [l for l in r.stdout.splitlines() if l.startswith("TOTAL ")]
    assert line, r.stdout
    prob = synth.as_float32(synth.zeldovich_3d(n=8, grid=16, sigma_cells=1.0, seed=2))
    want = float(oracle.project(prob)["mass"].sum())
    assert abs(float(line[0].split()[1]) - want) <= 1e-7 * abs(want)
