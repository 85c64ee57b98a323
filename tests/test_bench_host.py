"""Host-side pieces of bench.py (no GPU): the refusal of more than one GPU,
the exact total of the synthetic inputs, and the reading of the committed
counter summary."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1509_07720_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_exact_total_of_an_undisplaced_lattice_is_the_box_volume():
    # unit density on a lattice that tiles the unit box: total mass 1
    p = synth.zeldovich_3d(n=8, grid=16, sigma_cells=0.0, seed=1)
    p = dict(p, rho=np.ones_like(np.asarray(p["rho"])))
    assert abs(bench.exact_total(p) - 1.0) < 1e-12


def test_counter_summary_is_read_or_reported_stale():
    traffic, src = bench.clip_traffic()
    assert src in ("counters", "kernels changed since the counters were taken")
    if src == "counters":
        assert traffic > 0
    else:
        assert traffic is None
