"""Write work_counts.json: the slab recursion's work counts (oracle/work.py:
intersection points, classifications, fan tetrahedra, and the flops they are
priced at) on samples of the benchmark workloads' recipes.  Calls only the
oracle and the input generators.  Run from the repository root:

    python tests/golden/make_work_counts.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import work  # noqa: E402
from paper_1509_07720_amd import synth  # noqa: E402

SAMPLES = {
    # the 10M-tetrahedron soup onto 256^3: the same recipe, 4000 tetrahedra
    "tet-soup-to-256^3": lambda: synth.tet_soup(n_tets=4000, grid=256, seed=3),
    # the 64^3 Zel'dovich lattice onto 128^3: every 64th tetrahedron
    "zeldovich-64^3-lattice-to-128^3": lambda: synth.subset(synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5,
                                                                               seed=2), 64),
}


def main():
    out = {"model": "oracle/work.py slab recursion",
           "flops": {"intersection": work.FLOPS_INT, "classification": work.FLOPS_CLS, "fan": work.FLOPS_FAN}}
    for name, make in SAMPLES.items():
        t = time.time()
        prob = make()
        c = work.counts(work.cell_corners(prob))
        c["n_simplex"] = int(prob["simplices"].shape[0])
        out[name] = c
        print(name, c, "%.1fs" % (time.time() - t))
    with open(os.path.join(HERE, "work_counts.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
