#!/usr/bin/env python3
"""Throughput of the exact simplex-to-grid projection on one MI355X.

Workload: the 10M-tetrahedron soup onto a 256^3 periodic grid (volumes
log-uniform over 1e-6..20 voxels, aspect ratios up to 50, float32 positions,
per-corner densities), generated synthetically from a fixed seed.  One step
is one complete sp_project_tets call: set-up and binning, single-cell
deposits, clip-integrate-deposit of every other simplex, and the hi+lo merge
with the FP64 total-mass reduction.  Inputs are resident in HBM before the
timed region.  The same workload is also timed in FP64 mode.

Also reported (not part of `value`): the per-vertex density estimate on the
64^3 lattice, the accuracy-controlled projection of cancelling densities
against plain FP32C and FP64, the two-stage (coarsened + donor-cell)
projection against the exact one, the other 3D configurations with their
roofline fractions, and the paper's corner-sum formulation against the
clipping projection.  The batched workload (64 Zel'dovich meshes of
1e4..2e6 tets onto grids of 32^3..256^3) is timed as one captured graph
launch for all 64 problems, after the autotuner has picked its launch
parameters, against 64 sequential calls, in FP32C and FP64 (--no-batch
skips it).

Prints one JSON line (see the "metric" field).  --gpus above 1 is refused:
this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
COUNTERS = os.path.join(ROOT, "profiles", "k_clip_soup10M_256_fp32c_counters.md")
MBENCH = os.path.join(ROOT, "paper_1509_07720_amd", "mbench")

# Algorithmic work per deposited piece: the slab recursion's counted
# intersection points (10 flops: a division and four fused multiply-adds),
# vertex classifications (2) and fan tetrahedra (20: a determinant and a
# density sum), per piece, on samples of each workload's recipe (stored by
# tests/golden/make_work_counts.py from the oracle's work-count model).
WORK_COUNTS = os.path.join(ROOT, "tests", "golden", "work_counts.json")
with open(WORK_COUNTS) as _f:
    _WORK = json.load(_f)
FLOPS_PER_PIECE = _WORK["tet-soup-to-256^3"]["flops_per_piece"]            # the soup
FLOPS_PER_PIECE_LATTICE = _WORK["zeldovich-64^3-lattice-to-128^3"]["flops_per_piece"]  # deformed lattices
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def exact_total(prob) -> float:
    from paper_1509_07720_amd import synth

    tot = 0.0
    S = prob["simplices"]
    R = prob["rho"]
    for s0 in range(0, S.shape[0], 1 << 21):
        sub = S[s0:s0 + (1 << 21)]
        P = synth.unwrapped_corners(prob["xyz"], sub, prob["extent"], prob["periodic"])
        r = R[s0:s0 + (1 << 21)] if prob["rho_per_corner"] else R[sub]
        tot += float(np.sum(np.abs(synth.signed_volumes(P)) * r.mean(axis=1)))
    return tot


def clip_traffic():
    """HBM bytes per clip launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs, each scaled by what the same counter read for a copy kernel
    of known size; None when the kernels changed since the counters were
    taken (or no summary exists)."""
    from paper_1509_07720_amd import build

    if not os.path.exists(COUNTERS):
        return None, "no counter summary"
    txt = open(COUNTERS).read()
    start = txt.find("```json")
    if start < 0:
        return None, "counter summary has no json block"
    rec = json.loads(txt[start + 7:txt.index("```", start + 7)])
    if rec["source_sha256"] != build.kernel_source_hash():
        return None, "kernels changed since the counters were taken"
    f_scale = rec["copy_bytes"] / (rec["copy_fetch_kib"] * 1024.0)
    w_scale = rec["copy_bytes"] / (rec["copy_write_kib"] * 1024.0)
    return rec["fetch_kib"] * 1024.0 * f_scale + rec["write_kib"] * 1024.0 * w_scale, "counters"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def atomic_peaks():
    """Measured rates of atomic adds to random cells of a 64 MiB grid (the
    deposit's pattern), from the mbench program: {"fp32c": compensated FP32
    pairs/s, "fp64": FP64 adds/s}, or None."""
    import subprocess

    if not os.path.exists(MBENCH):
        return None
    try:
        out = subprocess.run([MBENCH, "atomic", "64", "3"], capture_output=True, text=True, timeout=120)
    except (OSError, subprocess.TimeoutExpired):
        return None
    recs = [json.loads(l) for l in out.stdout.splitlines() if l.startswith("{")]
    peak = {}
    for prec, kind in (("fp32c", "returning+compensated"), ("fp64", "f64")):
        rates = [r["adds_per_s"] for r in recs if r.get("kind") == kind]
        peak[prec] = max(rates) if rates else None
    return peak


def batch_leg(ctx, steps, warmup, peaks=None):
    """The batched workload: one graph launch for 64 problems against 64
    sequential calls; FP32C and FP64.  The launch parameters are tuned on the
    64 problems first (sp_autotune with a cache file, timed separately; it
    times candidates as the batched launch).
    With the pieces counted one problem at a time (untimed), the batched
    launch's ALU, HBM and atomic fractions as for the other workloads, over
    the whole launch."""
    import tempfile

    import torch

    from paper_1509_07720_amd import simproj, synth

    t = time.time()
    probs = synth.batch_3d()
    log(f"batch: generated {len(probs)} problems in {time.time() - t:.1f}s")
    res = {"n_problems": len(probs), "n_simplex": int(sum(p["simplices"].shape[0] for p in probs)),
           "cells": int(sum(int(np.prod(p["dims"])) for p in probs))}
    dev = torch.device("cuda:0")
    for prec in ("fp32c", "fp64"):
        dt = torch.float32 if prec == "fp32c" else torch.float64
        code = simproj.SP_PREC_FP32C if prec == "fp32c" else simproj.SP_PREC_FP64
        keep, recs = [], []
        for p in probs:
            xyz = torch.tensor(np.asarray(p["xyz"]), dtype=dt, device=dev)
            simp = torch.tensor(np.asarray(p["simplices"]), dtype=torch.int32, device=dev)
            rho = torch.tensor(np.asarray(p["rho"]), dtype=dt, device=dev)
            out = torch.empty(tuple(reversed(list(p["dims"]))), dtype=dt, device=dev)
            keep.append((xyz, simp, rho, out))
            recs.append(simproj.make_problem(xyz, simp, rho, p["dims"], p["origin"], p["extent"], p["periodic"],
                                             p["rho_per_corner"], out, out_mass=True))
        stream = simproj._stream_ptr(None)

        def batched():
            simproj._check(simproj.sp_project_batch(ctx.handle, 3, recs, code, stream), "sp_project_batch")

        def sequential():
            for r in recs:
                simproj._check(simproj.sp_project_tets(ctx.handle, r, code, stream), "sp_project_tets")

        saved = ctx.tuning()
        cache = os.path.join(tempfile.mkdtemp(prefix="simproj-tune-"), "tune.txt")
        t = time.perf_counter()
        tuned = ctx.autotune(3, recs, precision=prec, cache_path=cache)
        tune_s = time.perf_counter() - t
        t = time.perf_counter()
        ctx.autotune(3, recs, precision=prec, cache_path=cache)  # found in the cache: no timing
        cached_s = time.perf_counter() - t
        log(f"batch {prec}: autotuned slab group {tuned[0]}, blocks/CU {tuned[1]}, item pieces {tuned[2]} "
            f"in {tune_s:.1f}s (cache hit {cached_s * 1e3:.1f} ms)")
        pieces = 0
        ctx.profile(2)
        for r in recs:
            simproj._check(simproj.sp_project_tets(ctx.handle, r, code, stream), "sp_project_tets")
            torch.cuda.synchronize()
            pieces += ctx.profile_read()["pieces"]
        ctx.profile(0)
        nb = 4 if prec == "fp32c" else 8
        algo = sum(k[0].numel() * nb + k[1].numel() * 4 + k[2].numel() * nb + k[3].numel() * 8
                   for k in keep)
        t = time.perf_counter()
        batched()  # first call: capture and instantiation
        torch.cuda.synchronize()
        first = time.perf_counter() - t
        row = {"first_call_ms": first * 1e3, "pieces": pieces,
               "autotune": {"slab_group": tuned[0], "blocks_per_cu": tuned[1], "item_pieces": tuned[2],
                            "tune_s": tune_s, "cache_hit_s": cached_s}}
        for name, fn in (("batched", batched), ("sequential", sequential)):
            # the batched launch with the tuned parameters; the calls one by
            # one with the default ones (the item size then follows each
            # call's own size)
            if name == "batched":
                ctx.set_tuning(*tuned)
            else:
                ctx.set_tuning(*saved)
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / steps
            row[name] = {"ms_per_step": sec * 1e3, "value": res["n_simplex"] / sec}
        sec = row["batched"]["ms_per_step"] * 1e-3
        peak_alu = PEAK_FP32_TFLOPS if prec == "fp32c" else PEAK_FP64_TFLOPS
        apk = peaks.get(prec) if peaks else None
        row["batched"].update({"alu_frac": pieces * FLOPS_PER_PIECE_LATTICE / sec / 1e12 / peak_alu,
                               "hbm_frac": algo / sec / 1e9 / PEAK_HBM_GBS,
                               "atomic_frac": pieces / sec / apk if apk else None})
        ctx.set_tuning(*saved)
        res[prec] = row
        log(f"batch {prec}: batched {row['batched']['ms_per_step']:.1f} ms, "
            f"sequential {row['sequential']['ms_per_step']:.1f} ms, first call {first * 1e3:.0f} ms")
        del keep, recs
        torch.cuda.empty_cache()
    res["unit"] = "simplices/s"
    return res


def vertex_density_leg(ctx, steps, warmup):
    """The per-vertex density estimate on the 64^3 Zel'dovich lattice (1.57M
    tets, 262,144 vertices), FP32 and FP64 inputs, equal masses."""
    import torch

    from paper_1509_07720_amd import synth

    prob = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2)
    dev = torch.device("cuda:0")
    simp = torch.tensor(np.asarray(prob["simplices"]), dtype=torch.int32, device=dev)
    ns, nv = simp.shape[0], prob["xyz"].shape[0]
    res = {"workload": "zeldovich-64^3-lattice", "n_simplex": ns, "n_vert": nv}
    for prec, dt, b in (("fp32c", torch.float32, 4), ("fp64", torch.float64, 8)):
        xyz = torch.tensor(np.asarray(prob["xyz"]), dtype=dt, device=dev)
        out = torch.empty(nv, dtype=dt, device=dev)
        for _ in range(warmup):
            ctx.vertex_density(xyz, simp, None, 1.0 / ns, precision=prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.vertex_density(xyz, simp, None, 1.0 / ns, precision=prec, out=out)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        # connectivity once, each corner's coordinates, vertex output, the
        # two FP64 accumulators per vertex (zeroed, then read)
        algo = ns * 16 + ns * 4 * 3 * b + nv * b + nv * 16 * 2
        res[prec] = {"ms": sec * 1e3, "simplices_per_s": ns / sec, "algorithmic_bytes": algo,
                     "hbm_gbs": algo / sec / 1e9, "hbm_frac": algo / sec / 1e9 / PEAK_HBM_GBS,
                     "fp64_atomics_per_s": ns * 4 * 2 / sec}
        log(f"vertex density {prec}: {sec * 1e3:.3f} ms ({ns / sec:.3e} tets/s)")
    return res


def accuracy_leg(ctx, steps, warmup):
    """Per-voxel accuracy control on cancelling densities: the 64^3 Zel'dovich
    sheet plus, over half of it, a copy displaced by 1e-4 of its displacement
    with the opposite density, onto 128^3.  Times the plain FP32C call, the
    accuracy-controlled call (A = 12, W = 10) and the plain FP64 call."""
    import torch

    from paper_1509_07720_amd import synth

    a = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=21)
    b = synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5 * (1.0 + 1e-4), seed=21)
    nb = b["simplices"].shape[0] // 2
    nv = a["xyz"].shape[0]
    xyz = np.vstack([a["xyz"], b["xyz"]])
    simp = np.vstack([a["simplices"], b["simplices"][:nb] + nv]).astype(np.int32)
    rho = np.concatenate([a["rho"], -b["rho"]])
    dev = torch.device("cuda:0")
    s = torch.tensor(simp, dtype=torch.int32, device=dev)
    x32, r32 = torch.tensor(xyz, dtype=torch.float32, device=dev), torch.tensor(rho, dtype=torch.float32, device=dev)
    x64, r64 = x32.double(), r32.double()
    dims = [128] * 3
    res = {"workload": "cancelling-zeldovich-sheets-64^3(+half)-to-128^3", "n_simplex": int(simp.shape[0]),
           "accurate_bits": 12, "wrong_bits": 10}
    runs = {
        "fp32c": lambda: ctx.project(x32, s, r32, dims, precision="fp32c", out_mass=True),
        "accurate": lambda: ctx.project_accurate(x32, s, r32, dims, accurate_bits=12, wrong_bits=10, out_mass=True),
        "fp64": lambda: ctx.project(x64, s, r64, dims, precision="fp64", out_mass=True),
    }
    for name, fn in runs.items():
        for _ in range(warmup):
            out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        res[name] = {"ms": sec * 1e3, "simplices_per_s": simp.shape[0] / sec}
        if name == "accurate":
            res[name]["flagged_cells"], res[name]["reprojected_simplices"] = int(out[2]), int(out[3])
        log(f"accuracy leg {name}: {sec * 1e3:.2f} ms")
    return res


def amr_leg(ctx, steps, warmup):
    """Two-stage projection against the exact one where simplices are large
    against the cells: the 32^3 Zel'dovich lattice (196,608 tets of ~8 cells)
    onto 256^3, FP32C, max_level 3.  Reports both times, the simplices per
    level and the L1 difference of the two grids relative to the total."""
    import torch

    from paper_1509_07720_amd import synth

    prob = synth.zeldovich_3d(n=32, grid=256, sigma_cells=1.5, seed=44)
    dev = torch.device("cuda:0")
    x = torch.tensor(prob["xyz"], dtype=torch.float32, device=dev)
    s = torch.tensor(prob["simplices"], dtype=torch.int32, device=dev)
    r = torch.tensor(prob["rho"], dtype=torch.float32, device=dev)
    dims = [256] * 3
    res = {"workload": "zeldovich-32^3-lattice-to-256^3", "n_simplex": int(s.shape[0]), "max_level": 3}
    outs = {}
    for name in ("exact", "amr"):
        def fn():
            if name == "exact":
                return ctx.project(x, s, r, dims, precision="fp32c", out_mass=True)[0], None
            g, _, counts = ctx.project_amr(x, s, r, dims, 3, precision="fp32c", out_mass=True)
            return g, counts
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g, counts = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        outs[name] = g
        res[name] = {"ms": sec * 1e3, "simplices_per_s": s.shape[0] / sec}
        if counts is not None:
            res[name]["simplices_per_level"] = counts
        log(f"amr leg {name}: {sec * 1e3:.2f} ms")
    res["l1_difference_rel"] = float((outs["amr"].double() - outs["exact"].double()).abs().sum() /
                                     outs["exact"].double().abs().sum())
    return res


_REFINED = []


def refined_mesh():
    """The two-level refined 128^3 lattice onto 512^3 (50.3M tets), generated
    once per run (about a minute of CPU)."""
    from paper_1509_07720_amd import synth

    if not _REFINED:
        _REFINED.append(synth.refined_3d(n=128, grid=512, sigma_cells=4.0, seed=5))
    return _REFINED[0]


def configs_leg(ctx, steps, warmup, peaks, refined=True):
    """The other 3D configurations, each in FP32C and FP64: the 64^3
    Zel'dovich lattice onto 128^3 (1.57M tets, per-vertex densities) and the
    two-level refined 128^3 lattice onto 512^3 (50.3M tets, heavy shell
    crossing).  Per precision: time per call, pieces, error of the total mass,
    and the three fractions -- ALU (pieces x the lattice's counted flops per
    piece over the clip kernel's time against the vector peak of that
    precision), HBM (inputs read once plus the output grids written once,
    over the call) and atomic (deposits over the clip kernel's time against
    the measured rate)."""
    import torch

    from paper_1509_07720_amd import synth

    work = [("zeldovich-64^3-lattice-to-128^3", lambda: synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2))]
    if refined:
        work.append(("refined-128^3-kuhn-2-levels-to-512^3", refined_mesh))
    dev = torch.device("cuda:0")
    res = {}
    for name, gen in work:
        t = time.time()
        prob = synth.as_float32(gen())
        exact = exact_total(prob)
        log(f"config {name}: generated in {time.time() - t:.1f}s")
        dims = [int(d) for d in prob["dims"]]
        per_corner = bool(prob["rho_per_corner"])
        simp = torch.from_numpy(np.ascontiguousarray(prob["simplices"], dtype=np.int32)).to(dev)
        row = {"n_simplex": int(simp.shape[0]), "grid": dims, "rho": "per-corner" if per_corner else "per-vertex"}
        for prec, dt, nb, peak_alu in (("fp32c", torch.float32, 4, PEAK_FP32_TFLOPS),
                                       ("fp64", torch.float64, 8, PEAK_FP64_TFLOPS)):
            xyz = torch.from_numpy(np.asarray(prob["xyz"])).to(dev, dt).contiguous()
            rho = torch.from_numpy(np.asarray(prob["rho"])).to(dev, dt).contiguous()
            out = torch.empty(tuple(reversed(dims)), dtype=dt, device=dev)

            def call():
                return ctx.project(xyz, simp, rho, dims, precision=prec, rho_per_corner=per_corner, out=out,
                                   out_mass=True)

            ctx.profile(2)
            call()
            pieces = ctx.profile_read()["pieces"]
            ctx.profile(0)
            for _ in range(warmup):
                call()
            torch.cuda.synchronize()
            ctx.profile(1)
            t0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            prof = ctx.profile_read()
            ctx.profile(0)
            _, total = call()
            assert ctx.sync_status() == 0
            clip_s = prof["ms_clip"] / max(prof["calls"], 1) * 1e-3
            algo = xyz.numel() * nb + simp.numel() * 4 + rho.numel() * nb + out.numel() * (8 if prec == "fp32c" else nb)
            dep_rate = pieces / clip_s
            apk = peaks.get(prec) if peaks else None
            row[prec] = {"ms_per_call": sec * 1e3, "simplices_per_s": simp.shape[0] / sec, "clip_ms": clip_s * 1e3,
                         "pieces": pieces, "mass_rel_err": abs(float(total.cpu()[0]) - exact) / exact,
                         "alu_frac": pieces * FLOPS_PER_PIECE_LATTICE / clip_s / 1e12 / peak_alu,
                         "hbm_frac": algo / sec / 1e9 / PEAK_HBM_GBS,
                         "atomic_frac": dep_rate / apk if apk else None, "deposits_per_s": dep_rate}
            log(f"config {name} {prec}: {sec * 1e3:.2f} ms/call, {pieces} pieces")
            del xyz, rho, out
        res[name] = row
        del simp, prob
        torch.cuda.empty_cache()
    return res


def tris_leg(ctx, steps, warmup):
    """2D: the two-sine triangle lattice (1024^2 vertices, 2.1M triangles,
    per-vertex densities) onto 2048^2, FP32C and FP64 (sp_project_tris):
    time per call, pieces and the error of the total mass."""
    import torch

    from paper_1509_07720_amd import synth

    prob = synth.as_float32(synth.two_sine_2d(n=1024, grid=2048, seed=1))
    dims = [int(d) for d in prob["dims"][:2]]
    exact = float(exact_total_2d(prob))
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(prob["simplices"], dtype=np.int32)).to(dev)
    res = {"workload": "two-sine-1024^2-lattice-to-2048^2", "n_simplex": int(s.shape[0]), "grid": dims}
    for prec, dt in (("fp32c", torch.float32), ("fp64", torch.float64)):
        xyz = torch.from_numpy(np.ascontiguousarray(prob["xyz"])).to(dev, dt)
        rho = torch.from_numpy(np.ascontiguousarray(prob["rho"])).to(dev, dt)
        out = torch.empty(tuple(reversed(dims)), dtype=dt, device=dev)

        def call():
            return ctx.project(xyz, s, rho, dims, precision=prec, out=out, out_mass=True)

        ctx.profile(2)
        call()
        pieces = ctx.profile_read()["pieces"]
        ctx.profile(0)
        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        _, total = call()
        assert ctx.sync_status() == 0
        res[prec] = {"ms_per_call": sec * 1e3, "simplices_per_s": s.shape[0] / sec, "pieces": pieces,
                     "mass_rel_err": abs(float(total.cpu()[0]) - exact) / exact}
        log(f"2d {prec}: {sec * 1e3:.2f} ms/call, {pieces} pieces")
    return res


def exact_total_2d(prob) -> float:
    """Exact FP64 total of a 2D problem: sum of |area| x mean corner density."""
    from paper_1509_07720_amd import synth

    P = synth.unwrapped_corners(np.asarray(prob["xyz"]), np.asarray(prob["simplices"]), np.asarray(prob["extent"]),
                                prob["periodic"])
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    R = np.asarray(prob["rho"])
    r = R if prob["rho_per_corner"] else R[np.asarray(prob["simplices"])]
    return float(np.sum(area * r.mean(axis=1)))


def corner_leg(ctx, steps, warmup):
    """The paper's corner-sum formulation (sp_project_tets_corners, FP64),
    also with the fused facet contributions (sp_project_tets_corners_fused),
    against the clipping projection in FP64 and FP32C, on the 64^3
    Zel'dovich lattice onto 128^3 and on every 64th tetrahedron of the
    two-level refined 128^3 lattice onto 512^3 (786,432 tets): time per call
    and the largest cell difference from the FP64 clipping result relative
    to the largest cell."""
    import torch

    from paper_1509_07720_amd import synth

    work = [("zeldovich-64^3-lattice-to-128^3", lambda: synth.zeldovich_3d(n=64, grid=128, sigma_cells=1.5, seed=2)),
            ("refined-128^3-every-64th-tet-to-512^3",
             lambda: synth.subset(refined_mesh(), 64))]
    dev = torch.device("cuda:0")
    res = {}
    for name, gen in work:
        prob = gen()
        dims = [int(d) for d in prob["dims"]]
        pc = bool(prob["rho_per_corner"])
        s = torch.from_numpy(np.ascontiguousarray(prob["simplices"], dtype=np.int32)).to(dev)
        x64 = torch.from_numpy(np.ascontiguousarray(prob["xyz"], dtype=np.float64)).to(dev)
        r64 = torch.from_numpy(np.ascontiguousarray(prob["rho"], dtype=np.float64)).to(dev)
        x32, r32 = x64.float(), r64.float()
        runs = {
            "corners_fp64": lambda: ctx.project_corners(x64, s, r64, dims, rho_per_corner=pc, out_mass=True),
            "corners_fused_fp64": lambda: ctx.project_corners(x64, s, r64, dims, rho_per_corner=pc, out_mass=True,
                                                              fused=True),
            "clip_fp64": lambda: ctx.project(x64, s, r64, dims, precision="fp64", rho_per_corner=pc, out_mass=True),
            "clip_fp32c": lambda: ctx.project(x32, s, r32, dims, precision="fp32c", rho_per_corner=pc, out_mass=True),
        }
        row = {"n_simplex": int(s.shape[0]), "grid": dims}
        grids = {}
        for k, fn in runs.items():
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g, _ = fn()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            st = ctx.sync_status()
            grids[k] = g.double()
            row[k] = {"ms": sec * 1e3, "simplices_per_s": s.shape[0] / sec, "status": int(st)}
            log(f"corner leg {name} {k}: {sec * 1e3:.2f} ms (status {st})")
        ref = grids["clip_fp64"]
        scale = float(ref.abs().max())
        for k in ("corners_fp64", "corners_fused_fp64", "clip_fp32c"):
            row[k]["max_cell_diff_rel"] = float((grids[k] - ref).abs().max()) / scale
        res[name] = row
        del grids, s, x64, r64, x32, r32
        torch.cuda.empty_cache()
    return res


def time_steps(ctx, args_dev, steps, warmup, prec):
    import torch

    xyz, simp, rho, out, total, kw = args_dev
    for _ in range(warmup):
        ctx.project(xyz, simp, rho, kw["dims"], precision=prec, rho_per_corner=True, out=out, out_mass=True)
    torch.cuda.synchronize()
    ctx.profile(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.project(xyz, simp, rho, kw["dims"], precision=prec, rho_per_corner=True, out=out, out_mass=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(0)
    return (t1 - t0) / steps, prof


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-tets", type=int, default=10_000_000)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=200_000, help="tets projected by the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched workload")
    ap.add_argument("--no-atomic-peak", action="store_true", help="skip the atomic-rate measurement (mbench)")
    ap.add_argument("--no-vertex-density", action="store_true", help="skip the per-vertex density leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy-control leg")
    ap.add_argument("--no-amr", action="store_true", help="skip the two-stage projection leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the other-configuration leg")
    ap.add_argument("--no-refined", action="store_true", help="other configurations without the 50M-tet one")
    ap.add_argument("--no-corners", action="store_true", help="skip the corner-sum comparison leg")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D (triangle) leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        return 2

    # measured in a child process before this one touches the GPU
    peaks = None if args.no_atomic_peak else atomic_peaks()
    apeak = peaks.get("fp32c") if peaks else None

    import torch

    from paper_1509_07720_amd import simproj, synth

    t = time.time()
    prob = synth.tet_soup(n_tets=args.n_tets, grid=args.grid, seed=3)
    log(f"generated {args.n_tets} tets in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    n = args.n_tets
    dims = [args.grid] * 3
    xyz32 = torch.from_numpy(np.ascontiguousarray(prob["xyz"], dtype=np.float32)).to(dev)
    simp = torch.from_numpy(np.ascontiguousarray(prob["simplices"], dtype=np.int32)).to(dev)
    rho32 = torch.from_numpy(np.ascontiguousarray(prob["rho"], dtype=np.float32)).to(dev)
    out32 = torch.empty(tuple(dims), dtype=torch.float32, device=dev)
    ctx = simproj.Context(0)
    exact = exact_total(synth.as_float32(prob))
    log("inputs resident; timing FP32C")

    # piece count: one extra call with counting on, outside the timed region
    ctx.profile(2)
    ctx.project(xyz32, simp, rho32, dims, precision="fp32c", rho_per_corner=True, out=out32, out_mass=True)
    pieces = ctx.profile_read()["pieces"]
    ctx.profile(0)

    sec, prof = time_steps(ctx, (xyz32, simp, rho32, out32, None, dict(dims=dims)), args.steps, args.warmup, "fp32c")
    g, total = ctx.project(xyz32, simp, rho32, dims, precision="fp32c", rho_per_corner=True, out=out32,
                           out_mass=True)
    assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
    mass_err = abs(float(total.cpu()[0]) - exact) / exact
    value = n / sec
    clip_ms = prof["ms_clip"] / max(prof["calls"], 1)
    achieved = pieces * FLOPS_PER_PIECE / (clip_ms * 1e-3) / 1e12
    in_bytes = xyz32.numel() * 4 + simp.numel() * 4 + rho32.numel() * 4
    grid_bytes = 2 * out32.numel() * 4  # hi and lo grids
    hbm_gbs = (in_bytes + grid_bytes) / sec / 1e9
    log(f"fp32c: {sec * 1e3:.3f} ms/step, {value:.3e} tets/s, clip {clip_ms:.3f} ms, pieces {pieces}, "
        f"mass err {mass_err:.2e}")
    stages = {k: round(v / max(prof["calls"], 1), 4) for k, v in prof.items() if k.startswith("ms_")}

    fp64 = None
    if not args.no_fp64:
        xyz64 = xyz32.double()
        rho64 = rho32.double()
        out64 = torch.empty(tuple(dims), dtype=torch.float64, device=dev)
        sec64, prof64 = time_steps(ctx, (xyz64, simp, rho64, out64, None, dict(dims=dims)), args.steps,
                                   args.warmup, "fp64")
        _, total64 = ctx.project(xyz64, simp, rho64, dims, precision="fp64", rho_per_corner=True, out=out64,
                                 out_mass=True)
        assert ctx.sync_status() == simproj.SP_OK, simproj.sp_last_error()
        err64 = abs(float(total64.cpu()[0]) - exact) / exact
        clip64_s = prof64["ms_clip"] / max(prof64["calls"], 1) * 1e-3
        apk64 = peaks.get("fp64") if peaks else None
        fp64 = {"value": n / sec64, "ms_per_step": sec64 * 1e3, "mass_rel_err": err64, "clip_ms": clip64_s * 1e3,
                "hbm_gbs": (xyz64.numel() * 8 + simp.numel() * 4 + rho64.numel() * 8 + out64.numel() * 8) / sec64 / 1e9,
                "alu_frac": pieces * FLOPS_PER_PIECE / clip64_s / 1e12 / PEAK_FP64_TFLOPS,
                "atomic_frac": pieces / clip64_s / apk64 if apk64 else None}
        log(f"fp64: {sec64 * 1e3:.3f} ms/step, {n / sec64:.3e} tets/s, mass err {err64:.2e}")
        del xyz64, rho64, out64

    batch = None if args.no_batch else batch_leg(ctx, max(1, min(args.steps, 3)), 1, peaks)
    vdens = None if args.no_vertex_density else vertex_density_leg(ctx, max(1, args.steps), 1)
    accur = None if args.no_accuracy else accuracy_leg(ctx, max(1, min(args.steps, 5)), 1)
    amr = None if args.no_amr else amr_leg(ctx, max(1, min(args.steps, 5)), 1)
    configs = None if args.no_configs else configs_leg(ctx, max(1, min(args.steps, 3)), 1, peaks,
                                                      refined=not args.no_refined)
    corners = None if args.no_corners else corner_leg(ctx, max(1, min(args.steps, 3)), 1)
    tris = None if args.no_2d else tris_leg(ctx, max(1, min(args.steps, 3)), 1)

    traffic, traffic_src = clip_traffic()
    deposits_per_s = pieces / (clip_ms * 1e-3)
    log(f"traffic: {traffic} ({traffic_src}); atomic peaks {peaks}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        k = min(args.cpu_sample, n)
        sub = dict(synth.as_float32(prob), simplices=np.ascontiguousarray(prob["simplices"][:k]),
                   rho=np.ascontiguousarray(np.asarray(prob["rho"], dtype=np.float32)[:k].astype(np.float64)))
        threads = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS"):
            threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
        t = time.perf_counter()
        oracle.project(sub, nthreads=threads, coverage=False)
        dt = time.perf_counter() - t
        # one thread, on a tenth of the sample
        k1 = max(1, k // 10)
        sub1 = dict(sub, simplices=np.ascontiguousarray(sub["simplices"][:k1]), rho=np.ascontiguousarray(sub["rho"][:k1]))
        t = time.perf_counter()
        oracle.project(sub1, nthreads=1, coverage=False)
        dt1 = time.perf_counter() - t
        cpu = {"value": k / dt, "unit": "simplices/s", "cores": threads, "kind": "oracle",
               "sample": f"first {k} tets of the workload, FP64 brute-force clip of every candidate cell, "
                         f"{dt:.1f} s wall on {threads} threads",
               "single_thread_value": k1 / dt1, "cpu_model": cpu_model()}
        log(f"cpu oracle: {k / dt:.3e} tets/s on {threads} threads ({dt:.1f}s), {k1 / dt1:.3e} on one")

    line = {
        "metric": "simplices projected/sec + HBM GB/s at 10M tets->256^3, FP32 vs FP64 at stated error",
        "value": value,
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"tet-soup-{n}-to-{args.grid}^3", "n_simplex": n, "grid": dims,
                   "precision": "fp32c", "rho": "per-corner", "seed": 3},
        "hbm_gbs": hbm_gbs,
        "mass_rel_err": mass_err,
        "pieces": pieces,
        "stages_ms": stages,
        "fp64": fp64,
        "roofline": {"bound": "alu", "kernel": "k_clip", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_source": traffic_src, "flops_per_piece": FLOPS_PER_PIECE, "clip_ms": clip_ms,
                     "hbm_frac_step": hbm_gbs / PEAK_HBM_GBS,
                     "atomic": {"deposits_per_s": deposits_per_s, "measured_peak_per_s": apeak,
                                "frac": deposits_per_s / apeak if apeak else None}},
        "batch": batch,
        "vertex_density": vdens,
        "accuracy_control": accur,
        "two_stage": amr,
        "configs": configs,
        "corner_sums": corners,
        "triangles_2d": tris,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
