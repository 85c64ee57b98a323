"""Test oracle for the exact simplex-to-grid projection -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The projection library never does.

* ``project``        -- plain FP64 brute-force projection (C, OpenMP), every
                        candidate cell of every simplex clipped and integrated
                        (``simproj_oracle.c``).
* ``exact``          -- the same quantity in exact rational arithmetic by a
                        different construction (sequential clipping of the
                        simplex by the cell's half-spaces with cap facets).
* ``franklin``       -- the paper's first-order corner sum (Section 3.1), used
                        to cross-check the piece integrals.
* ``mc``             -- Monte Carlo deposit, the paper's particle-sampling
                        check (Section 5.2).
* ``vertex_density`` -- the per-vertex density estimate (Section 4).
* ``amr``            -- the two-stage projection: exact onto an adaptive
                        grid refined region by region until no cell is larger
                        than the smallest height of a simplex meeting it,
                        then donor cell onto the uniform grid (Section 4).
* ``work``           -- work counts of the slab recursion (intersection
                        points, classifications, fan tetrahedra) that price
                        the projection's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simproj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (portable x86-64 code, no FMA
    contraction so that the TwoSum accumulators stay exact)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("xyz", ctypes.c_void_p),
        ("n_vert", ctypes.c_int64),
        ("simp", ctypes.c_void_p),
        ("n_simplex", ctypes.c_int64),
        ("rho", ctypes.c_void_p),
        ("rho_per_corner", ctypes.c_int),
        ("origin", ctypes.c_double * 3),
        ("extent", ctypes.c_double * 3),
        ("dims", ctypes.c_int64 * 3),
        ("periodic", ctypes.c_int * 3),
        ("cell_mask", ctypes.c_void_p),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("n_zero_volume", ctypes.c_int64),
        ("n_bad_span", ctypes.c_int64),
        ("n_bad_index", ctypes.c_int64),
        ("n_candidates", ctypes.c_int64),
        ("n_pieces", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.or_project.restype = ctypes.c_int
        lib.or_project.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Stats), ctypes.c_int]
        lib.or_simplex_mass.restype = None
        lib.or_simplex_mass.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _marshal(prob, cell_mask=None):
    dim = int(prob["dim"])
    xyz = np.ascontiguousarray(prob["xyz"], dtype=np.float64).reshape(-1, dim)
    simp = np.ascontiguousarray(prob["simplices"], dtype=np.int32).reshape(-1, dim + 1)
    rho = np.ascontiguousarray(prob["rho"], dtype=np.float64)
    P = _Problem()
    P.dim = dim
    P.xyz = xyz.ctypes.data
    P.n_vert = xyz.shape[0]
    P.simp = simp.ctypes.data
    P.n_simplex = simp.shape[0]
    P.rho = rho.ctypes.data
    P.rho_per_corner = int(bool(prob["rho_per_corner"]))
    for d in range(3):
        P.origin[d] = float(prob["origin"][d])
        P.extent[d] = float(prob["extent"][d])
        P.dims[d] = int(prob["dims"][d])
        P.periodic[d] = int(bool(prob["periodic"][d]))
    keep = [xyz, simp, rho]
    if cell_mask is not None:
        cm = np.ascontiguousarray(cell_mask, dtype=np.uint8)
        keep.append(cm)
        P.cell_mask = cm.ctypes.data
    return P, keep


def grid_shape(prob):
    dims = [int(v) for v in prob["dims"]]
    return (dims[2], dims[1], dims[0]) if int(prob["dim"]) == 3 else (dims[1], dims[0])


def project(prob, nthreads: Optional[int] = None, cell_mask=None, coverage: bool = True,
            per_simplex: bool = False) -> dict:
    """FP64 brute-force projection.  Returns dict(mass=grid of mass per cell
    (C order, x fastest), cov=coverage scale per cell, simplex_mass,
    simplex_moment, stats)."""
    lib = _load()
    P, keep = _marshal(prob, cell_mask)
    shape = grid_shape(prob)
    mass = np.zeros(shape, dtype=np.float64)
    cov = np.zeros(shape, dtype=np.float64) if coverage else None
    ns = int(P.n_simplex)
    sm = np.zeros(ns, dtype=np.float64) if per_simplex else None
    smom = np.zeros((ns, 3), dtype=np.float64) if per_simplex else None
    st = _Stats()
    nt = int(nthreads or os.cpu_count() or 1)
    lib.or_project(ctypes.byref(P), _ptr(mass), _ptr(cov), _ptr(sm), _ptr(smom), ctypes.byref(st), nt)
    del keep
    stats = {k: int(getattr(st, k)) for k, _ in _Stats._fields_}
    return dict(mass=mass, cov=cov, simplex_mass=sm, simplex_moment=smom, stats=stats)


def simplex_mass(prob) -> np.ndarray:
    """|V_i| * mean_a rho_a per simplex (box units)."""
    lib = _load()
    P, keep = _marshal(prob)
    out = np.zeros(int(P.n_simplex), dtype=np.float64)
    lib.or_simplex_mass(ctypes.byref(P), _ptr(out))
    del keep
    return out


def cell_error(gpu_mass: np.ndarray, ref: dict) -> dict:
    """Error of a projected grid against the oracle: the per-cell error
    normalised by max(|R_j|, C_j) (C_j = coverage scale), the L1 error, and
    the relative error of the total mass."""
    R = ref["mass"]
    C = ref["cov"]
    g = np.asarray(gpu_mass, dtype=np.float64).reshape(R.shape)
    den = np.maximum(np.abs(R), C)
    diff = np.abs(g - R)
    touched = den > 0
    e_cell = float(np.max(diff[touched] / den[touched])) if touched.any() else 0.0
    stray = float(np.max(diff[~touched])) if (~touched).any() else 0.0
    tot_r = float(np.sum(R))
    return dict(e_cell=e_cell, stray=stray,
                l1=float(np.sum(diff) / max(np.sum(np.abs(R)), 1e-300)),
                e_mass=abs(float(np.sum(g)) - tot_r) / max(abs(tot_r), 1e-300))
