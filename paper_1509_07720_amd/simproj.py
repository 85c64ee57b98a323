"""Python binding of libsimproj (include/simproj.h).

The functions ``sp_create`` ... ``sp_last_error`` mirror the C ABI one to one
and only marshal arguments; every step of the projection runs in the HIP
kernels of ``libsimproj.so``.  PyTorch provides device memory and streams.
``project`` is a convenience wrapper that allocates the output grid.

Importing this module fails loudly when the library has not been built: there
is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsimproj.so")

SP_OK = 0
SP_E_INVALID_ARG = 1
SP_E_OUT_OF_RANGE = 2
SP_E_NONFINITE = 3
SP_E_PERIODIC_SPAN = 4
SP_E_NO_MEMORY = 5
SP_E_DEVICE = 6
SP_E_UNSUPPORTED = 7
SP_E_INTERNAL = 8

SP_PREC_FP64 = 0
SP_PREC_FP32C = 1

SP_PERIODIC_X = 1
SP_PERIODIC_Y = 2
SP_PERIODIC_Z = 4
SP_RHO_PER_CORNER = 8
SP_OUT_MASS = 16
SP_ACCUMULATE = 32
SP_VALIDATE = 64

STATUS_NAMES = {0: "SP_OK", 1: "SP_E_INVALID_ARG", 2: "SP_E_OUT_OF_RANGE", 3: "SP_E_NONFINITE",
                4: "SP_E_PERIODIC_SPAN", 5: "SP_E_NO_MEMORY", 6: "SP_E_DEVICE", 7: "SP_E_UNSUPPORTED",
                8: "SP_E_INTERNAL"}


class sp_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("extent", ctypes.c_double * 3),
                ("dims", ctypes.c_int32 * 3), ("flags", ctypes.c_uint32)]


class sp_problem(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n_vert", ctypes.c_int64), ("simplices", ctypes.c_void_p),
                ("n_simplex", ctypes.c_int64), ("rho", ctypes.c_void_p), ("grid", sp_grid),
                ("out", ctypes.c_void_p), ("out_lo", ctypes.c_void_p), ("total_mass", ctypes.c_void_p)]


class sp_profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int), ("ms_call", ctypes.c_double), ("ms_fill", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_bin", ctypes.c_double), ("ms_clip", ctypes.c_double),
                ("ms_clip_retry", ctypes.c_double), ("ms_finalize", ctypes.c_double),
                ("pieces", ctypes.c_longlong), ("items", ctypes.c_longlong), ("clip_blocks", ctypes.c_int)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)
_V = ctypes.c_void_p
_lib.sp_create.argtypes = [ctypes.c_int, ctypes.POINTER(_V)]
_lib.sp_create.restype = ctypes.c_int
_lib.sp_destroy.argtypes = [_V]
_lib.sp_destroy.restype = None
for _name in ("sp_project_tets", "sp_project_tris", "sp_project_tets_noalloc"):
    getattr(_lib, _name).argtypes = [_V, ctypes.POINTER(sp_problem), ctypes.c_int, _V]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.sp_project_tets_accurate.argtypes = [_V, ctypes.POINTER(sp_problem), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int64), _V]
_lib.sp_project_tets_accurate.restype = ctypes.c_int
_lib.sp_project_tets_amr.argtypes = [_V, ctypes.POINTER(sp_problem), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int64), _V]
_lib.sp_project_tets_amr.restype = ctypes.c_int
_lib.sp_project_tets_corners.argtypes = [_V, ctypes.POINTER(sp_problem), _V]
_lib.sp_project_tets_corners.restype = ctypes.c_int
_lib.sp_project_tets_corners_fused.argtypes = [_V, ctypes.POINTER(sp_problem), _V]
_lib.sp_project_tets_corners_fused.restype = ctypes.c_int
_lib.sp_project_batch.argtypes = [_V, ctypes.c_int, ctypes.POINTER(sp_problem), ctypes.c_int, ctypes.c_int, _V]
_lib.sp_project_batch.restype = ctypes.c_int
_lib.sp_sync_status.argtypes = [_V, _V]
_lib.sp_sync_status.restype = ctypes.c_int
_lib.sp_autotune.argtypes = [_V, ctypes.c_int, ctypes.POINTER(sp_problem), ctypes.c_int, ctypes.c_int,
                             ctypes.c_char_p]
_lib.sp_autotune.restype = ctypes.c_int
_lib.sp_tuning_read.argtypes = [_V, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
_lib.sp_tuning_read.restype = ctypes.c_int
_lib.sp_tuning_set.argtypes = [_V, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.sp_tuning_set.restype = ctypes.c_int
_lib.sp_vertex_density.argtypes = [_V, ctypes.c_int, _V, ctypes.c_int64, _V, ctypes.c_int64, _V, ctypes.c_double,
                                   ctypes.POINTER(sp_grid), _V, ctypes.c_int, _V]
_lib.sp_vertex_density.restype = ctypes.c_int
_lib.sp_profile_enable.argtypes = [_V, ctypes.c_int]
_lib.sp_profile_enable.restype = ctypes.c_int
_lib.sp_profile_read.argtypes = [_V, ctypes.POINTER(sp_profile)]
_lib.sp_profile_read.restype = ctypes.c_int
_lib.sp_last_error.argtypes = [_V]
_lib.sp_last_error.restype = ctypes.c_char_p


class SimprojError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.sp_last_error(None).decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(st: int, where: str) -> int:
    if st != SP_OK:
        raise SimprojError(st, where)
    return st


# --------------------------------------------------------------------------
# one-to-one wrappers (return the status code; the raising helpers are below)

def sp_create(device: int = 0):
    h = _V()
    st = _lib.sp_create(int(device), ctypes.byref(h))
    return st, h


def sp_destroy(ctx) -> None:
    _lib.sp_destroy(ctx)


def sp_project_tets(ctx, prob: sp_problem, prec: int, stream=None) -> int:
    return _lib.sp_project_tets(ctx, ctypes.byref(prob), int(prec), stream)


def sp_project_tets_noalloc(ctx, prob: sp_problem, prec: int, stream=None) -> int:
    return _lib.sp_project_tets_noalloc(ctx, ctypes.byref(prob), int(prec), stream)


def sp_project_tris(ctx, prob: sp_problem, prec: int, stream=None) -> int:
    return _lib.sp_project_tris(ctx, ctypes.byref(prob), int(prec), stream)


def sp_project_tets_accurate(ctx, prob: sp_problem, accurate_bits: int, wrong_bits: int, stream=None):
    counts = (ctypes.c_int64 * 2)()
    st = _lib.sp_project_tets_accurate(ctx, ctypes.byref(prob), int(accurate_bits), int(wrong_bits), counts, stream)
    return st, counts[0], counts[1]


def sp_project_tets_corners(ctx, prob: sp_problem, stream=None) -> int:
    return _lib.sp_project_tets_corners(ctx, ctypes.byref(prob), stream)


def sp_project_tets_corners_fused(ctx, prob: sp_problem, stream=None) -> int:
    return _lib.sp_project_tets_corners_fused(ctx, ctypes.byref(prob), stream)


def sp_project_tets_amr(ctx, prob: sp_problem, prec: int, max_level: int, stream=None):
    counts = (ctypes.c_int64 * (max(0, int(max_level)) + 1))()
    st = _lib.sp_project_tets_amr(ctx, ctypes.byref(prob), int(prec), int(max_level), counts, stream)
    return st, list(counts)


def sp_project_batch(ctx, dim: int, probs: Sequence[sp_problem], prec: int, stream=None) -> int:
    arr = (sp_problem * len(probs))(*probs)
    return _lib.sp_project_batch(ctx, int(dim), arr, len(probs), int(prec), stream)


def sp_sync_status(ctx, stream=None) -> int:
    return _lib.sp_sync_status(ctx, stream)


def sp_autotune(ctx, dim: int, sample: Sequence[sp_problem], prec: int, cache_path: Optional[str] = None) -> int:
    arr = (sp_problem * len(sample))(*sample)
    cp = cache_path.encode() if cache_path else None
    return _lib.sp_autotune(ctx, int(dim), arr, len(sample), int(prec), cp)


def sp_vertex_density(ctx, dim: int, xyz, n_vert: int, simplices, n_simplex: int, mass, mass_uniform: float,
                      box: sp_grid, rho_out, prec: int, stream=None) -> int:
    return _lib.sp_vertex_density(ctx, int(dim), xyz, int(n_vert), simplices, int(n_simplex), mass,
                                  float(mass_uniform), ctypes.byref(box), rho_out, int(prec), stream)


def sp_tuning_read(ctx):
    g, c, ip = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    st = _lib.sp_tuning_read(ctx, ctypes.byref(g), ctypes.byref(c), ctypes.byref(ip))
    return st, g.value, c.value, ip.value


def sp_tuning_set(ctx, slab_group: int, blocks_per_cu: int, item_pieces: int = 0) -> int:
    return _lib.sp_tuning_set(ctx, int(slab_group), int(blocks_per_cu), int(item_pieces))


def sp_profile_enable(ctx, on: int) -> int:
    return _lib.sp_profile_enable(ctx, int(on))


def sp_profile_read(ctx):
    prof = sp_profile()
    st = _lib.sp_profile_read(ctx, ctypes.byref(prof))
    return st, prof


def sp_last_error(ctx=None) -> str:
    return _lib.sp_last_error(ctx).decode(errors="replace")


# --------------------------------------------------------------------------
# torch glue

def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_problem(xyz, simplices, rho, dims, origin=(0.0, 0.0, 0.0), extent=(1.0, 1.0, 1.0),
                 periodic=(True, True, True), rho_per_corner=False, out=None, out_lo=None, total_mass=None,
                 out_mass=False, accumulate=False, validate=False) -> sp_problem:
    """Fill an sp_problem from device tensors (no copies)."""
    dim = int(xyz.shape[1]) if xyz.dim() == 2 else 3
    p = sp_problem()
    p.xyz = xyz.data_ptr() if xyz.numel() else None
    p.n_vert = int(xyz.shape[0])
    p.simplices = simplices.data_ptr() if simplices.numel() else None
    p.n_simplex = int(simplices.shape[0])
    p.rho = rho.data_ptr() if rho.numel() else None
    for d in range(3):
        p.grid.origin[d] = float(origin[d]) if d < len(origin) else 0.0
        p.grid.extent[d] = float(extent[d]) if d < len(extent) else 1.0
        p.grid.dims[d] = int(dims[d]) if d < len(dims) else 1
    fl = 0
    for d in range(min(3, len(periodic))):
        if periodic[d]:
            fl |= 1 << d
    if rho_per_corner:
        fl |= SP_RHO_PER_CORNER
    if out_mass:
        fl |= SP_OUT_MASS
    if accumulate:
        fl |= SP_ACCUMULATE
    if validate:
        fl |= SP_VALIDATE
    p.grid.flags = fl
    p.out = out.data_ptr() if out is not None else None
    p.out_lo = out_lo.data_ptr() if out_lo is not None else None
    p.total_mass = total_mass.data_ptr() if total_mass is not None else None
    return p


class Context:
    """An sp_ctx on one device (created lazily, destroyed with the object)."""

    def __init__(self, device: int = 0):
        st, h = sp_create(device)
        _check(st, "sp_create")
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            sp_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the module globals this needs may already
        # be gone (even `sys`, hence the bound default argument); the default
        # contexts are closed by the atexit hook below while everything is
        # still alive, and the process end releases the rest.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def project(self, xyz, simplices, rho, dims, origin=(0.0, 0.0, 0.0), extent=(1.0, 1.0, 1.0),
                periodic=(True, True, True), precision: str = "fp32c", rho_per_corner: bool = False,
                out=None, out_lo=None, out_mass: bool = False, accumulate: bool = False,
                validate: bool = False, want_total: bool = True, stream=None):
        """Project a mesh held in device tensors; returns (grid, total_mass).
        ``grid`` has shape dims reversed (z, y, x) / (y, x)."""
        import torch

        dim = int(xyz.shape[1])
        prec = SP_PREC_FP32C if precision == "fp32c" else SP_PREC_FP64
        dt = torch.float32 if prec == SP_PREC_FP32C else torch.float64
        if xyz.dtype != dt or rho.dtype != dt:
            raise TypeError(f"xyz and rho must be {dt} for precision {precision}")
        if simplices.dtype != torch.int32:
            raise TypeError("simplices must be int32")
        for t in (xyz, simplices, rho):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("inputs must be contiguous device tensors")
        shape = tuple(int(d) for d in reversed(list(dims)[:dim]))
        if out is None:
            out = torch.empty(shape, dtype=dt, device=xyz.device)
        total = torch.zeros(1, dtype=torch.float64, device=xyz.device) if want_total else None
        p = make_problem(xyz, simplices, rho, dims, origin, extent, periodic, rho_per_corner, out, out_lo, total,
                         out_mass, accumulate, validate)
        fn = sp_project_tets if dim == 3 else sp_project_tris
        _check(fn(self.handle, p, prec, _stream_ptr(stream)), fn.__name__)
        return out, total

    def project_corners(self, xyz, simplices, rho, dims, origin=(0.0, 0.0, 0.0), extent=(1.0, 1.0, 1.0),
                        periodic=(True, True, True), rho_per_corner: bool = False, out=None, out_mass: bool = False,
                        accumulate: bool = False, validate: bool = False, want_total: bool = True, stream=None,
                        fused: bool = False):
        """FP64 projection of tetrahedra by corner sums
        (sp_project_tets_corners, or sp_project_tets_corners_fused with
        fused); returns (grid, total_mass)."""
        import torch

        if xyz.dtype != torch.float64 or rho.dtype != torch.float64:
            raise TypeError("xyz and rho must be float64 for the corner-sum projection")
        if simplices.dtype != torch.int32 or int(xyz.shape[1]) != 3:
            raise TypeError("simplices must be int32 tetrahedra")
        for t in (xyz, simplices, rho):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("inputs must be contiguous device tensors")
        shape = tuple(int(d) for d in reversed(list(dims)[:3]))
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=xyz.device)
        total = torch.zeros(1, dtype=torch.float64, device=xyz.device) if want_total else None
        p = make_problem(xyz, simplices, rho, dims, origin, extent, periodic, rho_per_corner, out, None, total,
                         out_mass, accumulate, validate)
        fn = sp_project_tets_corners_fused if fused else sp_project_tets_corners
        _check(fn(self.handle, p, _stream_ptr(stream)), fn.__name__)
        return out, total

    def vertex_density(self, xyz, simplices, mass=None, mass_uniform: float = 1.0, extent=(1.0, 1.0, 1.0),
                       periodic=(True, True, True), precision: str = "fp32c", out=None, stream=None):
        """Per-vertex density sum(M_i) / sum(|V_i|) over incident simplices
        (sp_vertex_density); returns a device tensor [n_vert]."""
        import torch

        dim = int(xyz.shape[1])
        prec = SP_PREC_FP32C if precision == "fp32c" else SP_PREC_FP64
        dt = torch.float32 if prec == SP_PREC_FP32C else torch.float64
        if xyz.dtype != dt or (mass is not None and mass.dtype != dt):
            raise TypeError(f"xyz and mass must be {dt} for precision {precision}")
        if simplices.dtype != torch.int32:
            raise TypeError("simplices must be int32")
        for t in (xyz, simplices) + ((mass,) if mass is not None else ()):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("inputs must be contiguous device tensors")
        if out is None:
            out = torch.empty(int(xyz.shape[0]), dtype=dt, device=xyz.device)
        box = sp_grid()
        for d in range(3):
            box.extent[d] = float(extent[d]) if d < len(extent) else 1.0
        box.flags = sum(1 << d for d in range(min(3, len(periodic))) if periodic[d])
        st = sp_vertex_density(self.handle, dim, xyz.data_ptr() if xyz.numel() else None, int(xyz.shape[0]),
                               simplices.data_ptr() if simplices.numel() else None, int(simplices.shape[0]),
                               mass.data_ptr() if mass is not None else None, mass_uniform, box,
                               out.data_ptr() if out.numel() else None, prec, _stream_ptr(stream))
        _check(st, "sp_vertex_density")
        return out

    def project_accurate(self, xyz, simplices, rho, dims, accurate_bits: int = 10, wrong_bits: int = 10,
                         origin=(0.0, 0.0, 0.0), extent=(1.0, 1.0, 1.0), periodic=(True, True, True),
                         rho_per_corner: bool = False, out=None, out_lo=None, out_mass: bool = False,
                         validate: bool = False, want_total: bool = True, stream=None):
        """FP32C projection with per-voxel accuracy control
        (sp_project_tets_accurate); returns (grid, total_mass, flagged_cells,
        reprojected_simplices)."""
        import torch

        for t, dt in ((xyz, torch.float32), (rho, torch.float32), (simplices, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise TypeError("xyz/rho must be contiguous float32 and simplices int32 device tensors")
        shape = tuple(int(d) for d in reversed(list(dims)[:3]))
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=xyz.device)
        total = torch.zeros(1, dtype=torch.float64, device=xyz.device) if want_total else None
        p = make_problem(xyz, simplices, rho, dims, origin, extent, periodic, rho_per_corner, out, out_lo, total,
                         out_mass, False, validate)
        st, nflag, ntag = sp_project_tets_accurate(self.handle, p, accurate_bits, wrong_bits, _stream_ptr(stream))
        _check(st, "sp_project_tets_accurate")
        return out, total, nflag, ntag

    def project_amr(self, xyz, simplices, rho, dims, max_level: int, origin=(0.0, 0.0, 0.0),
                    extent=(1.0, 1.0, 1.0), periodic=(True, True, True), precision: str = "fp32c",
                    rho_per_corner: bool = False, out=None, out_mass: bool = False, validate: bool = False,
                    want_total: bool = True, stream=None):
        """Adaptive-grid projection gathered onto the uniform grid
        (sp_project_tets_amr); returns (grid, total_mass, simplices projected
        at each level)."""
        import torch

        prec = SP_PREC_FP32C if precision == "fp32c" else SP_PREC_FP64
        dt = torch.float32 if prec == SP_PREC_FP32C else torch.float64
        if xyz.dtype != dt or rho.dtype != dt or simplices.dtype != torch.int32:
            raise TypeError(f"xyz and rho must be {dt}, simplices int32")
        shape = tuple(int(d) for d in reversed(list(dims)[:3]))
        if out is None:
            out = torch.empty(shape, dtype=dt, device=xyz.device)
        total = torch.zeros(1, dtype=torch.float64, device=xyz.device) if want_total else None
        p = make_problem(xyz, simplices, rho, dims, origin, extent, periodic, rho_per_corner, out, None, total,
                         out_mass, False, validate)
        st, counts = sp_project_tets_amr(self.handle, p, prec, max_level, _stream_ptr(stream))
        _check(st, "sp_project_tets_amr")
        return out, total, counts

    def project_batch(self, problems, precision: str = "fp32c", dim: int = 3, stream=None) -> None:
        """Project several problems of dimension `dim` (sp_problem records
        built with make_problem; their tensors must stay alive) in one
        launch."""
        prec = SP_PREC_FP32C if precision == "fp32c" else SP_PREC_FP64
        _check(sp_project_batch(self.handle, dim, list(problems), prec, _stream_ptr(stream)), "sp_project_batch")

    def autotune(self, dim: int, sample, precision: str = "fp32c", cache_path: Optional[str] = None):
        """Tune the launch parameters on sample problems (several are timed
        as one batched launch); returns (slab_group, blocks_per_cu,
        item_pieces) now in use."""
        prec = SP_PREC_FP32C if precision == "fp32c" else SP_PREC_FP64
        _check(sp_autotune(self.handle, dim, list(sample), prec, cache_path), "sp_autotune")
        return self.tuning()

    def set_tuning(self, slab_group: int, blocks_per_cu: int = 0, item_pieces: int = 0) -> None:
        _check(sp_tuning_set(self.handle, slab_group, blocks_per_cu, item_pieces), "sp_tuning_set")

    def tuning(self):
        """(slab_group, blocks_per_cu, item_pieces) in use."""
        st, g, c, ip = sp_tuning_read(self.handle)
        _check(st, "sp_tuning_read")
        return g, c, ip

    def sync_status(self, stream=None) -> int:
        return sp_sync_status(self.handle, _stream_ptr(stream))

    def profile(self, on: int) -> None:
        _check(sp_profile_enable(self.handle, on), "sp_profile_enable")

    def profile_read(self) -> dict:
        st, prof = sp_profile_read(self.handle)
        _check(st, "sp_profile_read")
        return {k: getattr(prof, k) for k, _ in sp_profile._fields_}


# --------------------------------------------------------------------------
# module-level helpers on a per-device default context

_DEFAULT = {}


def _close_defaults() -> None:
    """Close the default contexts at interpreter exit, before module teardown
    (each close waits for its device and frees its memory)."""
    while _DEFAULT:
        _, ctx = _DEFAULT.popitem()
        ctx.close()


atexit.register(_close_defaults)


def default_context(device: int = 0) -> Context:
    """The context this module's helpers use on `device` (created once)."""
    if device not in _DEFAULT:
        _DEFAULT[device] = Context(device)
    return _DEFAULT[device]


def project(xyz, simplices, rho, dims, **kw):
    """Context.project on the default context of the tensors' device."""
    return default_context(xyz.device.index or 0).project(xyz, simplices, rho, dims, **kw)


def project_batch(problems, precision: str = "fp32c", dim: int = 3, device: int = 0, stream=None) -> None:
    """Context.project_batch on the default context of `device`."""
    default_context(device).project_batch(problems, precision=precision, dim=dim, stream=stream)
