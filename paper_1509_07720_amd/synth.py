"""Seeded synthetic meshes standing in for the paper's workloads.

This module holds input generation only: lattices, displacements, random
tetrahedron soups and the per-vertex density estimate that the solver feeds
to the projection (Section 4.4).  It performs no part of the projection
itself, so both the projection library and the test oracle may consume what
it produces.

Every generator returns a ``Problem`` dict with the keys

    dim        2 or 3
    xyz        float64 [n_vert][dim]   vertex positions inside [origin, origin+extent)
    simplices  int32   [n_simplex][dim+1]
    rho        float64 [n_vert]  or [n_simplex][dim+1] when ``rho_per_corner``
    rho_per_corner  bool
    origin, extent  float64 [3]  (2D: third entry unused)
    dims       int64 [3]         (2D: third entry 1)
    periodic   tuple of bools (3)
    meta       dict with the recipe and its parameters

The lattice meshes follow the paper's workloads: a Lagrangian sheet sampled
on a regular lattice, displaced either by the two-sine field of Section 5.2
or by a Zel'dovich displacement of a Gaussian random field (Appendix F.2),
with equal Lagrangian masses per simplex (Section 4.1) and vertex densities
from the mass/volume estimator of Section 4.4.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

Problem = Dict[str, object]

# ---------------------------------------------------------------------------
# lattices


def lattice_tris(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Periodic n x n lattice in the unit square, each square split along its
    (0,0)-(1,1) diagonal into two counter-clockwise triangles.

    Returns (q [n*n][2] Lagrangian positions in [0,1), tris [2n^2][3])."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    q = np.stack([i / n, j / n], axis=1).astype(np.float64)

    def vid(a, b):
        return (a % n) + n * (b % n)

    v00, v10, v11, v01 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
    tris = np.empty((2 * n * n, 3), dtype=np.int64)
    tris[0::2] = np.stack([v00, v10, v11], axis=1)
    tris[1::2] = np.stack([v00, v11, v01], axis=1)
    return q, tris.astype(np.int32)


# The six Kuhn (Freudenthal) tetrahedra of the unit cube: for a permutation s
# of the axes, v0=0, v1=e_s0, v2=e_s0+e_s1, v3=(1,1,1).  They share the main
# diagonal.  Odd permutations are reordered so that every tet is positively
# oriented.
_PERMS = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]


def _kuhn_offsets() -> List[np.ndarray]:
    out = []
    for s in _PERMS:
        v0 = np.zeros(3, np.int64)
        v1 = v0.copy()
        v1[s[0]] = 1
        v2 = v1.copy()
        v2[s[1]] = 1
        v3 = np.ones(3, np.int64)
        out.append(np.stack([v0, v1, v2, v3]))
    return out


def _orient_positive(off: np.ndarray) -> np.ndarray:
    d = np.linalg.det((off[1:] - off[0]).astype(np.float64))
    if d < 0:
        off = off[[0, 2, 1, 3]]
    return off


def lattice_tets(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Periodic n^3 Kuhn lattice in the unit cube: 6 n^3 positively oriented
    tets, vertex index i + n*(j + n*k)."""
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    q = np.stack([i / n, j / n, k / n], axis=1).astype(np.float64)
    tets = np.empty((6 * n ** 3, 4), dtype=np.int64)
    for t, off in enumerate(_kuhn_offsets()):
        off = _orient_positive(off)
        cols = []
        for a in range(4):
            cols.append(((i + off[a, 0]) % n) + n * (((j + off[a, 1]) % n) + n * ((k + off[a, 2]) % n)))
        tets[t::6] = np.stack(cols, axis=1)
    return q, tets.astype(np.int32)


def _bisected_kuhn_offsets() -> List[np.ndarray]:
    """Children of two levels of edge bisection of each Kuhn tet, as offsets on
    the doubled lattice (a coarse cube spans 2 fine steps).

    Level 1 bisects the shared main diagonal (v0,v3) at the cube centre c:
    (v0,v1,v2,c) and (c,v1,v2,v3).  Level 2 bisects a face diagonal of each
    child -- (v0,v2) for the first, (v1,v3) for the second -- at a face centre.
    Both bisected face diagonals are the Kuhn diagonals of the cube faces, so
    neighbouring cubes split every shared face the same way and the refined
    mesh stays conforming.  Every coarse cube then carries 5 vertices (corner,
    centre, three face centres) and 24 tets."""
    out = []
    for off in _kuhn_offsets():
        v0, v1, v2, v3 = [2 * o for o in off]
        c = (v0 + v3) // 2
        ma = (v0 + v2) // 2
        mb = (v1 + v3) // 2
        for ch in ((v0, v1, ma, c), (ma, v1, v2, c), (c, v1, v2, mb), (c, mb, v2, v3)):
            out.append(_orient_positive(np.stack(ch)))
    return out


def bisected_lattice_tets(n: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """2-level bisection of the periodic n^3 Kuhn lattice: 24 n^3 tets whose
    vertices sit on the (2n)^3 half lattice, 5 n^3 of its points in use.

    Returns (q [5n^3][3], tets [24n^3][4], fine [5n^3][3] integer half-lattice
    coordinates of each vertex)."""
    m = 2 * n
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    offs = _bisected_kuhn_offsets()
    # map of used fine lattice points -> compact index
    used = np.zeros(m ** 3, dtype=bool)
    fine_cols = []
    for off in offs:
        cols = []
        for a in range(4):
            fi = (2 * i + off[a, 0]) % m
            fj = (2 * j + off[a, 1]) % m
            fk = (2 * k + off[a, 2]) % m
            cols.append(fi + m * (fj + m * fk))
        fine_cols.append(cols)
        for c in cols:
            used[c] = True
    remap = -np.ones(m ** 3, dtype=np.int64)
    idx = np.nonzero(used)[0]
    remap[idx] = np.arange(idx.size)
    tets = np.empty((24 * n ** 3, 4), dtype=np.int32)
    for t, cols in enumerate(fine_cols):
        tets[t::24] = np.stack([remap[c] for c in cols], axis=1)
    fi = idx % m
    fj = (idx // m) % m
    fk = idx // (m * m)
    fine = np.stack([fi, fj, fk], axis=1)
    q = fine.astype(np.float64) / m
    return q, tets, fine


# ---------------------------------------------------------------------------
# displacement fields


def zeldovich(n: int, sigma: float, seed: int, dim: int = 3) -> np.ndarray:
    """Zel'dovich displacement Psi on the periodic n^dim lattice of the unit box.

    delta is a Gaussian random field whose power spectrum falls as k^-2, so its
    Fourier amplitude is white noise times 1/k, with the k=0 mode and the
    Nyquist planes removed.  Psi_k = i k delta_k / k^2, which makes
    div Psi = -delta (Appendix F.2).  Psi is scaled so that the rms of |Psi|
    equals ``sigma`` (box units).  Returns [n^dim][dim], lattice index with x
    fastest."""
    rng = np.random.default_rng(seed)
    shape = (n,) * dim
    white = rng.standard_normal(shape)
    wk = np.fft.rfftn(white)
    freqs = [np.fft.fftfreq(n, d=1.0 / n) for _ in range(dim - 1)] + [np.fft.rfftfreq(n, d=1.0 / n)]
    grids = np.meshgrid(*freqs, indexing="ij")  # axis 0 = slowest = last coordinate
    kvec = [2 * np.pi * g for g in grids]
    k2 = sum(kk * kk for kk in kvec)
    nyq = np.zeros(k2.shape, dtype=bool)
    for g in grids:
        nyq |= np.abs(g) == n // 2
    amp = np.zeros_like(k2)
    good = (k2 > 0) & ~nyq
    amp[good] = 1.0 / np.sqrt(k2[good])
    dk = wk * amp
    psi = []
    # grid axis a holds coordinate dim-1-a
    for coord in range(dim):
        kk = kvec[dim - 1 - coord]
        pk = np.zeros_like(dk)
        pk[good] = 1j * kk[good] * dk[good] / k2[good]
        psi.append(np.fft.irfftn(pk, s=shape, axes=tuple(range(dim))).ravel())
    psi = np.stack(psi, axis=1)
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=1))))
    return psi * (sigma / rms)


# ---------------------------------------------------------------------------
# per-vertex density (Section 4.4 estimator)


def unwrapped_corners(xyz: np.ndarray, simplices: np.ndarray, extent: np.ndarray, periodic) -> np.ndarray:
    """Corner positions of each simplex, minimum-image unwrapped relative to
    its first vertex on periodic axes.  [n_simplex][dim+1][dim]"""
    dim = xyz.shape[1]
    p = xyz[simplices].astype(np.float64)
    for d in range(dim):
        if periodic[d]:
            L = extent[d]
            rel = p[:, :, d] - p[:, :1, d]
            p[:, :, d] -= L * np.rint(rel / L)
    return p


def signed_volumes(corners: np.ndarray) -> np.ndarray:
    dim = corners.shape[2]
    e = corners[:, 1:, :] - corners[:, :1, :]
    return np.linalg.det(e) / math.factorial(dim)


def rho_vertex(xyz, simplices, masses, extent, periodic) -> np.ndarray:
    """rho_j = sum of masses of simplices sharing vertex j over the sum of their
    (unsigned) volumes (Section 4.4)."""
    vol = np.abs(signed_volumes(unwrapped_corners(xyz, simplices, extent, periodic)))
    nv = xyz.shape[0]
    k = simplices.shape[1]
    num = np.bincount(simplices.ravel(), weights=np.repeat(masses, k), minlength=nv)
    den = np.bincount(simplices.ravel(), weights=np.repeat(vol, k), minlength=nv)
    out = np.zeros(nv)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out


def _wrap(x: np.ndarray, L: float) -> np.ndarray:
    x = np.mod(x, L)
    x[x >= L] -= L
    return x


def _problem(dim, xyz, simp, rho, per_corner, dims, meta, periodic=(True, True, True)) -> Problem:
    dims3 = np.ones(3, np.int64)
    dims3[:dim] = dims
    return dict(dim=dim, xyz=xyz, simplices=np.ascontiguousarray(simp, dtype=np.int32),
                rho=rho, rho_per_corner=per_corner,
                origin=np.zeros(3), extent=np.ones(3), dims=dims3,
                periodic=tuple(bool(p) for p in periodic), meta=meta)


# ---------------------------------------------------------------------------
# the five workloads


def two_sine_2d(n: int = 32, grid: int = 64, amp_cells: float = 0.3, seed: int = 1,
                per_corner: bool = False) -> Problem:
    """2D sheet: n x n periodic lattice, 2n^2 triangles, displaced by two
    orthogonal sine waves of amplitude ``amp_cells`` Lagrangian cells with
    seeded phases (the two-sine collapse of Section 5.2), projected onto a
    grid x grid mesh.  Equal Lagrangian masses 1/(2n^2); per-vertex density
    from the Section 4.4 estimator, or per-corner rho = M_i/|V_i| which makes
    every triangle's mass exactly its Lagrangian area."""
    rng = np.random.default_rng(seed)
    q, tris = lattice_tris(n)
    A = amp_cells / n
    phi = rng.uniform(0.0, 2 * np.pi, size=2)
    x = q.copy()
    x[:, 0] = q[:, 0] + A * np.sin(2 * np.pi * q[:, 0] + phi[0])
    x[:, 1] = q[:, 1] + A * np.sin(2 * np.pi * q[:, 1] + phi[1])
    x = _wrap(x, 1.0)
    m = np.full(tris.shape[0], 1.0 / tris.shape[0])
    ext = np.ones(3)
    per = (True, True, True)
    if per_corner:
        vol = np.abs(signed_volumes(unwrapped_corners(x, tris, ext, per)))
        rho = np.repeat((m / vol)[:, None], 3, axis=1)
    else:
        rho = rho_vertex(x, tris, m, ext, per)
    meta = dict(recipe="two-sine 2D", n=n, grid=grid, amp_cells=amp_cells, seed=seed, phases=phi.tolist())
    return _problem(2, x, tris, rho, per_corner, [grid, grid], meta)


def zeldovich_3d(n: int = 64, grid: int = 128, sigma_cells: float = 1.5, seed: int = 2,
                 per_corner: bool = False) -> Problem:
    """3D sheet: periodic n^3 Kuhn lattice (6 n^3 tets) displaced by a
    Zel'dovich field with P(k) ~ k^-2 and rms |Psi| of ``sigma_cells``
    Lagrangian cells, projected onto grid^3.  Equal Lagrangian masses
    1/(6n^3); per-vertex density from the Section 4.4 estimator."""
    q, tets = lattice_tets(n)
    psi = zeldovich(n, sigma_cells / n, seed)
    x = _wrap(q + psi, 1.0)
    m = np.full(tets.shape[0], 1.0 / tets.shape[0])
    ext = np.ones(3)
    per = (True, True, True)
    if per_corner:
        vol = np.abs(signed_volumes(unwrapped_corners(x, tets, ext, per)))
        rho = np.repeat((m / vol)[:, None], 4, axis=1)
    else:
        rho = rho_vertex(x, tets, m, ext, per)
    meta = dict(recipe="Kuhn lattice + Zel'dovich", n=n, grid=grid, sigma_cells=sigma_cells, seed=seed)
    return _problem(3, x, tets, rho, per_corner, [grid] * 3, meta)


def _random_rotations(rng, n):
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


_REG_TET = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
_REG_VOL = 8.0 / 3.0


def tet_soup(n_tets: int = 10_000_000, grid: int = 256, vmin: float = 1e-6, vmax: float = 20.0,
             amax: float = 50.0, seed: int = 3, chunk: int = 1 << 20) -> Problem:
    """Independent tetrahedra standing in for an adaptively refined sheet:
    centres uniform in the unit box, volumes log-uniform in [vmin, vmax] voxel
    volumes, aspect ratio A log-uniform in [1, amax] (a randomly rotated
    regular tet stretched by A^(2/3) along a random axis and by A^(-1/3)
    across it), equal masses 1/n_tets carried by a per-corner density
    rho_a = (m/|V|)(1 + g_a/2) with centred g ~ U[-1,1] (so the mass of each
    tet is exactly m).  Coordinates are float32 wrapped into [0,1); the
    densities are computed from the float32 geometry."""
    rng = np.random.default_rng(seed)
    h = 1.0 / grid
    xyz = np.empty((4 * n_tets, 3), dtype=np.float32)
    rho = np.empty((n_tets, 4), dtype=np.float64)
    m0 = 1.0 / n_tets
    for s in range(0, n_tets, chunk):
        e = min(n_tets, s + chunk)
        n = e - s
        c = rng.random((n, 3))
        vol = np.exp(rng.uniform(math.log(vmin), math.log(vmax), n)) * h ** 3
        A = np.exp(rng.uniform(0.0, math.log(amax), n))
        R = _random_rotations(rng, n)
        d = rng.standard_normal((n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        spar = A ** (2.0 / 3.0)
        sper = A ** (-1.0 / 3.0)
        S = sper[:, None, None] * np.eye(3)[None] + (spar - sper)[:, None, None] * d[:, :, None] * d[:, None, :]
        base = np.einsum("vk,njk->nvj", _REG_TET, R)
        st = np.einsum("nvk,njk->nvj", base, S)
        scale = np.cbrt(vol / _REG_VOL)
        p = c[:, None, :] + st * scale[:, None, None]
        p = _wrap(p.reshape(-1, 3), 1.0).astype(np.float32)
        p[p >= np.float32(1.0)] = np.float32(0.0)
        xyz[4 * s:4 * e] = p
        g = rng.uniform(-1.0, 1.0, (n, 4))
        g -= g.mean(axis=1, keepdims=True)
        simp = np.arange(4 * n, dtype=np.int64).reshape(n, 4)
        v = np.abs(signed_volumes(unwrapped_corners(p.astype(np.float64), simp, np.ones(3), (True,) * 3)))
        rho[s:e] = (m0 / v)[:, None] * (1.0 + 0.5 * g)
    simp = np.arange(4 * n_tets, dtype=np.int32).reshape(n_tets, 4)
    meta = dict(recipe="tet soup", n_tets=n_tets, grid=grid, vmin=vmin, vmax=vmax, amax=amax, seed=seed)
    return _problem(3, xyz.astype(np.float64), simp, rho, True, [grid] * 3, meta)


def batch_sizes(count: int = 64, seed_base: int = 4000, nmin: float = 1e4, nmax: float = 2e6,
                smin: int = 32, smax: int = 256) -> List[Tuple[int, int, int]]:
    """(n_L, grid side, seed) per item of the batched workload: sizes
    log-uniform in [nmin, nmax] tets (n_L = max(2, rint(cbrt(N/6))), 6 n_L^3
    tets), grid sides log-uniform in [smin, smax] rounded to multiples of 8."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed_base + i)
        N = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        nl = max(2, int(round((N / 6.0) ** (1.0 / 3.0))))
        s = math.exp(rng.uniform(math.log(smin), math.log(smax)))
        s = int(min(smax, max(smin, 8 * round(s / 8))))
        out.append((nl, s, seed_base + i))
    return out


def batch_3d(count: int = 64, seed_base: int = 4000, **kw) -> List[Problem]:
    """The batched workload: independent Zel'dovich lattice meshes of uneven
    size onto grids of uneven size."""
    return [zeldovich_3d(n=nl, grid=s, sigma_cells=1.5, seed=seed)
            for (nl, s, seed) in batch_sizes(count, seed_base, **kw)]


def refined_3d(n: int = 128, grid: int = 512, sigma_cells: float = 4.0, seed: int = 5,
               linear: bool = False) -> Problem:
    """Two-level bisection of the periodic n^3 Kuhn lattice (24 n^3 tets, 5 n^3
    vertices) displaced by a Zel'dovich field of rms ``sigma_cells`` coarse
    cells sampled on the (2n)^3 half lattice, projected onto grid^3.

    With ``linear=True`` the bisection vertices are instead placed at the
    Eulerian midpoints of the displaced parent edge and carry the average of
    the parent densities, so the refined mesh describes exactly the same
    piecewise-linear density as its 6 n^3 parent tets."""
    q, tets, fine = bisected_lattice_tets(n)
    m2 = 2 * n
    ext = np.ones(3)
    per = (True, True, True)
    mass = np.full(tets.shape[0], 1.0 / tets.shape[0])
    if not linear:
        psi_full = zeldovich(m2, sigma_cells / n, seed)
        lid = fine[:, 0] + m2 * (fine[:, 1] + m2 * fine[:, 2])
        x = _wrap(q + psi_full[lid], 1.0)
        rho = rho_vertex(x, tets, mass, ext, per)
        meta = dict(recipe="2-level bisected Kuhn + Zel'dovich", n=n, grid=grid, sigma_cells=sigma_cells, seed=seed)
        return _problem(3, x, tets, rho, False, [grid] * 3, meta)
    # linear variant: parent lattice displaced on the coarse lattice
    psi = zeldovich(n, sigma_cells / n, seed)
    par_q, par_tets = lattice_tets(n)
    xp = _wrap(par_q + psi, 1.0)
    rho_p = rho_vertex(xp, par_tets, np.full(par_tets.shape[0], 1.0 / par_tets.shape[0]), ext, per)
    odd = fine % 2
    x = np.empty((fine.shape[0], 3))
    rho = np.empty(fine.shape[0])
    # each used half-lattice point is the average of the coarse-lattice corners
    # of the axis-aligned box it centres (1, 2, 4 or 8 corners: corner, edge
    # midpoint, face centre, cube centre); the bisection midpoints here are
    # only corners, face centres and cube centres, and the bisected edge always
    # joins two opposite corners of that box, whose minimum-image average is
    # the Eulerian midpoint used below.
    base = fine // 2
    a = base % n
    b = (base + odd) % n

    def cid(v):
        return v[:, 0] + n * (v[:, 1] + n * v[:, 2])

    # the bisected edges are Kuhn diagonals: they join the low corner of the
    # box to its high corner
    pa = xp[cid(a)]
    pb = xp[cid(b)]
    d = pb - pa
    d -= np.rint(d)
    x = _wrap(pa + 0.5 * d, 1.0)
    rho = 0.5 * (rho_p[cid(a)] + rho_p[cid(b)])
    meta = dict(recipe="2-level bisected Kuhn, linear midpoints", n=n, grid=grid, sigma_cells=sigma_cells,
                seed=seed)
    return _problem(3, x, tets, rho, False, [grid] * 3, meta)


def subset(prob: Problem, stride: int, offset: int = 0) -> Problem:
    """The simplices i with i % stride == offset (projection is additive over
    simplices, so a subset projects to its own share of the grid)."""
    p = dict(prob)
    sel = np.arange(offset, prob["simplices"].shape[0], stride)
    p["simplices"] = np.ascontiguousarray(prob["simplices"][sel])
    if prob["rho_per_corner"]:
        p["rho"] = np.ascontiguousarray(prob["rho"][sel])
    p["meta"] = dict(prob["meta"], subset_stride=stride, subset_offset=offset)
    return p


def as_float32(prob: Problem) -> Problem:
    """The same problem with positions and densities rounded to float32 (and
    kept as float64 arrays holding those float32 values), so that an FP64
    reference sees exactly the inputs an FP32 run sees."""
    p = dict(prob)
    x32 = np.array(prob["xyz"], dtype=np.float32)
    # a coordinate that rounds up onto the far face of a periodic box is the
    # same point as the near face
    origin = np.asarray(prob.get("origin", np.zeros(3)), dtype=np.float64)
    extent = np.asarray(prob.get("extent", np.ones(3)), dtype=np.float64)
    periodic = prob.get("periodic", (True, True, True))
    for d in range(x32.shape[1]):
        if periodic[d]:
            col = x32[:, d]
            col[col >= np.float32(origin[d] + extent[d])] = np.float32(origin[d])
    p["xyz"] = x32.astype(np.float64)
    p["rho"] = np.asarray(prob["rho"], dtype=np.float32).astype(np.float64)
    return p


def config(i: int, **kw) -> object:
    """Workload i (1-based, as numbered in the design notes) at full size;
    keyword arguments override sizes (tests use reduced sizes)."""
    if i == 1:
        return two_sine_2d(**kw)
    if i == 2:
        return zeldovich_3d(**kw)
    if i == 3:
        return tet_soup(**kw)
    if i == 4:
        return batch_3d(**kw)
    if i == 5:
        return refined_3d(**kw)
    raise ValueError(i)
