"""Monte Carlo deposit -- TEST INFRASTRUCTURE.

The paper checks its grid projection against particles drawn at random
inside every simplex (Section 5.2, the radial-profile comparison).  Here each
simplex receives K points uniform inside it (barycentric coordinates drawn
from Dirichlet(1,...,1)), each carrying |V| rho(point) / K; binning the
points gives an unbiased estimate of every cell's mass together with its
sampling variance, against which the oracle is compared by z-score.
"""
from __future__ import annotations

import numpy as np


def project(prob, K: int = 64, seed: int = 0, chunk: int = 4096):
    """Returns (estimate, variance) grids of mass per cell (C order, x
    fastest)."""
    rng = np.random.default_rng(seed)
    dim = int(prob["dim"])
    xyz = np.asarray(prob["xyz"], dtype=np.float64).reshape(-1, dim)
    simp = np.asarray(prob["simplices"]).reshape(-1, dim + 1)
    rho = np.asarray(prob["rho"], dtype=np.float64)
    dims = [int(v) for v in prob["dims"]][:dim]
    org = np.asarray(prob["origin"], dtype=np.float64)[:dim]
    ext = np.asarray(prob["extent"], dtype=np.float64)[:dim]
    per = prob["periodic"]
    ncell = int(np.prod(dims))
    est = np.zeros(ncell)
    var = np.zeros(ncell)
    for s0 in range(0, simp.shape[0], chunk):
        S = simp[s0:s0 + chunk]
        n = S.shape[0]
        P = xyz[S]  # n, k, dim
        for d in range(dim):
            if per[d]:
                L = ext[d]
                P[:, :, d] -= L * np.rint((P[:, :, d] - P[:, :1, d]) / L)
        R = rho[s0:s0 + chunk] if prob["rho_per_corner"] else rho[S]
        E = P[:, 1:, :] - P[:, :1, :]
        vol = np.abs(np.linalg.det(E)) / (2.0 if dim == 2 else 6.0)
        lam = rng.dirichlet(np.ones(dim + 1), size=(n, K))  # n, K, k
        pts = np.einsum("nka,nad->nkd", lam, P)
        w = (vol[:, None] * np.einsum("nka,na->nk", lam, R)) / K
        idx = np.zeros((n, K), dtype=np.int64)
        stride = 1
        ok = np.ones((n, K), dtype=bool)
        for d in range(dim):
            c = np.floor((pts[:, :, d] - org[d]) * (dims[d] / ext[d])).astype(np.int64)
            if per[d]:
                c %= dims[d]
            else:
                ok &= (c >= 0) & (c < dims[d])
                c = np.clip(c, 0, dims[d] - 1)
            idx += c * stride
            stride *= dims[d]
        idx = idx[ok]
        ww = w[ok]
        est += np.bincount(idx, weights=ww, minlength=ncell)
        var += np.bincount(idx, weights=ww * ww, minlength=ncell)
    shape = tuple(reversed(dims))
    return est.reshape(shape), var.reshape(shape)
