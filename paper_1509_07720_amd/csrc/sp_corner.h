// sp_corner.h -- the projection by first-order corner sums: the integral of
// a linear function over a polyhedron as a sum of terms that depend only on
// the local geometry at each of its vertices (Section 3.1, eq.
// eq_firstOrder with the corner terms of eq. eq:E03D and eq:E13D), summed
// for every cell over the four kinds of vertex a simplex-cell intersection
// has (Appendix D): A a simplex corner inside the cell, B a simplex edge
// through a cell face, C a simplex facet through a cell edge, D a cell
// corner inside the simplex.  No intersection polytope is ever built; each
// vertex's terms go straight to the cell(s) whose piece it is a vertex of.
//
// For a vertex at P with three edges (unit directions T leaving it) and
// three facets (unit inward normals B), every (edge, facet holding it) pair
// contributes E0 (rho0 + E1 . grad) with
//   N  = the unit vector in the facet, orthogonal to T, pointing into it,
//   E0 = -(P.T)(P.N)(P.B) / 6,   E1 = ((P.T) T + 2 (P.N) N + 3 (P.B) B) / 4,
// where P and rho0 refer to one origin shared by all vertices of the same
// piece.  The origin of the piece of cell c is the point of the simplex's
// bounding box nearest to the centre of c, so that P stays as short as the
// piece allows and the signed terms cancel little.
//
// FP64 only.  The terms are signed and cancel within a cell; the paper's
// own implementation ran them in double-double for that reason.  Predicates
// are evaluated in FP64 and need general position: a simplex with a corner
// on a grid plane is moved off it by a tiny offset (below); a cell edge
// through a facet's boundary or a cell corner on a facet that remains is
// reported as degenerate (the sum is then not trustworthy).  So is a
// simplex whose bounding box holds more than 2^24 cells (one thread
// enumerates them all).  The clipping projection has neither restriction.
#pragma once

#include "sp_setup.h"

namespace sp {

struct D3 {
    double x, y, z;
};

SP_HD inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
SP_HD inline D3 operator+(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
SP_HD inline D3 operator-(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
SP_HD inline D3 operator*(double s, D3 a) { return d3(s * a.x, s * a.y, s * a.z); }
SP_HD inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
SP_HD inline D3 cross(D3 a, D3 b) { return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
SP_HD inline D3 unit(D3 a) { return (1.0 / sqrt(dot(a, a))) * a; }
SP_HD inline double comp(D3 a, int d) { return d == 0 ? a.x : (d == 1 ? a.y : a.z); }
SP_HD inline D3 axis(int d, double s) { return d3(d == 0 ? s : 0.0, d == 1 ? s : 0.0, d == 2 ? s : 0.0); }

// The corner terms of one vertex: edges t[0..2], facets with inward normals
// b[0..2], facet f holding edges fe[f][0] and fe[f][1].  The fixed-count
// loops here and below are unrolled so that these small arrays are indexed
// by constants (registers, not scratch memory).
SP_HD inline double vertex_terms(D3 P, double rho0, D3 g, const D3 *t, const D3 *b, const int (*fe)[2])
{
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const D3 T = t[fe[f][k]];
            const D3 other = t[fe[f][1 - k]];
            D3 N = unit(cross(b[f], T));
            if (dot(N, other) < 0.0) N = -1.0 * N;
            const double pt = dot(P, T), pn = dot(P, N), pb = dot(P, b[f]);
            const double e0 = -pt * pn * pb / 6.0;
            const double e1g = 0.25 * (pt * dot(T, g) + 2.0 * pn * dot(N, g) + 3.0 * pb * dot(b[f], g));
            s += e0 * (rho0 + e1g);
        }
    }
    return s;
}

// Projection of one simplex (local cell coordinates, as set up for the
// clipping path) by corner sums; dep(ix, iy, iz, value) receives each term
// sum at local cell indices, in cell-volume units.  Returns the number of
// degenerate configurations met.
template <typename Dep>
SP_HD inline int corner_project(const Local<double> &L, Dep &dep)
{
    D3 v[4];
    double r[4];
    for (int a = 0; a < 4; ++a) {
        v[a] = d3(L.v[a].x, L.v[a].y, L.v[a].z);
        r[a] = L.v[a].r;
    }
    int degenerate = 0;
    // A corner on a grid plane (common with FP32 inputs, and everywhere on
    // lattice-aligned meshes) puts the simplex outside general position.
    // The sum is continuous in the corner positions, so such a simplex is
    // moved, with its density, by a tiny generic offset (components
    // 1 : sqrt 2 : sqrt 3 times 2^-40 cells): its pieces change by about
    // 1e-12 of a cell's coverage, its total not at all.
    bool on_plane = false;
    for (int a = 0; a < 4; ++a)
        on_plane = on_plane || v[a].x == floor(v[a].x) || v[a].y == floor(v[a].y) || v[a].z == floor(v[a].z);
    if (on_plane) {
        const D3 shift = d3(9.094947017729282e-13, 1.2862197421537486e-12, 1.5752910326854155e-12);
        for (int a = 0; a < 4; ++a) v[a] = v[a] + shift;
    }
    // gradient of rho: (v_k - v_0) . g = r_k - r_0 (Cramer's rule)
    const D3 e1 = v[1] - v[0], e2 = v[2] - v[0], e3 = v[3] - v[0];
    const D3 c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
    const double det = dot(e1, c23);
    const double inv = 1.0 / det;
    const D3 g = (inv * (r[1] - r[0])) * c23 + (inv * (r[2] - r[0])) * c31 + (inv * (r[3] - r[0])) * c12;
    D3 lo = v[0], hi = v[0];
    for (int a = 1; a < 4; ++a) {
        lo = d3(fmin(lo.x, v[a].x), fmin(lo.y, v[a].y), fmin(lo.z, v[a].z));
        hi = d3(fmax(hi.x, v[a].x), fmax(hi.y, v[a].y), fmax(hi.z, v[a].z));
    }
    // one thread walks every grid point of the bounding box: a simplex over
    // more than 2^24 cells is not summed (reported like a degenerate one)
    if ((floor(hi.x) - floor(lo.x) + 1.0) * (floor(hi.y) - floor(lo.y) + 1.0) * (floor(hi.z) - floor(lo.z) + 1.0) >
        16777216.0)
        return 1;
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            if (comp(v[a], d) == floor(comp(v[a], d))) ++degenerate;  // a corner on a grid plane

    // origin of the piece in cell (cx, cy, cz), and the density there
    auto origin = [&](int cx, int cy, int cz) {
        return d3(fmin(fmax(cx + 0.5, lo.x), hi.x), fmin(fmax(cy + 0.5, lo.y), hi.y), fmin(fmax(cz + 0.5, lo.z), hi.z));
    };
    auto rho_at = [&](D3 X) { return r[0] + dot(g, X - v[0]); };
    auto deposit = [&](int cx, int cy, int cz, D3 X, const D3 *t, const D3 *b, const int (*fe)[2]) {
        const D3 o = origin(cx, cy, cz);
        const double s = vertex_terms(X - o, rho_at(o), g, t, b, fe);
        if (s != 0.0) dep(cx, cy, cz, s);
    };
    // inward unit normal of the facet opposite corner m
    auto inward = [&](int m) {
        const int i = (m + 1) & 3, j = (m + 2) & 3, k = (m + 3) & 3;
        D3 n = cross(v[j] - v[i], v[k] - v[i]);
        if (dot(n, v[m] - v[i]) < 0.0) n = -1.0 * n;
        return unit(n);
    };
    D3 nf[4];
    for (int m = 0; m < 4; ++m) nf[m] = inward(m);

    // A: every simplex corner, in its own cell; facet k of the corner's
    // cone is the simplex facet opposite the corner's edge k
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int o3[3], n = 0;
        for (int k = 0; k < 4; ++k)
            if (k != a) o3[n++] = k;
        D3 t[3], b[3];
        int fe[3][2];
        for (int k = 0; k < 3; ++k) {
            t[k] = unit(v[o3[k]] - v[a]);
            b[k] = nf[o3[k]];  // the facet without o3[k] holds the other two edges
            fe[k][0] = (k + 1) % 3;
            fe[k][1] = (k + 2) % 3;
        }
        deposit((int)floor(v[a].x), (int)floor(v[a].y), (int)floor(v[a].z), v[a], t, b, fe);
    }

    // B: every edge through every grid plane it crosses; the crossing point
    // is a vertex of the pieces on both sides of the plane
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int bq = a + 1; bq < 4; ++bq) {
            int m1 = -1, m2 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != a && k != bq) (m1 < 0 ? m1 : m2) = k;
            // facet (a, bq, m1) is the one opposite m2, and the reverse
            const D3 n1 = nf[m2], n2 = nf[m1];
            for (int d = 0; d < 3; ++d) {
                const double pa = comp(v[a], d), pb = comp(v[bq], d);
                const double l = fmin(pa, pb), h = fmax(pa, pb);
                for (int c = (int)floor(l) + 1; (double)c < h; ++c) {
                    const double tt = ((double)c - pa) / (pb - pa);
                    D3 p = v[a] + tt * (v[bq] - v[a]);
                    if (d == 0) p.x = c; else if (d == 1) p.y = c; else p.z = c;
                    const D3 ed = axis(d, 1.0);
                    D3 u1 = unit(cross(n1, ed));
                    if (dot(u1, n2) < 0.0) u1 = -1.0 * u1;
                    D3 u2 = unit(cross(n2, ed));
                    if (dot(u2, n1) < 0.0) u2 = -1.0 * u2;
                    const D3 up = pb > pa ? unit(v[bq] - v[a]) : unit(v[a] - v[bq]);
                    for (int side = 0; side < 2; ++side) {
                        const double sg = side == 0 ? 1.0 : -1.0;
                        const D3 t[3] = {sg * up, u1, u2};
                        const D3 b[3] = {n1, n2, axis(d, sg)};
                        const int fe[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                        int cell[3] = {(int)floor(p.x), (int)floor(p.y), (int)floor(p.z)};
                        cell[d] = side == 0 ? c : c - 1;
                        for (int q = 0; q < 3; ++q)
                            if (q != d && comp(p, q) == floor(comp(p, q))) ++degenerate;
                        deposit(cell[0], cell[1], cell[2], p, t, b, fe);
                    }
                }
            }
        }
    }

    // C: every facet through every cell edge (grid line) it crosses; the
    // crossing is a vertex of the four pieces around that line
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int ia = (m + 1) & 3, ib = (m + 2) & 3, ic = (m + 3) & 3;
        const D3 nF = nf[m];
        for (int d = 0; d < 3; ++d) {
            const double nd = comp(nF, d);
            if (nd == 0.0) continue;  // lines along d run parallel to the facet
            const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            const double ax = comp(v[ia], d1), ay = comp(v[ia], d2);
            const double bx = comp(v[ib], d1), by = comp(v[ib], d2);
            const double cxx = comp(v[ic], d1), cyy = comp(v[ic], d2);
            const double l1 = fmin(ax, fmin(bx, cxx)), h1 = fmax(ax, fmax(bx, cxx));
            const double l2 = fmin(ay, fmin(by, cyy)), h2 = fmax(ay, fmax(by, cyy));
            for (int j = (int)floor(l1) + 1; (double)j < h1; ++j) {
                for (int k = (int)floor(l2) + 1; (double)k < h2; ++k) {
                    const double o1 = (bx - ax) * (k - ay) - (by - ay) * (j - ax);
                    const double o2 = (cxx - bx) * (k - by) - (cyy - by) * (j - bx);
                    const double o3 = (ax - cxx) * (k - cyy) - (ay - cyy) * (j - cxx);
                    if (o1 == 0.0 || o2 == 0.0 || o3 == 0.0) {
                        ++degenerate;
                        continue;
                    }
                    if (!((o1 > 0.0 && o2 > 0.0 && o3 > 0.0) || (o1 < 0.0 && o2 < 0.0 && o3 < 0.0))) continue;
                    const double qd = comp(v[ia], d) - (comp(nF, d1) * (j - ax) + comp(nF, d2) * (k - ay)) / nd;
                    D3 q = axis(d, qd) + axis(d1, (double)j) + axis(d2, (double)k);
                    const D3 tl = axis(d, nd > 0.0 ? 1.0 : -1.0);
                    const D3 w1r = unit(cross(nF, axis(d1, 1.0)));
                    const D3 w2r = unit(cross(nF, axis(d2, 1.0)));
                    if (qd == floor(qd)) ++degenerate;
                    for (int s1 = 0; s1 < 2; ++s1) {
                        for (int s2 = 0; s2 < 2; ++s2) {
                            const D3 w1 = ((comp(w1r, d2) > 0.0) == (s2 == 1)) ? w1r : -1.0 * w1r;
                            const D3 w2 = ((comp(w2r, d1) > 0.0) == (s1 == 1)) ? w2r : -1.0 * w2r;
                            const D3 t[3] = {tl, w1, w2};
                            const D3 b[3] = {nF, axis(d1, s1 ? 1.0 : -1.0), axis(d2, s2 ? 1.0 : -1.0)};
                            const int fe[3][2] = {{1, 2}, {0, 1}, {0, 2}};
                            int cell[3];
                            cell[d] = (int)floor(qd);
                            cell[d1] = j - 1 + s1;
                            cell[d2] = k - 1 + s2;
                            deposit(cell[0], cell[1], cell[2], q, t, b, fe);
                        }
                    }
                }
            }
        }
    }

    // D: every grid point strictly inside the simplex, a corner of its
    // eight cells
    double off[4];
    for (int m = 0; m < 4; ++m) off[m] = dot(nf[m], v[(m + 1) & 3]);
    const int x0 = (int)floor(lo.x) + 1, y0 = (int)floor(lo.y) + 1, z0 = (int)floor(lo.z) + 1;
    for (int z = z0; (double)z < hi.z; ++z) {
        for (int y = y0; (double)y < hi.y; ++y) {
            for (int x = x0; (double)x < hi.x; ++x) {
                const D3 w = d3(x, y, z);
                bool in = true;
                for (int m = 0; m < 4 && in; ++m) {
                    const double sd = dot(nf[m], w) - off[m];
                    if (sd == 0.0) ++degenerate;
                    in = sd > 0.0;
                }
                if (!in) continue;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
                    const D3 t[3] = {axis(0, dx ? -1.0 : 1.0), axis(1, dy ? -1.0 : 1.0), axis(2, dz ? -1.0 : 1.0)};
                    const D3 b[3] = {t[0], t[1], t[2]};  // the face across axis k holds the other two edges
                    const int fe[3][2] = {{1, 2}, {0, 2}, {0, 1}};
                    deposit(x - dx, y - dy, z - dz, w, t, b, fe);
                }
            }
        }
    }
    return degenerate;
}

}  // namespace sp
