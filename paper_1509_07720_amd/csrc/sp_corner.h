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
// own implementation ran them in double-double for that reason (here the
// origin of each piece is kept near it instead, which holds the per-cell
// error near 1e-14 of the cell's coverage).
//
// Degenerate positions (a corner on a grid plane, an edge through a grid
// line, a facet through a grid point...) are resolved by simulation of
// simplicity (Section 3.3, eq. eq_sos): the grid's vertices move to
// (x - e^2, y - e^3, z - e^4) for an infinitesimal e > 0, so no grid plane,
// line or point ever meets the simplex's boundary, and every predicate
// whose value is exactly zero takes the sign of the first non-zero term of
// its expansion in e (App. E.1, eq. eq_orientation_sos; for the crossing of
// an edge with grid planes this is the priority order of App. E.3).  The
// sum itself is evaluated at e = 0: it is continuous in the positions, and
// the perturbation only decides which vertices each piece has.  Predicates
// are filtered: an FP64 value larger than its rounding bound decides at
// once; a smaller one is evaluated again in double-double on the exact
// differences of the inputs (exact for inputs with up to about 26
// significant bits in cell units, such as FP32 data) before it is called a
// tie.  A simplex whose bounding box holds more than 2^24 cells (one
// thread enumerates them all) is not summed and is reported.
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

// ------------------------------------------------------------------------
// filtered predicates with simulation of simplicity

// exponent order of the perturbation: x (e^2) before y (e^3) before z (e^4)

struct DD {
    double hi, lo;
};
// (Error-free transformations: their additions must see the rounded
// products, so multiply-add contraction is off in them and in the
// predicates built on them.)
SP_HD inline DD dd_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return DD{s, (a - (s - bb)) + (b - bb)};
}
SP_HD inline DD dd_diff(double a, double b) { return dd_two_sum(a, -b); }  // a - b exactly
SP_HD inline DD dd_add(DD a, DD b)
{
#pragma clang fp contract(off)
    const DD s = dd_two_sum(a.hi, b.hi);
    return dd_two_sum(s.hi, s.lo + a.lo + b.lo);
}
SP_HD inline DD dd_neg(DD a) { return DD{-a.hi, -a.lo}; }
SP_HD inline DD dd_mul(DD a, DD b)
{
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    const double e = fma(a.hi, b.hi, -p);
    return dd_two_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}
SP_HD inline int sgn(double x) { return (x > 0.0) - (x < 0.0); }

// Sign of u1 v2 - u2 v1 for u = (a1 - b1, a2 - b2), v = (c1 - d1, c2 - d2),
// i.e. of (a1 - b1)(c2 - d2) - (a2 - b2)(c1 - d1), given by the end points
// (0: an exact tie, as far as double-double can tell).
SP_HD inline int sign_det2(double a1, double b1, double a2, double b2, double c1, double d1, double c2, double d2)
{
#pragma clang fp contract(off)
    const double u1 = a1 - b1, u2 = a2 - b2, v1 = c1 - d1, v2 = c2 - d2;
    const double x = u1 * v2, y = u2 * v1;
    const double r = x - y;
    const double mag = fabs(x) + fabs(y);
    if (fabs(r) > 0x1p-48 * mag) return sgn(r);
    const DD U1 = dd_diff(a1, b1), U2 = dd_diff(a2, b2), V1 = dd_diff(c1, d1), V2 = dd_diff(c2, d2);
    const DD R = dd_add(dd_mul(U1, V2), dd_neg(dd_mul(U2, V1)));
    return fabs(R.hi) > 0x1p-98 * mag ? sgn(R.hi) : 0;
}

// Sign of the triple product (p - o) . ((q - o) x (r - o)).
SP_HD inline int sign_tri(D3 p, D3 q, D3 r, D3 o)
{
#pragma clang fp contract(off)
    const D3 u = p - o, v = q - o, w = r - o;
    const double t = dot(u, cross(v, w));
    const double mag = (fabs(u.x) + fabs(u.y) + fabs(u.z)) * (fabs(v.x) + fabs(v.y) + fabs(v.z)) *
                       (fabs(w.x) + fabs(w.y) + fabs(w.z));
    if (fabs(t) > 0x1p-46 * mag) return sgn(t);
    const DD U[3] = {dd_diff(p.x, o.x), dd_diff(p.y, o.y), dd_diff(p.z, o.z)};
    const DD V[3] = {dd_diff(q.x, o.x), dd_diff(q.y, o.y), dd_diff(q.z, o.z)};
    const DD W[3] = {dd_diff(r.x, o.x), dd_diff(r.y, o.y), dd_diff(r.z, o.z)};
    DD T = DD{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = (k + 1) % 3, j = (k + 2) % 3;
        const DD c = dd_add(dd_mul(V[i], W[j]), dd_neg(dd_mul(V[j], W[i])));
        T = dd_add(T, dd_mul(U[k], c));
    }
    return fabs(T.hi) > 0x1p-94 * mag ? sgn(T.hi) : 0;
}

// Sign of the first non-zero component of (q - o) x (r - o) in the
// perturbation's order x, y, z (the normal of a plane through o, q, r).
SP_HD inline int sign_normal_first(D3 q, D3 r, D3 o)
{
    // component k of (q - o) x (r - o): (q_i - o_i)(r_j - o_j) - (q_j - o_j)(r_i - o_i)
    int s = sign_det2(q.y, o.y, q.z, o.z, r.y, o.y, r.z, o.z);  // x: qy rz - qz ry
    if (s) return s;
    s = sign_det2(q.z, o.z, q.x, o.x, r.z, o.z, r.x, o.x);      // y: qz rx - qx rz
    if (s) return s;
    return sign_det2(q.x, o.x, q.y, o.y, r.x, o.x, r.y, o.y);   // z: qx ry - qy rx
}

// Side of the perturbed grid point w - (e^2, e^3, e^4) relative to the plane
// through o, q, r: the sign of (w - o) . ((q - o) x (r - o)) under the
// perturbation (never 0).
SP_HD inline int sos_side(D3 w, D3 q, D3 r, D3 o)
{
    const int s = sign_tri(w, q, r, o);
    return s ? s : -sign_normal_first(q, r, o);
}

// Cell along axis q of the point where edge (a, b) crosses the (perturbed)
// grid plane x_d = c, approx its FP64 value: the largest m with the point's
// coordinate at or above the perturbed plane x_q = m.
SP_HD inline int sos_edge_cell(D3 a, D3 b, int d, int q, int c, double approx)
{
    const double ad = comp(a, d), bd = comp(b, d), aq = comp(a, q), bq = comp(b, q);
    const int sd = bd > ad ? 1 : -1;
    // sign of (p_q - m): ((a_q - m)(b_d - a_d) + (c - a_d)(b_q - a_q)) sign(b_d - a_d), and on a tie
    // the perturbation's first term: + for q before d, else -sign(b_q - a_q) sign(b_d - a_d)
    auto above = [&](int m) {
        int s = sign_det2(aq, (double)m, ad, (double)c, bq, aq, bd, ad);
        s *= sd;
        if (s) return s > 0;
        if (q < d) return true;
        const int t = (bq > aq) - (bq < aq);
        return t == 0 ? true : (-t * sd > 0);
    };
    int m = (int)floor(approx);
    while (!above(m)) --m;
    while (above(m + 1)) ++m;
    return m;
}

// Fused facet contributions (App. D, eq. eq_contribFused and eq_diffRho).
// A facet f shared by simplices s and j: every (vertex, edge, facet f) term
// of a piece of s in a cell has a twin in the piece of j in the same cell,
// with the same vertex, edge and in-facet direction and the opposite facet
// normal when s and j lie on opposite sides of f (the same normal when a
// fold puts both on one side), so with one origin O per cell shared by both
//   C_s + C_j = E0 ((rho_s(O) + sigma rho_j(O)) + E1 . (g_s + sigma g_j)),
// sigma = -1 on opposite sides, +1 on the same side, E0 and E1 those of s.
// The simplex of lower index sums each pair; the other leaves it out.
enum : int { FACET_PLAIN = 0, FACET_FUSED = 1, FACET_SKIP = 2 };

// How one simplex treats the terms on its facets (indexed by the corner
// opposite each facet, in the simplex's local corner order): the mode, and
// for a fused facet the pair's density rho_s + sigma rho_j as
// R + G . (X - xr), xr a corner of the facet (local coordinates): taken
// relative to a point of the facet, the difference of two densities that
// agree there is not the difference of two large values.
struct FacetFuse {
    int mode[4];
    D3 G[4];
    D3 xr[4];
    double R[4];
    bool cell_origin;  // origins at cell centres (any facet paired), shared with the neighbours
};

// The corner terms of one vertex: edges t[0..2], facets with inward normals
// b[0..2], facet f holding edges fe[f][0] and fe[f][1]; mf[f] is the
// simplex facet that b[f] lies on (the corner opposite it), or -1 for a
// grid plane.  P = vertex - O, rho0 = rho(O).  The fixed-count loops here
// and below are unrolled so that these small arrays are indexed by
// constants (registers, not scratch memory).
SP_HD inline double vertex_terms(D3 P, double rho0, D3 g, const D3 *t, const D3 *b, const int (*fe)[2], const int *mf,
                                 const FacetFuse *fz, D3 O)
{
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        double r0 = rho0;
        D3 gf = g;
        if (fz && mf[f] >= 0) {
            const int m = mf[f];
            if (fz->mode[m] == FACET_SKIP) continue;
            if (fz->mode[m] == FACET_FUSED) {
                r0 = fz->R[m] + dot(fz->G[m], O - fz->xr[m]);
                gf = fz->G[m];
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const D3 T = t[fe[f][k]];
            const D3 other = t[fe[f][1 - k]];
            D3 N = unit(cross(b[f], T));
            if (dot(N, other) < 0.0) N = -1.0 * N;
            const double pt = dot(P, T), pn = dot(P, N), pb = dot(P, b[f]);
            const double e0 = -pt * pn * pb / 6.0;
            const double e1g = 0.25 * (pt * dot(T, gf) + 2.0 * pn * dot(N, gf) + 3.0 * pb * dot(b[f], gf));
            s += e0 * (r0 + e1g);
        }
    }
    return s;
}

// One thread walks every grid point of a simplex's bounding box: a simplex
// over more than 2^24 cells is not summed (and is reported).
SP_HD inline bool corner_box_ok(const Local<double> &L)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        const double x0 = d == 0 ? L.v[0].x : (d == 1 ? L.v[0].y : L.v[0].z);
        lo[d] = hi[d] = x0;
        for (int a = 1; a < 4; ++a) {
            const double x = d == 0 ? L.v[a].x : (d == 1 ? L.v[a].y : L.v[a].z);
            lo[d] = fmin(lo[d], x);
            hi[d] = fmax(hi[d], x);
        }
    }
    return (floor(hi[0]) - floor(lo[0]) + 1.0) * (floor(hi[1]) - floor(lo[1]) + 1.0) *
               (floor(hi[2]) - floor(lo[2]) + 1.0) <=
           16777216.0;
}

// Gradient of the simplex's linear density: (v_k - v_0) . g = r_k - r_0
// (Cramer's rule), from its local corners; a neighbour's copy of this value
// is what the fused terms use.
SP_HD inline D3 corner_gradient(const Local<double> &L)
{
    const D3 v0 = d3(L.v[0].x, L.v[0].y, L.v[0].z);
    const D3 e1 = d3(L.v[1].x, L.v[1].y, L.v[1].z) - v0, e2 = d3(L.v[2].x, L.v[2].y, L.v[2].z) - v0,
             e3 = d3(L.v[3].x, L.v[3].y, L.v[3].z) - v0;
    const D3 c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
    const double inv = 1.0 / dot(e1, c23);
    return (inv * (L.v[1].r - L.v[0].r)) * c23 + (inv * (L.v[2].r - L.v[0].r)) * c31 +
           (inv * (L.v[3].r - L.v[0].r)) * c12;
}

// Whether a simplex takes part in fused terms: a density gradient of more
// than 1024 times its largest corner value per cell (a sliver: its terms
// are huge and cancel to a tiny piece) is left out, so that its terms keep
// cancelling within its own pieces; its neighbours then sum those facets
// alone.
SP_HD inline bool corner_fusable(const Local<double> &L, D3 g)
{
    double rmax = 0.0;
    for (int a = 0; a < 4; ++a) rmax = fmax(rmax, fabs(L.v[a].r));
    return fmax(fabs(g.x), fmax(fabs(g.y), fabs(g.z))) <= 1024.0 * rmax;
}

// Side of facet m (opposite local corner m) that the simplex lies on, in a
// frame every simplex sharing the facet agrees on: the sign of
// (X - A) . ((B - A) x (C - A)), with A, B, C the facet's corners in
// increasing vertex id vid[] and X the opposite corner (0 only for a flat
// simplex).
SP_HD inline int facet_side(const Local<double> &L, const int64_t *vid, int m)
{
    int c[3], n = 0;
    for (int a = 0; a < 4; ++a)
        if (a != m) c[n++] = a;
    // sort the three corners by vertex id
    if (vid[c[1]] < vid[c[0]]) { const int t = c[0]; c[0] = c[1]; c[1] = t; }
    if (vid[c[2]] < vid[c[1]]) { const int t = c[1]; c[1] = c[2]; c[2] = t; }
    if (vid[c[1]] < vid[c[0]]) { const int t = c[0]; c[0] = c[1]; c[1] = t; }
    auto P = [&](int a) { return d3(L.v[a].x, L.v[a].y, L.v[a].z); };
    return sign_tri(P(m), P(c[1]), P(c[2]), P(c[0]));
}

// Fused data of facet m of a simplex with local corners L and density
// gradient g: the neighbour across it has gradient gj, density rj at the
// facet's corner `a` (a local corner of this simplex, a != m), and lies on
// the same side of the facet (sigma = +1) or the other (-1).
SP_HD inline void fuse_facet(FacetFuse &fz, int m, const Local<double> &L, D3 g, int a, D3 gj, double rj, int sigma)
{
    const double sg = (double)sigma;
    fz.mode[m] = FACET_FUSED;
    fz.G[m] = g + sg * gj;
    fz.xr[m] = d3(L.v[a].x, L.v[a].y, L.v[a].z);
    fz.R[m] = L.v[a].r + sg * rj;
}

// Projection of one simplex (local cell coordinates, as set up for the
// clipping path) by corner sums; dep(ix, iy, iz, value) receives each term
// sum at local cell indices, in cell-volume units.  Returns 1 when the
// simplex was not summed (its bounding box holds more than 2^24 cells), 0
// otherwise.
// (Inlined at every call, so that a caller passing no fusion data compiles
// to the plain sums.)
template <typename Dep>
SP_HD __attribute__((always_inline)) inline int corner_project(const Local<double> &L, Dep &dep,
                                                                const FacetFuse *fz = nullptr)
{
    D3 v[4];
    double r[4];
    for (int a = 0; a < 4; ++a) {
        v[a] = d3(L.v[a].x, L.v[a].y, L.v[a].z);
        r[a] = L.v[a].r;
    }
    const D3 g = corner_gradient(L);
    D3 lo = v[0], hi = v[0];
    for (int a = 1; a < 4; ++a) {
        lo = d3(fmin(lo.x, v[a].x), fmin(lo.y, v[a].y), fmin(lo.z, v[a].z));
        hi = d3(fmax(hi.x, v[a].x), fmax(hi.y, v[a].y), fmax(hi.z, v[a].z));
    }
    if (!corner_box_ok(L)) return 1;

    // origin of the piece in cell (cx, cy, cz), and the density there: the
    // cell's centre when terms are fused with a neighbour's (both must use
    // the same origin), else the point of the bounding box nearest to it
    const bool cell_origin = fz && fz->cell_origin;
    auto origin = [&](int cx, int cy, int cz) {
        if (cell_origin) return d3(cx + 0.5, cy + 0.5, cz + 0.5);
        return d3(fmin(fmax(cx + 0.5, lo.x), hi.x), fmin(fmax(cy + 0.5, lo.y), hi.y), fmin(fmax(cz + 0.5, lo.z), hi.z));
    };
    auto rho_at = [&](D3 X) { return r[0] + dot(g, X - v[0]); };
    auto deposit = [&](int cx, int cy, int cz, D3 X, const D3 *t, const D3 *b, const int (*fe)[2], const int *mf) {
        const D3 o = origin(cx, cy, cz);
        const double s = vertex_terms(X - o, rho_at(o), g, t, b, fe, mf, fz, o);
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
    // which side of the plane through corners (i, j, k) of facet m the
    // opposite corner lies on (the simplex is not flat: decided in FP64)
    int in_side[4];
    for (int m = 0; m < 4; ++m) {
        const int i = (m + 1) & 3, j = (m + 2) & 3, k = (m + 3) & 3;
        in_side[m] = sgn(dot(v[m] - v[i], cross(v[j] - v[i], v[k] - v[i])));
    }

    // A: every simplex corner, in its own cell (a corner on a grid plane lies
    // above the perturbed plane); facet k of the corner's cone is the simplex
    // facet opposite the corner's edge k
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int o3[3], n = 0;
        for (int k = 0; k < 4; ++k)
            if (k != a) o3[n++] = k;
        D3 t[3], b[3];
        int fe[3][2], mf[3];
        for (int k = 0; k < 3; ++k) {
            t[k] = unit(v[o3[k]] - v[a]);
            b[k] = nf[o3[k]];  // the facet without o3[k] holds the other two edges
            mf[k] = o3[k];
            fe[k][0] = (k + 1) % 3;
            fe[k][1] = (k + 2) % 3;
        }
        deposit((int)floor(v[a].x), (int)floor(v[a].y), (int)floor(v[a].z), v[a], t, b, fe, mf);
    }

    // B: every edge through every (perturbed) grid plane it crosses: the
    // planes c with exactly one end below c, i.e. min < c <= max; the
    // crossing point is a vertex of the pieces on both sides of the plane
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
                for (int c = (int)floor(l) + 1; (double)c <= h; ++c) {
                    const double tt = ((double)c - pa) / (pb - pa);
                    D3 p = v[a] + tt * (v[bq] - v[a]);
                    if (d == 0) p.x = c; else if (d == 1) p.y = c; else p.z = c;
                    const D3 ed = axis(d, 1.0);
                    D3 u1 = unit(cross(n1, ed));
                    if (dot(u1, n2) < 0.0) u1 = -1.0 * u1;
                    D3 u2 = unit(cross(n2, ed));
                    if (dot(u2, n1) < 0.0) u2 = -1.0 * u2;
                    const D3 up = pb > pa ? unit(v[bq] - v[a]) : unit(v[a] - v[bq]);
                    int cell[3];
                    for (int q = 0; q < 3; ++q)
                        cell[q] = q == d ? c : sos_edge_cell(v[a], v[bq], d, q, c, comp(p, q));
                    for (int side = 0; side < 2; ++side) {
                        const double sg = side == 0 ? 1.0 : -1.0;
                        const D3 t[3] = {sg * up, u1, u2};
                        const D3 b[3] = {n1, n2, axis(d, sg)};
                        const int fe[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                        const int mf[3] = {m2, m1, -1};
                        int cs[3] = {cell[0], cell[1], cell[2]};
                        cs[d] = side == 0 ? c : c - 1;
                        deposit(cs[0], cs[1], cs[2], p, t, b, fe, mf);
                    }
                }
            }
        }
    }

    // C: every facet through every (perturbed) grid line it crosses; the
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
            // orientation of the perturbed line (j - e_d1, k - e_d2) against
            // the projected edge p -> q: the exact sign, or on a tie the first
            // term of the perturbation (the lower axis index first)
            auto orient = [&](double px, double py, double qx, double qy, int j, int k) {
                const int s0 = sign_det2(qx, px, qy, py, (double)j, px, (double)k, py);
                // (qx - px)(k - py) - (qy - py)(j - px); the line moves by -(e_d1, e_d2):
                // d/de_d1 = +(qy - py), d/de_d2 = -(qx - px)
                if (s0) return s0;
                const int s1 = sgn(qy - py), s2 = -sgn(qx - px);
                return d1 < d2 ? (s1 ? s1 : s2) : (s2 ? s2 : s1);
            };
            for (int j = (int)floor(l1) + 1; (double)j <= h1; ++j) {
                for (int k = (int)floor(l2) + 1; (double)k <= h2; ++k) {
                    const int o1 = orient(ax, ay, bx, by, j, k);
                    const int o2 = orient(bx, by, cxx, cyy, j, k);
                    const int o3 = orient(cxx, cyy, ax, ay, j, k);
                    if (!((o1 > 0 && o2 > 0 && o3 > 0) || (o1 < 0 && o2 < 0 && o3 < 0))) continue;
                    const double qd = comp(v[ia], d) - (comp(nF, d1) * (j - ax) + comp(nF, d2) * (k - ay)) / nd;
                    D3 q = axis(d, qd) + axis(d1, (double)j) + axis(d2, (double)k);
                    // cell along d: the largest i with the crossing at or
                    // above the perturbed plane x_d = i, from the side of
                    // the grid point (i at d, j, k) of the facet's plane
                    // (the sign of the d component of (b - a) x (c - a): nF is
                    // that normal turned toward the opposite corner)
                    const int sn = (nd > 0.0 ? 1 : -1) * in_side[m];
                    auto above = [&](int i) {
                        const D3 w = axis(d, (double)i) + axis(d1, (double)j) + axis(d2, (double)k);
                        // crossing - (i - e_d) has the sign of -side(w - e) . n / n_d
                        return -sos_side(w, v[ib], v[ic], v[ia]) * sn > 0;
                    };
                    int cd = (int)floor(qd);
                    while (!above(cd)) --cd;
                    while (above(cd + 1)) ++cd;
                    const D3 tl = axis(d, nd > 0.0 ? 1.0 : -1.0);
                    const D3 w1r = unit(cross(nF, axis(d1, 1.0)));
                    const D3 w2r = unit(cross(nF, axis(d2, 1.0)));
                    for (int s1 = 0; s1 < 2; ++s1) {
                        for (int s2 = 0; s2 < 2; ++s2) {
                            const D3 w1 = ((comp(w1r, d2) > 0.0) == (s2 == 1)) ? w1r : -1.0 * w1r;
                            const D3 w2 = ((comp(w2r, d1) > 0.0) == (s1 == 1)) ? w2r : -1.0 * w2r;
                            const D3 t[3] = {tl, w1, w2};
                            const D3 b[3] = {nF, axis(d1, s1 ? 1.0 : -1.0), axis(d2, s2 ? 1.0 : -1.0)};
                            const int fe[3][2] = {{1, 2}, {0, 1}, {0, 2}};
                            const int mf[3] = {m, -1, -1};
                            int cell[3];
                            cell[d] = cd;
                            cell[d1] = j - 1 + s1;
                            cell[d2] = k - 1 + s2;
                            deposit(cell[0], cell[1], cell[2], q, t, b, fe, mf);
                        }
                    }
                }
            }
        }
    }

    // D: every (perturbed) grid point inside the simplex, a corner of its
    // eight cells: lo < w <= hi on every axis, and on the simplex's side of
    // all four facet planes
    const int x0 = (int)floor(lo.x) + 1, y0 = (int)floor(lo.y) + 1, z0 = (int)floor(lo.z) + 1;
    for (int z = z0; (double)z <= hi.z; ++z) {
        for (int y = y0; (double)y <= hi.y; ++y) {
            for (int x = x0; (double)x <= hi.x; ++x) {
                const D3 w = d3(x, y, z);
                bool in = true;
                for (int m = 0; m < 4 && in; ++m) {
                    const int i = (m + 1) & 3, j = (m + 2) & 3, k = (m + 3) & 3;
                    in = sos_side(w, v[j], v[k], v[i]) == in_side[m];
                }
                if (!in) continue;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
                    const D3 t[3] = {axis(0, dx ? -1.0 : 1.0), axis(1, dy ? -1.0 : 1.0), axis(2, dz ? -1.0 : 1.0)};
                    const D3 b[3] = {t[0], t[1], t[2]};  // the face across axis k holds the other two edges
                    const int fe[3][2] = {{1, 2}, {0, 2}, {0, 1}};
                    const int mf[3] = {-1, -1, -1};
                    deposit(x - dx, y - dy, z - dz, w, t, b, fe, mf);
                }
            }
        }
    }
    return 0;
}

}  // namespace sp
