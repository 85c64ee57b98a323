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
// sum at local cell indices, in cell-volume units.  Returns 1 when the
// simplex was not summed (its bounding box holds more than 2^24 cells), 0
// otherwise.
template <typename Dep>
SP_HD inline int corner_project(const Local<double> &L, Dep &dep)
{
    D3 v[4];
    double r[4];
    for (int a = 0; a < 4; ++a) {
        v[a] = d3(L.v[a].x, L.v[a].y, L.v[a].z);
        r[a] = L.v[a].r;
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
    // more than 2^24 cells is not summed (reported)
    if ((floor(hi.x) - floor(lo.x) + 1.0) * (floor(hi.y) - floor(lo.y) + 1.0) * (floor(hi.z) - floor(lo.z) + 1.0) >
        16777216.0)
        return 1;

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
        int fe[3][2];
        for (int k = 0; k < 3; ++k) {
            t[k] = unit(v[o3[k]] - v[a]);
            b[k] = nf[o3[k]];  // the facet without o3[k] holds the other two edges
            fe[k][0] = (k + 1) % 3;
            fe[k][1] = (k + 2) % 3;
        }
        deposit((int)floor(v[a].x), (int)floor(v[a].y), (int)floor(v[a].z), v[a], t, b, fe);
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
                        int cs[3] = {cell[0], cell[1], cell[2]};
                        cs[d] = side == 0 ? c : c - 1;
                        deposit(cs[0], cs[1], cs[2], p, t, b, fe);
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
                            int cell[3];
                            cell[d] = cd;
                            cell[d1] = j - 1 + s1;
                            cell[d2] = k - 1 + s2;
                            deposit(cell[0], cell[1], cell[2], q, t, b, fe);
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
                    deposit(x - dx, y - dy, z - dz, w, t, b, fe);
                }
            }
        }
    }
    return 0;
}

}  // namespace sp
