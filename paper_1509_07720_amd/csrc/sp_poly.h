// sp_poly.h -- clip polytopes for the exact simplex-to-grid projection.
//
// A convex polytope is held as a vertex graph of degree three (every vertex of
// a tetrahedron cut by planes in general position has exactly three edges;
// degenerate cuts keep degree three by producing zero-length edges).  Each
// vertex stores its position, the density value carried along (linear
// interpolation of the simplex's vertex densities), and the indices of its
// three neighbours ordered counter-clockwise as seen from outside.  This is
// the vertex-graph representation of Powell & Abel's r3d (J. Comput. Phys.
// 2015), written here for one polytope per GPU lane.
//
// Cutting by an axis-aligned plane x_ax = c is exact in its classification
// (a vertex is "below" iff its stored coordinate is < c, ties go up: the
// half-open cells [k, k+1) of the simulation-of-simplicity convention,
// Section 3.3 eq. eq_sos).  Both sides of a cut use the very same
// intersection points (computed by one function, from the lower end toward
// the upper end), so a cut moves mass between its sides but never creates or
// loses any (Section 3.3's consistency requirement, met by construction).
//
// The integral of the linear density over a polytope (or over its part below
// a plane) is taken as a fan of tetrahedra from an apex: every facet is
// walked once, each facet polygon is fanned from its first vertex, and each
// fan triangle with the apex forms a tetrahedron whose integral is its
// volume times the mean of its four vertex densities (Appendix C).
#pragma once
#include <stdint.h>

#ifndef SP_HD
#if defined(__HIPCC__)
#define SP_HD __host__ __device__
#else
#define SP_HD
#endif
#endif

namespace sp {

template <typename T>
struct alignas(sizeof(T) * 4) V4 {
    T x, y, z, r;
};

template <typename T>
SP_HD inline T comp(const V4<T> &p, int ax)
{
    return ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
}

template <typename T>
SP_HD inline void set_comp(V4<T> &p, int ax, T v)
{
    if (ax == 0) p.x = v;
    else if (ax == 1) p.y = v;
    else p.z = v;
}

// Point where segment (a, b) meets the plane x_ax = c, for a strictly below
// and b at or above the plane.  The interpolation starts from the nearer end
// (halving the rounding of the long-edge case); the coordinate along ax is
// set to c exactly.  Always called as isect(lower, upper), so the two sides
// of a cut get bit-identical points.
template <typename T>
SP_HD inline V4<T> isect(const V4<T> &a, const V4<T> &b, int ax, T c)
{
    T ca = comp(a, ax), cb = comp(b, ax);
    T den = cb - ca;
    T ta = (c - ca) / den;
    V4<T> q;
    if (ta <= T(0.5)) {
        q.x = a.x + ta * (b.x - a.x);
        q.y = a.y + ta * (b.y - a.y);
        q.z = a.z + ta * (b.z - a.z);
        q.r = a.r + ta * (b.r - a.r);
    } else {
        T tb = (cb - c) / den;
        q.x = b.x + tb * (a.x - b.x);
        q.y = b.y + tb * (a.y - b.y);
        q.z = b.z + tb * (a.z - b.z);
        q.r = b.r + tb * (a.r - b.r);
    }
    set_comp(q, ax, c);
    return q;
}

SP_HD inline int nbr(uint32_t nb, int i) { return (int)((nb >> (8 * i)) & 0xffu); }
SP_HD inline uint32_t set_nbr(uint32_t nb, int i, int v)
{
    return (nb & ~(0xffu << (8 * i))) | ((uint32_t)v << (8 * i));
}
SP_HD inline int slot_of(uint32_t nb, int v)
{
    return nbr(nb, 0) == v ? 0 : (nbr(nb, 1) == v ? 1 : 2);
}
SP_HD inline uint32_t pack3(int a, int b, int c) { return (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16); }

// Vertex storage with a stride: on the GPU each lane's polytope is spread
// over LDS with stride = lanes per block, so that lanes touching the same
// slot hit consecutive words.
template <typename T, int MAXV, int STRIDE>
struct Poly3 {
    static_assert(MAXV <= 32, "vertex masks are 32-bit");
    V4<T> *p;
    uint32_t *nb;
    int n;

    SP_HD V4<T> P(int v) const { return p[v * STRIDE]; }
    SP_HD void setP(int v, const V4<T> &q) { p[v * STRIDE] = q; }
    SP_HD uint32_t N(int v) const { return nb[v * STRIDE]; }
    SP_HD void setN(int v, uint32_t x) { nb[v * STRIDE] = x; }
    SP_HD T coord(int v, int ax) const
    {
        const T *q = reinterpret_cast<const T *>(&p[v * STRIDE]);
        return q[ax];
    }

    // A positively oriented tetrahedron (det(v1-v0, v2-v0, v3-v0) > 0).
    SP_HD void init_tet(const V4<T> *v)
    {
        for (int i = 0; i < 4; ++i) setP(i, v[i]);
        setN(0, pack3(1, 3, 2));
        setN(1, pack3(2, 3, 0));
        setN(2, pack3(0, 3, 1));
        setN(3, pack3(1, 2, 0));
        n = 4;
    }

    SP_HD uint32_t below_mask(int ax, T c) const
    {
        uint32_t m = 0;
        for (int v = 0; v < n; ++v) m |= (uint32_t)(coord(v, ax) < c) << v;
        return m;
    }

    // Keep the part with x_ax >= c (keep_upper) or x_ax < c.  Returns false
    // when the vertex capacity would be exceeded or the graph is not a valid
    // polytope graph (the polytope is then left unusable).
    SP_HD bool clip(int ax, T c, bool keep_upper)
    {
        const uint32_t full = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
        uint32_t below = below_mask(ax, c);
        uint32_t keep = keep_upper ? (~below & full) : below;
        if (keep == full) return true;
        if (keep == 0) {
            n = 0;
            return true;
        }
        const int n0 = n;
        int m = n0;
        for (int v = 0; v < n0; ++v) {
            if (!((keep >> v) & 1u)) continue;
            uint32_t nbv = N(v);
            bool changed = false;
            for (int i = 0; i < 3; ++i) {
                int w = nbr(nbv, i);
                if ((keep >> w) & 1u) continue;
                if (m >= MAXV) return false;
                V4<T> pv = P(v), pw = P(w);
                V4<T> q = keep_upper ? isect(pw, pv, ax, c) : isect(pv, pw, ax, c);
                setP(m, q);
                setN(m, pack3(v, v, v));
                nbv = set_nbr(nbv, i, m);
                changed = true;
                ++m;
            }
            if (changed) setN(v, nbv);
        }
        // link the new vertices around the cap: walk each one's facet through
        // kept vertices until the next new vertex
        for (int u = n0; u < m; ++u) {
            int prev = u, cur = nbr(N(u), 0);
            int guard = 0;
            for (;;) {
                uint32_t nbc = N(cur);
                int j = slot_of(nbc, prev);
                int nxt = nbr(nbc, (j + 1) % 3);
                prev = cur;
                cur = nxt;
                if (cur >= n0) break;
                if (++guard > 2 * MAXV) return false;
            }
            setN(u, set_nbr(N(u), 2, cur));
            setN(cur, set_nbr(N(cur), 1, u));
        }
        // compact: survivors are the kept old vertices then the new ones
        const int nk = __builtin_popcount(keep);
        int dst = 0;
        for (int v = 0; v < m; ++v) {
            if (v < n0 && !((keep >> v) & 1u)) continue;
            uint32_t nbv = N(v);
            uint32_t out = 0;
            for (int i = 0; i < 3; ++i) {
                int w = nbr(nbv, i);
                int wn = w < n0 ? __builtin_popcount(keep & ((1u << w) - 1u)) : nk + (w - n0);
                out |= (uint32_t)wn << (8 * i);
            }
            if (dst != v) setP(dst, P(v));
            setN(dst, out);
            ++dst;
        }
        n = dst;
        return true;
    }

    // Integral of the carried density over the part below x_ax = c (or over
    // the whole polytope when whole is true).  Returns 6*volume in s6 and
    // 24*integral in s24 (both in the polytope's coordinate units; their sign
    // is the orientation convention, positive for this vertex ordering).
    SP_HD bool integrate_below(int ax, T c, bool whole, T &s6, T &s24) const
    {
        s6 = T(0);
        s24 = T(0);
        if (n == 0) return true;
        const uint32_t full = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
        uint32_t below = whole ? full : below_mask(ax, c);
        if (below == 0) return true;
        if (below == full) whole = true;
        V4<T> A;
        if (whole) {
            A = P(0);
        } else {
            // apex: a point of the cap (any crossing edge)
            bool found = false;
            for (int v = 0; v < n && !found; ++v) {
                if (!((below >> v) & 1u)) continue;
                uint32_t nbv = N(v);
                for (int i = 0; i < 3; ++i) {
                    int w = nbr(nbv, i);
                    if (!((below >> w) & 1u)) {
                        A = isect(P(v), P(w), ax, c);
                        found = true;
                        break;
                    }
                }
            }
        }
        uint32_t mk[3] = {0u, 0u, 0u};
        for (int vs = 0; vs < n; ++vs) {
            for (int ps = 0; ps < 3; ++ps) {
                if ((mk[ps] >> vs) & 1u) continue;
                int vcur = vs, pc = ps;
                V4<T> q0, qp;
                int cnt = 0;
                V4<T> a = P(vcur);
                bool ba = (below >> vcur) & 1u;
                int guard = 0;
                for (;;) {
                    mk[pc] |= 1u << vcur;
                    uint32_t nbc = N(vcur);
                    int vnext = nbr(nbc, pc);
                    V4<T> b = P(vnext);
                    bool bb = (below >> vnext) & 1u;
                    // emitted points of this edge: a (if below), then the
                    // crossing point (if the edge crosses)
                    for (int e = 0; e < 2; ++e) {
                        V4<T> q;
                        if (e == 0) {
                            if (!ba) continue;
                            q = a;
                        } else {
                            if (ba == bb) continue;
                            q = ba ? isect(a, b, ax, c) : isect(b, a, ax, c);
                        }
                        if (cnt == 0) {
                            q0 = q;
                        } else if (cnt >= 2) {
                            // tet (A, q0, q, qp)
                            T e1x = q0.x - A.x, e1y = q0.y - A.y, e1z = q0.z - A.z;
                            T e2x = q.x - A.x, e2y = q.y - A.y, e2z = q.z - A.z;
                            T e3x = qp.x - A.x, e3y = qp.y - A.y, e3z = qp.z - A.z;
                            T d = e1x * (e2y * e3z - e2z * e3y) - e1y * (e2x * e3z - e2z * e3x) +
                                  e1z * (e2x * e3y - e2y * e3x);
                            s6 += d;
                            s24 += d * (A.r + q0.r + q.r + qp.r);
                        }
                        qp = q;
                        ++cnt;
                    }
                    if (vnext == vs) break;
                    int np = slot_of(N(vnext), vcur);
                    pc = (np + 1) % 3;
                    vcur = vnext;
                    a = b;
                    ba = bb;
                    if (++guard > 2 * MAXV) return false;
                }
            }
        }
        return true;
    }
};

} // namespace sp
