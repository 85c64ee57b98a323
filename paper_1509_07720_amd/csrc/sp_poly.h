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
#include <math.h>
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

// Reciprocal used by the cut: the hardware reciprocal in FP32 (about one
// ulp; both sides of a cut call the same function with the same operands,
// so the shared points stay bit-identical), an exact division in FP64.
SP_HD inline float sp_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
// FP64: the hardware reciprocal estimate refined by two Newton-Raphson
// steps (r <- r + r(1 - x r)), each doubling the number of correct bits;
// within a few ulp, several instructions shorter than a correctly rounded
// division.  Only used for edge-plane intersections, where both sides of a
// cut call the same function.
SP_HD inline double sp_rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
SP_HD inline float sp_fmin(float a, float b) { return fminf(a, b); }
SP_HD inline float sp_fmax(float a, float b) { return fmaxf(a, b); }
SP_HD inline double sp_fmin(double a, double b) { return fmin(a, b); }
SP_HD inline double sp_fmax(double a, double b) { return fmax(a, b); }

// Point where segment (a, b) meets the plane x_ax = c, for a strictly below
// and b at or above the plane.  The interpolation starts from the nearer end
// (halving the rounding of the long-edge case); the coordinate along ax is
// set to c exactly.  Always called as isect(lower, upper), so the two sides
// of a cut get bit-identical points.
template <typename T>
SP_HD inline V4<T> isect(const V4<T> &a, const V4<T> &b, int ax, T c)
{
    T ca = comp(a, ax), cb = comp(b, ax);
    T rd = sp_rcp(cb - ca);
    T ta = (c - ca) * rd;
    bool from_a = ta <= T(0.5);
    const V4<T> &s = from_a ? a : b;
    const V4<T> &e = from_a ? b : a;
    T t = from_a ? ta : (cb - c) * rd;
    V4<T> q;
    q.x = s.x + t * (e.x - s.x);
    q.y = s.y + t * (e.y - s.y);
    q.z = s.z + t * (e.z - s.z);
    q.r = s.r + t * (e.r - s.r);
    set_comp(q, ax, c);
    return q;
}

// neighbour word: three slot indices of B bits each (B >= 5: at most 32
// slots).  FP32 polytopes use B = 5 (15 bits, stored as 16-bit words);
// FP64 ones B = 8, whose byte fields the hardware extracts and inserts
// without a separate bit-field instruction.
template <int B>
SP_HD inline int nbr(uint32_t nb, int i)
{
    return (int)((nb >> (B * i)) & ((1u << B) - 1u));
}
template <int B>
SP_HD inline uint32_t set_nbr(uint32_t nb, int i, int v)
{
    return (nb & ~(((1u << B) - 1u) << (B * i))) | ((uint32_t)v << (B * i));
}
template <int B>
SP_HD inline int slot_of(uint32_t nb, int v)
{
    return nbr<B>(nb, 0) == v ? 0 : (nbr<B>(nb, 1) == v ? 1 : 2);
}
template <int B>
SP_HD inline uint32_t pack3(int a, int b, int c)
{
    return (uint32_t)a | ((uint32_t)b << B) | ((uint32_t)c << (2 * B));
}
SP_HD inline int lowbit(uint32_t m) { return __builtin_ctz(m); }

// A polytope vertex as the walks hold it in registers: position and the
// packed neighbour word (in LDS the two live in separate arrays, below).
// The density is not stored per vertex: over a simplex it
// is an affine function of position (set once per simplex in the polytope),
// evaluated where an integral needs it.
template <typename T>
struct NbBits;
template <>
struct NbBits<float> {
    using type = uint32_t;
};
template <>
struct NbBits<double> {
    using type = uint64_t;
};

template <typename T>
struct alignas(sizeof(T) * 4) S4 {
    T x, y, z;
    typename NbBits<T>::type nb;
};
static_assert(sizeof(S4<float>) == sizeof(V4<float>) && sizeof(S4<double>) == sizeof(V4<double>),
              "polytope slots and polygon vertices share one LDS buffer");

// In LDS a polytope keeps its positions (3 T) and its neighbour words in
// two arrays: 12 + 2 bytes a slot in FP32 (12 resident waves per CU instead
// of 11 with 16-byte records) and 24 + 4 in FP64 (6 instead of 5 with
// 32-byte records; 16-bit words measured 3 % slower there).
template <typename T>
struct P3T {
    T x, y, z;
};
template <typename T>
struct NbStore;
template <>
struct NbStore<float> {
    using type = uint16_t;
    static constexpr int bits = 5;
};
template <>
struct NbStore<double> {
    using type = uint32_t;
    static constexpr int bits = 8;
};

// Point where segment (a, b) meets the plane x_ax = c, for a strictly below
// and b at or above the plane; the same rule as isect (nearer end, exact
// coordinate along ax), positions only.
template <typename T>
SP_HD inline S4<T> isect3(const S4<T> &a, const S4<T> &b, int ax, T c)
{
    T ca = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
    T cb = ax == 0 ? b.x : (ax == 1 ? b.y : b.z);
    T rd = sp_rcp(cb - ca);
    T ta = (c - ca) * rd;
    bool from_a = ta <= T(0.5);
    const S4<T> &s = from_a ? a : b;
    const S4<T> &e = from_a ? b : a;
    T t = from_a ? ta : (cb - c) * rd;
    S4<T> q;
    q.x = ax == 0 ? c : s.x + t * (e.x - s.x);
    q.y = ax == 1 ? c : s.y + t * (e.y - s.y);
    q.z = ax == 2 ? c : s.z + t * (e.z - s.z);
    q.nb = 0;
    return q;
}

// Gradient of the affine density through the four corner values of a
// tetrahedron: g solves g . (v_k - v_0) = r_k - r_0 (Cramer's rule in FP64
// on the exact differences of the corner data; 0 for a flat tetrahedron).
template <typename T>
SP_HD inline void density_gradient(const V4<T> *v, double *gd)
{
    double e[3][3], dr[3];
    for (int k = 0; k < 3; ++k) {
        e[k][0] = (double)v[k + 1].x - (double)v[0].x;
        e[k][1] = (double)v[k + 1].y - (double)v[0].y;
        e[k][2] = (double)v[k + 1].z - (double)v[0].z;
        dr[k] = (double)v[k + 1].r - (double)v[0].r;
    }
    double c[3][3];  // c[k] = e[k+1] x e[k+2]
    for (int k = 0; k < 3; ++k) {
        const double *a = e[(k + 1) % 3], *b = e[(k + 2) % 3];
        c[k][0] = a[1] * b[2] - a[2] * b[1];
        c[k][1] = a[2] * b[0] - a[0] * b[2];
        c[k][2] = a[0] * b[1] - a[1] * b[0];
    }
    const double det = e[0][0] * c[0][0] + e[0][1] * c[0][1] + e[0][2] * c[0][2];
    const double inv = det != 0.0 ? 1.0 / det : 0.0;
    for (int d = 0; d < 3; ++d) gd[d] = (dr[0] * c[0][d] + dr[1] * c[1][d] + dr[2] * c[2][d]) * inv;
}

// Vertex storage with a stride: on the GPU each lane's polytope is spread
// over LDS with stride = lanes per block, so that lanes touching the same
// slot hit consecutive words.  Slots in use are marked in `live`; a cut
// writes its new vertices into slots that were free before it and frees the
// removed ones, so vertices never move and neighbour indices never need
// renumbering.
template <typename T, int MAXV, int STRIDE>
struct Poly3 {
    static_assert(MAXV <= 32, "vertex masks are 32-bit");
    static constexpr uint32_t SLOTS = MAXV == 32 ? 0xffffffffu : ((1u << MAXV) - 1u);
    using NbW = typename NbStore<T>::type;
    static constexpr int NB = NbStore<T>::bits;
    P3T<T> *pp;      // positions
    NbW *pn;         // neighbour words
    uint32_t live;
    // density rho(q) = r0 + g . (q - o) of the simplex being swept; gd is
    // the gradient in double precision (for the one evaluation per piece
    // that spans the whole simplex), g the same in T.  Every evaluation is
    // clamped to [rlo, rhi], the range of the corner values: exact values
    // inside the simplex never leave it, and for a nearly flat simplex (a
    // huge gradient across it) the clamp bounds the effect of points that
    // rounding puts off its plane.
    double r0, gd[3];
    T g[3];
    T o[3];
    T rlo, rhi;

    SP_HD S4<T> V(int v) const
    {
        const P3T<T> q = pp[v * STRIDE];
        S4<T> r;
        r.x = q.x;
        r.y = q.y;
        r.z = q.z;
        r.nb = pn[v * STRIDE];
        return r;
    }
    SP_HD void setV(int v, const S4<T> &q)
    {
        pp[v * STRIDE] = P3T<T>{q.x, q.y, q.z};
        pn[v * STRIDE] = (NbW)q.nb;
    }
    SP_HD uint32_t N(int v) const { return pn[v * STRIDE]; }
    SP_HD void setN(int v, uint32_t x) { pn[v * STRIDE] = (NbW)x; }
    SP_HD T coord(int v, int ax) const
    {
        const T *q = reinterpret_cast<const T *>(&pp[v * STRIDE]);
        return q[ax];
    }
    SP_HD bool empty() const { return live == 0u; }

    // The affine density through the four corner values of a tetrahedron.
    SP_HD void set_density(const V4<T> *v)
    {
        double grad[3];
        density_gradient(v, grad);
        set_density(v, grad);
    }
    // The same with the gradient given (as density_gradient computes it).
    SP_HD void set_density(const V4<T> *v, const double *grad)
    {
        for (int d = 0; d < 3; ++d) {
            gd[d] = grad[d];
            g[d] = (T)gd[d];
        }
        r0 = (double)v[0].r;
        rlo = v[0].r < v[1].r ? v[0].r : v[1].r;
        rlo = v[2].r < rlo ? v[2].r : rlo;
        rlo = v[3].r < rlo ? v[3].r : rlo;
        rhi = v[0].r > v[1].r ? v[0].r : v[1].r;
        rhi = v[2].r > rhi ? v[2].r : rhi;
        rhi = v[3].r > rhi ? v[3].r : rhi;
        o[0] = v[0].x;
        o[1] = v[0].y;
        o[2] = v[0].z;
    }

    // (fmin/fmax return the other operand for a NaN, so an overflowed
    // gradient cannot poison the sums)
    SP_HD T clamp_rho(T r) const { return sp_fmin(sp_fmax(r, rlo), rhi); }

    // density at a point, in double
    SP_HD double rho_at(const S4<T> &q) const
    {
        return r0 + gd[0] * ((double)q.x - (double)o[0]) + gd[1] * ((double)q.y - (double)o[1]) +
               gd[2] * ((double)q.z - (double)o[2]);
    }

    // A positively oriented tetrahedron (det(v1-v0, v2-v0, v3-v0) > 0).
    SP_HD void init_tet(const V4<T> *v)
    {
        const uint32_t nbs[4] = {pack3<NB>(1, 3, 2), pack3<NB>(2, 3, 0), pack3<NB>(0, 3, 1), pack3<NB>(1, 2, 0)};
        for (int i = 0; i < 4; ++i) {
            S4<T> q;
            q.x = v[i].x;
            q.y = v[i].y;
            q.z = v[i].z;
            q.nb = nbs[i];
            setV(i, q);
        }
        live = 0xfu;
    }

    // The tetrahedron translated by (-dx, -dy, 0), with the density's origin
    // moved along (the gradient does not change): the sweep builds every
    // column in a frame local to it.
    SP_HD void init_tet_at(const V4<T> *v, T dx, T dy)
    {
        V4<T> w[4];
        for (int i = 0; i < 4; ++i) {
            w[i] = v[i];
            w[i].x -= dx;
            w[i].y -= dy;
        }
        init_tet(w);
        o[0] = w[0].x;
        o[1] = w[0].y;
        o[2] = w[0].z;
    }

    // Move the frame by d along ax: every slot (used or not) and the
    // density's origin.  Exact for whole cells when no coordinate changes
    // sign, as for a column shifted down to its lowest cell.
    SP_HD void shift(int ax, T d)
    {
#pragma unroll
        for (int v = 0; v < MAXV; ++v) {
            T *q = reinterpret_cast<T *>(&pp[v * STRIDE]);
            q[ax] -= d;
        }
        o[ax] -= d;
    }

    // Every slot is read (unused slots hold stale but readable values) so
    // that the loads issue back to back instead of one per loop trip; the
    // result is masked by `live`.
    SP_HD uint32_t below_mask(int ax, T c) const
    {
        uint32_t m = 0;
#pragma unroll
        for (int v = 0; v < MAXV; ++v) m |= (uint32_t)(coord(v, ax) < c) << v;
        return m & live;
    }

    SP_HD void range(int ax, T &mn, T &mx) const
    {
        const T c0 = coord(lowbit(live), ax);
        mn = mx = c0;
#pragma unroll
        for (int v = 0; v < MAXV; ++v) {
            const T c = coord(v, ax);
            const bool in = (live >> v) & 1u;
            mn = in && c < mn ? c : mn;
            mx = in && c > mx ? c : mx;
        }
    }

    // Keep the part with x_ax >= c (keep_upper) or x_ax < c.  Returns false
    // when the vertex capacity would be exceeded or the graph is not a valid
    // polytope graph (the polytope is then left unusable).
    SP_HD bool clip(int ax, T c, bool keep_upper) { return clip_classified(ax, c, keep_upper, below_mask(ax, c)); }

    // The same with the live vertices below the plane already known.
    SP_HD bool clip_classified(int ax, T c, bool keep_upper, uint32_t below)
    {
        uint32_t keep = keep_upper ? (live & ~below) : below;
        if (keep == live) return true;
        if (keep == 0u) {
            live = 0u;
            return true;
        }
        uint32_t gone = live & ~keep;
        uint32_t freem = ~live & SLOTS;
        uint32_t fresh = 0u;
        // removed vertices with no kept neighbour are never read again: their
        // slots are free before any new vertex is placed, which keeps the
        // peak slot count at about the larger of the two polytopes' sizes
        {
            uint32_t inner = 0u;
            for (uint32_t w = gone; w; w &= w - 1u) {
                const int x = lowbit(w);
                const uint32_t nbx = N(x);
                if (!(((keep >> nbr<NB>(nbx, 0)) | (keep >> nbr<NB>(nbx, 1)) | (keep >> nbr<NB>(nbx, 2))) & 1u)) inner |= 1u << x;
            }
            freem |= inner;
            gone &= ~inner;
        }
        // one new vertex per edge between a removed and a kept vertex; the
        // removed side is usually the smaller one (the piece being cut off).
        // A removed vertex is dead once its own edges are done (its position
        // and neighbours are held in registers and no kept vertex refers to
        // it any more), so its slot takes its first new vertex -- the kept
        // neighbour's list then needs no edit -- or returns to the free pool.
        for (uint32_t w = gone; w; w &= w - 1u) {
            const int x = lowbit(w);
            const S4<T> px = V(x);
            const uint32_t nbx = (uint32_t)px.nb;
            // the three neighbours are read together up front
            const int v3[3] = {nbr<NB>(nbx, 0), nbr<NB>(nbx, 1), nbr<NB>(nbx, 2)};
            const S4<T> pv3[3] = {V(v3[0]), V(v3[1]), V(v3[2])};
            // straight-line code with selects over the three neighbours (the
            // stores are the only conditional steps), so that the lanes of a
            // wave stay in step; running out of slots is reported after them
            bool reused = false, full = false;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int v = v3[i];
                const bool kv = (keep >> v) & 1u;
                const bool own = kv && !reused;          // first new vertex: the removed vertex's slot
                const bool other = kv && reused;         // later ones: a free slot
                const bool ok = !(other && freem == 0u);
                full = full || !ok;
                // (bit 31 keeps lowbit defined when no slot is free; u is then unused)
                const int u = own ? x : lowbit(freem | 0x80000000u);
                freem = other && ok ? (freem & (freem - 1u)) : freem;
                reused = reused || kv;
                fresh |= kv && ok ? (1u << u) : 0u;
                // (unused, and possibly not finite, when v is not kept)
                S4<T> q = keep_upper ? isect3(px, pv3[i], ax, c) : isect3(pv3[i], px, ax, c);
                q.nb = pack3<NB>(v, v, v);
                if (kv && ok) setV(u, q);
                if (other && ok) {
                    const uint32_t nbv = N(v);
                    setN(v, set_nbr<NB>(nbv, slot_of<NB>(nbv, x), u));
                }
            }
            if (full) return false;
            if (!reused) freem |= 1u << x;
        }
        // link the new vertices around the cap: from each one, walk its
        // facet through kept vertices to the next new vertex.  One flat loop
        // over all walk steps keeps the lanes of a wave in step.
        uint32_t todo = fresh;
        int u = lowbit(todo);
        int prev = u, cur = nbr<NB>(N(u), 0);
        // (the step bound, reported after the loop, catches a corrupted graph)
        for (int guard = 0; todo && guard <= 4 * MAXV * MAXV; ++guard) {
            uint32_t nbc = N(cur);
            int j = slot_of<NB>(nbc, prev);
            int nxt = nbr<NB>(nbc, (j + 1) % 3);
            prev = cur;
            cur = nxt;
            if ((fresh >> cur) & 1u) {
                setN(u, set_nbr<NB>(N(u), 2, cur));
                setN(cur, set_nbr<NB>(N(cur), 1, u));
                todo &= todo - 1u;
                // the next new vertex (u itself again when none is left)
                u = todo ? lowbit(todo) : u;
                prev = u;
                cur = nbr<NB>(N(u), 0);
            }
        }
        if (todo) return false;
        live = keep | fresh;
        return true;
    }

    // Integral of the density over the part below x_ax = c (or over the
    // whole polytope when whole is true).  Returns 6*volume in s6 and
    // 24*integral in s24.  Returns false if the walk does not close (a
    // corrupted graph).
    //
    // below_out (optional): the live vertices below the plane (when whole is
    // false), for a cut at the same plane.
    SP_HD bool integrate_below(int ax, T c, bool whole, T &s6, T &s24, uint32_t *below_out = nullptr) const
    {
        s6 = T(0);
        s24 = T(0);
        uint32_t below = whole ? live : below_mask(ax, c);
        if (below_out) *below_out = below;
        // nothing below (below is part of live, so also no polytope): the
        // walk below takes no step and the sums stay zero; the slot indices
        // read meanwhile stay valid
        const bool none = below == 0u;
        if (below == live) whole = true;
        S4<T> A = V(live ? lowbit(live) : 0);
        if (!whole) {
            // a below vertex with a neighbour at or above the plane (one
            // exists, since below is neither empty nor every live vertex);
            // the three neighbours are tested with selects
            for (uint32_t w = below; w; w &= w - 1u) {
                const int v = lowbit(w);
                const uint32_t nbv = N(v);
                const int x0 = nbr<NB>(nbv, 0), x1 = nbr<NB>(nbv, 1), x2 = nbr<NB>(nbv, 2);
                const bool o0 = !((below >> x0) & 1u), o1 = !((below >> x1) & 1u), o2 = !((below >> x2) & 1u);
                if (o0 || o1 || o2) {
                    A = isect3(V(v), V(o0 ? x0 : (o1 ? x1 : x2)), ax, c);
                    break;
                }
            }
        }
        // density at the apex in double, then at each corner q as
        // rho(A) + g . (q - A)
        const T rA = clamp_rho((T)rho_at(A));
        // only facets holding a vertex below the plane contribute; each is
        // reached from a directed edge leaving one of its below vertices
        uint32_t un0 = live, un1 = live, un2 = live;
        int vs = 0, vcur = 0, pc = 0, cnt = 0;
        uint32_t ncur = 0u;
        bool ba = false;
        S4<T> a;
        T e0x = 0, e0y = 0, e0z = 0, epx = 0, epy = 0, epz = 0, rf = 0, rp = 0;
        // one point of the facet polygon, if valid: the fan triangle it
        // closes with the first and the previous point.  Straight-line code
        // with selects (every lane of a wave runs it whether its point is
        // valid or not), so that the walk carries no nested branches.
        auto acc = [&](const S4<T> &q, bool valid) {
            const T ex = q.x - A.x, ey = q.y - A.y, ez = q.z - A.z;
            const T rq = clamp_rho(rA + (g[0] * ex + g[1] * ey + g[2] * ez));
            const T cx = ey * epz - ez * epy;
            const T cy = ez * epx - ex * epz;
            const T cz = ex * epy - ey * epx;
            const T d = e0x * cx + e0y * cy + e0z * cz;
            const bool tri = valid && cnt >= 2;
            s6 += tri ? d : T(0);
            s24 += tri ? d * (rA + rf + rp + rq) : T(0);
            const bool first = valid && cnt == 0;
            e0x = first ? ex : e0x;
            e0y = first ? ey : e0y;
            e0z = first ? ez : e0z;
            rf = first ? rq : rf;
            epx = valid ? ex : epx;
            epy = valid ? ey : epy;
            epz = valid ? ez : epz;
            rp = valid ? rq : rp;
            cnt += valid ? 1 : 0;
        };
        // the first facet: from the lowest below vertex through its slot 0
        vs = vcur = none ? 0 : lowbit(below);
        a = V(vcur);
        ncur = (uint32_t)a.nb;
        ba = true;
        const int steps = none ? 0 : 3 * __builtin_popcount(live);
        bool done = false;
        // (three steps per trip: the walk state rotates through registers
        // instead of being copied at every back-edge; 44.5 -> 43.2 ms on the
        // soup, 2 and 4 measured in between)
#pragma unroll 3
        for (int it = 0; it < steps && !done; ++it) {
            const uint32_t bit = 1u << vcur;
            un0 &= pc == 0 ? ~bit : ~0u;
            un1 &= pc == 1 ? ~bit : ~0u;
            un2 &= pc == 2 ? ~bit : ~0u;
            // the neighbour word of the current vertex comes with its
            // position, so each step waits for one LDS read
            const int vnext = nbr<NB>(ncur, pc);
            const S4<T> b = V(vnext);
            const uint32_t nnext = (uint32_t)b.nb;
            const bool bb = (below >> vnext) & 1u;
            acc(a, ba);
            // the crossing point of an edge across the plane, always from its
            // lower end; unused (and possibly not finite) on other edges
            S4<T> lo, hi;  // (selected by value: a conditional reference would go to scratch memory)
            lo.x = ba ? a.x : b.x;
            lo.y = ba ? a.y : b.y;
            lo.z = ba ? a.z : b.z;
            hi.x = ba ? b.x : a.x;
            hi.y = ba ? b.y : a.y;
            hi.z = ba ? b.z : a.z;
            acc(isect3(lo, hi, ax, c), ba != bb);
            const int np = slot_of<NB>(nnext, vcur);
            // A facet closes when the walk is back at its first vertex; the
            // next one starts at the lowest below vertex with an edge not yet
            // walked, and when there is none every facet is done.  The start
            // is chosen with selects and its vertex read on every step (from
            // a live slot), so that the walk carries no nested branch.
            const bool closed = vnext == vs;
            const uint32_t any = (un0 | un1 | un2) & below;
            const int vn = any ? lowbit(any) : vnext;
            const S4<T> an = V(vn);
            done = closed && any == 0u;
            const int pn = ((un0 >> vn) & 1u) ? 0 : (((un1 >> vn) & 1u) ? 1 : 2);
            vs = closed ? vn : vs;
            pc = closed ? pn : (np == 2 ? 0 : np + 1);
            vcur = closed ? vn : vnext;
            cnt = closed ? 0 : cnt;
            a.x = closed ? an.x : b.x;
            a.y = closed ? an.y : b.y;
            a.z = closed ? an.z : b.z;
            ncur = closed ? (uint32_t)an.nb : nnext;
            ba = closed || bb;  // a facet starts at a below vertex
        }
        return done || none;
    }
};

} // namespace sp
