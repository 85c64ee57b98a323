// sp_wave.h -- the clip sweep with one polytope per group of 16 lanes.
//
// The FP32 3D clip kernel runs four groups of 16 lanes per wave.  A group
// sweeps one work item (a simplex, or a run of its x-slabs) and holds the
// polytopes of that sweep in LDS, one vertex per lane: every operation on a
// polytope (classify against a plane, cut, link the cap, integrate) runs on
// all its vertices at once, so the lanes of a group do the same work instead
// of each lane walking its own polytope.
//
// Polytopes are vertex graphs of degree three (as in sp_poly.h), stored
// compactly in slots 0..n-1 of a 16-slot buffer: position (x, y, z) and one
// word holding the three neighbours (4 bits each, counter-clockwise seen
// from outside) and the labels of the three faces around the vertex (4 bits
// each): face j of vertex v is the face walked when leaving v towards its
// neighbour j, i.e. the one between neighbours j-1 and j.  Labels 0-3 are
// the simplex's faces (named after the opposite corner), 4 + 2 axis + side
// the planes of the current cell (side 0: lower, 1: upper).
//
// The sweep splits, never re-clips: the simplex remainder R0 is split at the
// next x-plane into a slab R1 and the rest, R1 at the next y-plane into a
// column R2 and the rest, R2 at the next z-plane into a piece and the rest.
// Each split computes the crossing points once and builds both sides from
// them (the lower one stored or integrated, the upper one stored), so mass
// moves between sides but is never lost or doubled (Section 3.3's
// consistency requirement, met by construction).  Each polytope is kept in a
// frame local to the cell it is next cut at: after a split the upper part
// moves down by one cell along the split axis (exactly: the coordinates it
// keeps are >= 1), and a new slab or column is moved to its first cell.
//
// Precision: the remainder and the slabs (R0, R1) hold FP64 positions, the
// columns (R2) FP32 ones.  A slab's vertices lie anywhere on its cross
// section, tens of cells from any one origin for a large simplex; held in
// FP32 they would carry the rounding of that distance (about 2e-6 of a cell
// at 50 cells) into every piece.  In FP64 they reach the column exactly
// enough, and the column is written in FP32 already moved to its first cell,
// so the z sweep that makes the pieces -- most of the work, and all of the
// integration -- runs in FP32 on coordinates of a few cells.
//
// A piece's integral (Appendix C: cones from an apex over the faces, each
// face fanned into triangles) is taken edge by edge: with the apex A on the
// cutting plane and, for each face F, a point p_F of F (a crossing point of
// F when F crosses the plane, else one of its vertices), every directed
// lower edge (a -> b) of F contributes the tetrahedron (A, p_F, b, a); the
// cap and the parts of faces on the plane contribute zero volume.  The terms
// are independent, so no lane walks a face.
//
// The same source compiles for the GPU and, for tests, for the host, where
// the 16 lanes of a group run one after the other (WV_LANES blocks); code in
// one WV_LANES block never reads what another lane writes in the same block.
#pragma once
#include <math.h>
#include <stdint.h>

#include "sp_setup.h"

namespace sp {
namespace wv {

constexpr int G = 16;      // lanes per group = vertex slots per polytope
constexpr int NLAB = 10;   // face labels
constexpr int LAB_CELL = 4;

template <typename T>
struct SlotT {
    T x, y, z;
    uint32_t w;
};
using Slot = SlotT<float>;
using SlotD = SlotT<double>;

template <typename T>
struct P3T {
    T x, y, z, pad;
};
using P3 = P3T<float>;

constexpr int NBUF_D = 3;  // FP64 buffers: remainder and slab (and one being written)
constexpr int NBUF_F = 2;  // FP32 buffers: column (and its next remainder)

// LDS of one group
struct GroupLDS {
    SlotD bd[NBUF_D][G];
    Slot bf[NBUF_F][G];
    P3 rep[NLAB];       // a point of each face, for the integration
    P3 apex;            // the integration's apex
    int prevcap[G];     // cap predecessor of each new vertex
};

SP_HD inline int wnb(uint32_t w, int j) { return (int)((w >> (4 * j)) & 15u); }
SP_HD inline int wlab(uint32_t w, int j) { return (int)((w >> (12 + 4 * j)) & 15u); }
SP_HD inline uint32_t wpack(int n0, int n1, int n2, int l0, int l1, int l2)
{
    return (uint32_t)n0 | ((uint32_t)n1 << 4) | ((uint32_t)n2 << 8) | ((uint32_t)l0 << 12) | ((uint32_t)l1 << 16) |
           ((uint32_t)l2 << 20);
}
SP_HD inline int wslot(uint32_t w, int v) { return wnb(w, 0) == v ? 0 : (wnb(w, 1) == v ? 1 : 2); }
SP_HD inline int popc16(uint32_t m) { return __builtin_popcount(m & 0xffffu); }
SP_HD inline int rank16(uint32_t m, int v) { return __builtin_popcount(m & ((1u << v) - 1u)); }
template <typename T>
SP_HD inline T wcoord(const SlotT<T> &s, int ax) { return ax == 0 ? s.x : (ax == 1 ? s.y : s.z); }
template <typename T>
SP_HD inline T pcoord(const P3T<T> &s, int ax) { return ax == 0 ? s.x : (ax == 1 ? s.y : s.z); }

// Point where the edge from a (below x_ax = c) to b (at or above) meets the
// plane; the nearer end starts the interpolation, the coordinate along ax is
// c exactly.  Both lanes that see the edge call it as (lower, upper).
template <typename T>
SP_HD inline P3T<T> cross_point(const SlotT<T> &a, const SlotT<T> &b, int ax, T c)
{
    const T ca = wcoord(a, ax), cb = wcoord(b, ax);
    const T rd = sp_rcp(cb - ca);
    const T ta = (c - ca) * rd;
    const bool from_a = ta <= T(0.5);
    const SlotT<T> &s = from_a ? a : b;
    const SlotT<T> &e = from_a ? b : a;
    const T t = from_a ? ta : (cb - c) * rd;
    P3T<T> q;
    q.x = ax == 0 ? c : s.x + t * (e.x - s.x);
    q.y = ax == 1 ? c : s.y + t * (e.y - s.y);
    q.z = ax == 2 ? c : s.z + t * (e.z - s.z);
    q.pad = T(0);
    return q;
}

// ------------------------------------------------------------------------
// lanes of a group: device form and host emulation

#if defined(__HIP_DEVICE_COMPILE__)

template <typename T>
struct PL {
    T v;
    __device__ T &operator()() { return v; }
};
__device__ inline int wv_lane() { return (int)(threadIdx.x & (G - 1)); }
#define WV_LANES if (true)
__device__ inline uint32_t wv_ballot_(bool p)
{
    const uint64_t b = __ballot(p);
    return (uint32_t)(b >> (threadIdx.x & 48u)) & 0xffffu;
}
#define WV_BALLOT(expr) ::sp::wv::wv_ballot_(expr)
__device__ inline float wv_sum_(float v)
{
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    return v;
}
__device__ inline float wv_min_(float v)
{
    v = fminf(v, __shfl_xor(v, 8, 16));
    v = fminf(v, __shfl_xor(v, 4, 16));
    v = fminf(v, __shfl_xor(v, 2, 16));
    v = fminf(v, __shfl_xor(v, 1, 16));
    return v;
}
__device__ inline float wv_max_(float v)
{
    v = fmaxf(v, __shfl_xor(v, 8, 16));
    v = fmaxf(v, __shfl_xor(v, 4, 16));
    v = fmaxf(v, __shfl_xor(v, 2, 16));
    v = fmaxf(v, __shfl_xor(v, 1, 16));
    return v;
}
#define WV_SUM(expr) ::sp::wv::wv_sum_(expr)
#define WV_MIN(expr) ::sp::wv::wv_min_(expr)
#define WV_MAX(expr) ::sp::wv::wv_max_(expr)
// LDS written by some lanes of the wave and read by others: order the
// accesses (one wave per block, so the workgroup is the wave)
__device__ inline void wv_sync_()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
#define WV_SYNC() ::sp::wv::wv_sync_()

#else

extern thread_local int wv_cur_lane;
template <typename T>
struct PL {
    T v[G];
    T &operator()() { return v[wv_cur_lane]; }
};
inline int wv_lane() { return wv_cur_lane; }
#define WV_LANES for (::sp::wv::wv_cur_lane = 0; ::sp::wv::wv_cur_lane < ::sp::wv::G; ++::sp::wv::wv_cur_lane)
template <typename F>
inline uint32_t wv_ballot_h(F f)
{
    uint32_t m = 0;
    for (wv_cur_lane = 0; wv_cur_lane < G; ++wv_cur_lane) m |= (uint32_t)(f() ? 1u : 0u) << wv_cur_lane;
    return m;
}
template <typename F>
inline float wv_red_h(F f, int op)
{
    float r = 0.0f;
    for (wv_cur_lane = 0; wv_cur_lane < G; ++wv_cur_lane) {
        const float x = f();
        r = wv_cur_lane == 0 ? x : (op == 0 ? r + x : (op == 1 ? fminf(r, x) : fmaxf(r, x)));
    }
    return r;
}
#define WV_BALLOT(expr) ::sp::wv::wv_ballot_h([&]() -> bool { return (expr); })
#define WV_SUM(expr) ::sp::wv::wv_red_h([&]() -> float { return (expr); }, 0)
#define WV_MIN(expr) ::sp::wv::wv_red_h([&]() -> float { return (expr); }, 1)
#define WV_MAX(expr) ::sp::wv::wv_red_h([&]() -> float { return (expr); }, 2)
#define WV_SYNC() ((void)0)

#endif

// ------------------------------------------------------------------------
// one split

struct SplitOut {
    int nl, nu;         // vertices of the lower and upper parts (0: empty)
    bool fail;          // out of slots, or a cap that does not close
    float lmin, lmax;   // range of the lower part along the requested axis
    int lshift;         // the lower part's first cell along that axis
    float s6, s24;      // lower part: 6 x volume, 24 x integral of rho
};

// Density over the polytope's frame: rho(x) = r0 + g . x, clamped to
// [rlo, rhi] (the range of the simplex's corner values).
struct Dens {
    float r0, g[3], rlo, rhi;
    SP_HD float at(float x, float y, float z) const
    {
        const float r = r0 + (g[0] * x + g[1] * y + g[2] * z);
        return fminf(fmaxf(r, rlo), rhi);
    }
};

// Split the polytope held in qb (nq vertices) by the plane coord[ax] = c
// (c = +inf: the whole polytope is the lower part).  The lower part goes to
// lb (NULL: not stored), the upper part to ub (NULL: not stored), moved by
// -ushift along ax.  rax >= 0: the lower part's range along rax is returned,
// and the lower part is stored moved by -(its first cell along rax), the
// first cell being floor of the range's low end clamped to [0, rmax]
// (returned in o.lshift).  With integ (FP32 only), the lower part is
// integrated; the apex is a point of the piece (a crossing point when the
// plane cuts, else a vertex), so that the density there is the simplex's
// own linear value.
template <typename TQ, typename TL, typename TU>
SP_HD inline SplitOut split(GroupLDS *sh, const SlotT<TQ> *qb, int nq, int ax, TQ c, SlotT<TL> *lb, SlotT<TU> *ub,
                            TQ ushift, bool integ, int rax, int rmax, const Dens &rho)
{
    using S = SlotT<TQ>;
    using Q = P3T<TQ>;
    SplitOut o;
    o.fail = false;
    o.s6 = o.s24 = 0.0f;
    o.lmin = o.lmax = 0.0f;
    o.lshift = 0;
    PL<S> me, n0, n1, n2;
    PL<int> crs;  // bit j: the edge to neighbour j crosses the plane (this vertex below)
    PL<Q> q0, q1, q2;
    PL<int> ei0, ei1, ei2, ea0, ea1, ea2, eb0, eb1, eb2;  // own new-vertex index, walk result, predecessor
    PL<bool> below;
    WV_LANES
    {
        const int v = wv_lane();
        if (v < nq) me() = qb[v];
        below() = v < nq && wcoord(me(), ax) < c;
    }
    const uint32_t live = nq >= G ? 0xffffu : ((1u << nq) - 1u);
    const uint32_t Bb = WV_BALLOT(below());
    const uint32_t Ba = live & ~Bb;
    const int nb = popc16(Bb), na = popc16(Ba);
    WV_LANES
    {
        const int v = wv_lane();
        crs() = 0;
        if (v < nq) {
            const uint32_t w = me().w;
            n0() = qb[wnb(w, 0)];
            n1() = qb[wnb(w, 1)];
            n2() = qb[wnb(w, 2)];
            if (below()) {
                for (int j = 0; j < 3; ++j)
                    if (!((Bb >> wnb(w, j)) & 1u)) crs() |= 1 << j;
            }
        }
    }
    const uint32_t C0 = WV_BALLOT((crs() & 1) != 0);
    const uint32_t C1 = WV_BALLOT((crs() & 2) != 0);
    const uint32_t C2 = WV_BALLOT((crs() & 4) != 0);
    const int base1 = popc16(C0), base2 = base1 + popc16(C1);
    const int nnew = base2 + popc16(C2);
    o.nl = nb > 0 ? nb + nnew : 0;
    o.nu = na > 0 ? na + nnew : 0;
    if ((lb && o.nl > G) || (ub && o.nu > G)) {
        o.fail = true;
        return o;
    }
    // crossing points, own new-vertex indices, cap walks through the lower
    // vertices along the face after the crossing edge
    PL<bool> walk_ok;
    WV_LANES
    {
        const int v = wv_lane();
        walk_ok() = true;
        for (int j = 0; j < 3; ++j) {
            if (!((crs() >> j) & 1)) continue;
            const S nbj = j == 0 ? n0() : (j == 1 ? n1() : n2());
            const Q q = cross_point(me(), nbj, ax, c);
            const int e = (j == 0 ? 0 : (j == 1 ? base1 : base2)) + rank16(j == 0 ? C0 : (j == 1 ? C1 : C2), v);
            int prev = wnb(me().w, j), cur = v, e1 = -1;
            uint32_t cw = me().w;
            for (int it = 0; it < G; ++it) {
                const int k = (wslot(cw, prev) + 1) % 3;
                const int nx = wnb(cw, k);
                if (!((Bb >> nx) & 1u)) {
                    e1 = (k == 0 ? 0 : (k == 1 ? base1 : base2)) + rank16(k == 0 ? C0 : (k == 1 ? C1 : C2), cur);
                    break;
                }
                prev = cur;
                cur = nx;
                cw = qb[cur].w;
            }
            if (e1 < 0 || e1 >= nnew) walk_ok() = false;
            if (j == 0) q0() = q, ei0() = e, ea0() = e1;
            else if (j == 1) q1() = q, ei1() = e, ea1() = e1;
            else q2() = q, ei2() = e, ea2() = e1;
        }
    }
    if (WV_BALLOT(!walk_ok()) != 0u) {
        o.fail = true;
        return o;
    }
    if (nnew > 0) {
        WV_LANES { sh->prevcap[wv_lane()] = -1; }
        WV_SYNC();
        WV_LANES
        {
            if (crs() & 1) sh->prevcap[ea0()] = ei0();
            if (crs() & 2) sh->prevcap[ea1()] = ei1();
            if (crs() & 4) sh->prevcap[ea2()] = ei2();
        }
        WV_SYNC();
        PL<bool> cap_ok;
        WV_LANES
        {
            cap_ok() = true;
            if (crs() & 1) eb0() = sh->prevcap[ei0()], cap_ok() = cap_ok() && eb0() >= 0;
            if (crs() & 2) eb1() = sh->prevcap[ei1()], cap_ok() = cap_ok() && eb1() >= 0;
            if (crs() & 4) eb2() = sh->prevcap[ei2()], cap_ok() = cap_ok() && eb2() >= 0;
        }
        if (WV_BALLOT(!cap_ok()) != 0u) {
            o.fail = true;
            return o;
        }
    }
    // range of the lower part (before it is written, for its frame)
    TQ lsh = TQ(0);
    if (rax >= 0) {
        PL<float> mn, mx;
        WV_LANES
        {
            TQ a = TQ(INFINITY), b = TQ(-INFINITY);
            if (below()) a = b = wcoord(me(), rax);
            if (crs() & 1) a = fmin(a, pcoord(q0(), rax)), b = fmax(b, pcoord(q0(), rax));
            if (crs() & 2) a = fmin(a, pcoord(q1(), rax)), b = fmax(b, pcoord(q1(), rax));
            if (crs() & 4) a = fmin(a, pcoord(q2(), rax)), b = fmax(b, pcoord(q2(), rax));
            // floor is taken on the rounded-down float, so the first cell is
            // never above the lowest point
            mn() = (float)a;
            mx() = (float)b;
            if ((TQ)mn() > a) mn() = nextafterf(mn(), -INFINITY);
        }
        o.lmin = WV_MIN(mn());
        o.lmax = WV_MAX(mx());
        int f = (int)floorf(o.lmin);
        f = f > rmax ? rmax : f;
        f = f < 0 ? 0 : f;
        o.lshift = f;
        lsh = (TQ)f;
    }
    // the two parts
    WV_LANES
    {
        const int v = wv_lane();
        if (v < nq) {
            const uint32_t w = me().w;
            const bool bv = below();
            // a kept vertex's neighbour across the plane becomes the new
            // vertex on that edge
            int nbr[3];
            for (int j = 0; j < 3; ++j) {
                const int n = wnb(w, j);
                const bool bn = (Bb >> n) & 1u;
                if (bv == bn) {
                    nbr[j] = bv ? rank16(Bb, n) : rank16(Ba, n);
                } else if (bv) {
                    nbr[j] = nb + (j == 0 ? ei0() : (j == 1 ? ei1() : ei2()));
                } else {
                    const S nn = j == 0 ? n0() : (j == 1 ? n1() : n2());
                    const int k = wslot(nn.w, v);
                    const int e = (k == 0 ? 0 : (k == 1 ? base1 : base2)) + rank16(k == 0 ? C0 : (k == 1 ? C1 : C2), n);
                    nbr[j] = na + e;
                }
            }
            const uint32_t wk = wpack(nbr[0], nbr[1], nbr[2], wlab(w, 0), wlab(w, 1), wlab(w, 2));
            if (bv && lb) {
                SlotT<TL> t;
                t.x = (TL)(rax == 0 ? me().x - lsh : me().x);
                t.y = (TL)(rax == 1 ? me().y - lsh : me().y);
                t.z = (TL)(rax == 2 ? me().z - lsh : me().z);
                t.w = wk;
                lb[rank16(Bb, v)] = t;
            } else if (!bv && ub) {
                SlotT<TU> t;
                t.x = (TU)(ax == 0 ? me().x - ushift : me().x);
                t.y = (TU)(ax == 1 ? me().y - ushift : me().y);
                t.z = (TU)(ax == 2 ? me().z - ushift : me().z);
                t.w = wk;
                ub[rank16(Ba, v)] = t;
            }
            for (int j = 0; j < 3; ++j) {
                if (!((crs() >> j) & 1)) continue;
                const Q q = j == 0 ? q0() : (j == 1 ? q1() : q2());
                const int e = j == 0 ? ei0() : (j == 1 ? ei1() : ei2());
                const int e1 = j == 0 ? ea0() : (j == 1 ? ea1() : ea2());
                const int e2 = j == 0 ? eb0() : (j == 1 ? eb1() : eb2());
                const int n = wnb(w, j);
                const int la = wlab(w, j), lb_ = wlab(w, (j + 1) % 3);
                if (lb) {
                    SlotT<TL> t;
                    t.x = (TL)(rax == 0 ? q.x - lsh : q.x);
                    t.y = (TL)(rax == 1 ? q.y - lsh : q.y);
                    t.z = (TL)(rax == 2 ? q.z - lsh : q.z);
                    t.w = wpack(rank16(Bb, v), nb + e2, nb + e1, lb_, la, LAB_CELL + 2 * ax + 1);
                    lb[nb + e] = t;
                }
                if (ub) {
                    SlotT<TU> t;
                    t.x = (TU)(ax == 0 ? q.x - ushift : q.x);
                    t.y = (TU)(ax == 1 ? q.y - ushift : q.y);
                    t.z = (TU)(ax == 2 ? q.z - ushift : q.z);
                    t.w = wpack(rank16(Ba, n), na + e1, na + e2, la, lb_, LAB_CELL + 2 * ax + 0);
                    ub[na + e] = t;
                }
            }
        }
    }
    WV_SYNC();
    if constexpr (sizeof(TQ) == 4) {
        if (integ && nb > 0) {
            // a point of every face of the lower part: its lower vertices
            // first, then, overwriting, its crossing points; the apex: the
            // first lower vertex, then the first crossing point
            const uint32_t X = WV_BALLOT(crs() != 0);
            const int first_b = __builtin_ctz(Bb), first_x = X ? __builtin_ctz(X) : -1;
            WV_LANES
            {
                if (below()) {
                    P3 p;
                    p.x = me().x, p.y = me().y, p.z = me().z, p.pad = 0.0f;
                    for (int j = 0; j < 3; ++j) sh->rep[wlab(me().w, j)] = p;
                    if (wv_lane() == first_b) sh->apex = p;
                }
            }
            WV_SYNC();
            WV_LANES
            {
                for (int j = 0; j < 3; ++j) {
                    if (!((crs() >> j) & 1)) continue;
                    const P3 q = j == 0 ? q0() : (j == 1 ? q1() : q2());
                    sh->rep[wlab(me().w, j)] = q;
                    sh->rep[wlab(me().w, (j + 1) % 3)] = q;
                }
                if (wv_lane() == first_x) sh->apex = (crs() & 1) ? q0() : ((crs() & 2) ? q1() : q2());
            }
            WV_SYNC();
            const P3 Ap = sh->apex;
            const float A[3] = {Ap.x, Ap.y, Ap.z};
            const float rA = rho.at(A[0], A[1], A[2]);
            PL<float> a6, a24;
            WV_LANES
            {
                a6() = 0.0f;
                a24() = 0.0f;
                const int v = wv_lane();
                if (v < nq) {
                    const uint32_t w = me().w;
                    const bool bv = below();
                    const float rv = rho.at(me().x, me().y, me().z);
                    for (int j = 0; j < 3; ++j) {
                        const int n = wnb(w, j);
                        const bool bn = (Bb >> n) & 1u;
                        if (!bv && !bn) continue;
                        const S nn = j == 0 ? n0() : (j == 1 ? n1() : n2());
                        P3 a, b;
                        float ra;
                        if (bv) {
                            a.x = me().x, a.y = me().y, a.z = me().z;
                            ra = rv;
                            if (bn) {
                                b.x = nn.x, b.y = nn.y, b.z = nn.z;
                            } else {
                                b = j == 0 ? q0() : (j == 1 ? q1() : q2());
                            }
                        } else {
                            a = cross_point(nn, me(), ax, c);
                            ra = rho.at(a.x, a.y, a.z);
                            b.x = nn.x, b.y = nn.y, b.z = nn.z;
                        }
                        const float rb = rho.at(b.x, b.y, b.z);
                        const P3 f = sh->rep[wlab(w, j)];
                        const float fx = f.x - A[0], fy = f.y - A[1], fz = f.z - A[2];
                        const float ax_ = a.x - A[0], ay = a.y - A[1], az = a.z - A[2];
                        const float bx = b.x - A[0], by = b.y - A[1], bz = b.z - A[2];
                        // det(f, b, a): the walk runs clockwise seen from outside
                        const float d = fx * (by * az - bz * ay) + fy * (bz * ax_ - bx * az) + fz * (bx * ay - by * ax_);
                        const float rf = rho.at(f.x, f.y, f.z);
                        a6() += d;
                        a24() += d * ((rA + rf) + (ra + rb));
                    }
                }
            }
            o.s6 = WV_SUM(a6());
            o.s24 = WV_SUM(a24());
        }
    }
    return o;
}

// Move the polytope in b (n vertices) by -d along ax.
template <typename T>
SP_HD inline void translate(SlotT<T> *b, int n, int ax, T d)
{
    WV_LANES
    {
        const int v = wv_lane();
        if (v < n) {
            T *p = reinterpret_cast<T *>(&b[v]);
            p[ax] -= d;
        }
    }
    WV_SYNC();
}

// ------------------------------------------------------------------------
// the sweep of one work item by one group

enum Phase : int { PH_IDLE = 0, PH_TRIM = 1, PH_SLAB = 2, PH_COL = 3, PH_PIECE = 4 };

// A free-list of buffer indices (bits of a mask).
struct Pool {
    uint32_t free;
    SP_HD int take()
    {
        const int b = __builtin_ctz(free);
        free &= free - 1u;
        return b;
    }
    SP_HD void give(int b)
    {
        if (b >= 0) free |= 1u << b;
    }
};

struct Sweep {
    int phase;
    int ix, send, sx, sy, sz;
    int iy, yhi;
    int iz, zhi;
    int r0, r1, r2, n0, n1, n2;  // remainder, slab (FP64 pool), column (FP32 pool)
    Pool pd, pf;
    // density: value at the simplex's first corner (FP64), gradient, that
    // corner (anchor frame), clamp range
    double r0d, gd[3], v0[3];
    float g[3], rlo, rhi;
    int fail[3];
};

// Start sweeping slabs [sb, sb + sc) of a simplex: L its set-up (relabelled
// to its sweep order, positively oriented), X its corners in the same frame
// exactly (FP64).
SP_HD inline void sweep_start(GroupLDS *sh, Sweep &S, const Local<float> &L, const double (*X)[3], int sb, int sc)
{
    S.pd.free = (1u << NBUF_D) - 1u;
    S.pf.free = (1u << NBUF_F) - 1u;
    S.ix = sb;
    S.send = sb + sc;
    S.sx = L.span[0];
    S.sy = L.span[1];
    S.sz = L.span[2];
    S.iy = S.yhi = S.iz = S.zhi = 0;
    S.r1 = S.r2 = -1;
    S.n1 = S.n2 = 0;
    S.r0 = S.pd.take();
    S.n0 = 4;
    S.fail[0] = sb, S.fail[1] = 0, S.fail[2] = 0;
    // the tetrahedron in the frame of slab sb: neighbours counter-clockwise
    // from outside, face j of vertex v opposite the corner not in
    // {v, neighbour j-1, neighbour j}
    // (neighbours of corner v: {1,3,2}, {2,3,0}, {0,3,1}, {1,2,0}, as nibble
    // tables indexed by the lane, and the corner as selects, so that nothing
    // is indexed by the lane at run time)
    WV_LANES
    {
        const int v = wv_lane();
        if (v < 4) {
            const int a = (0x1021 >> (4 * v)) & 15, b = (0x2333 >> (4 * v)) & 15, c = (0x0102 >> (4 * v)) & 15;
            SlotD t;
            t.x = (v == 0 ? X[0][0] : v == 1 ? X[1][0] : v == 2 ? X[2][0] : X[3][0]) - (double)sb;
            t.y = v == 0 ? X[0][1] : v == 1 ? X[1][1] : v == 2 ? X[2][1] : X[3][1];
            t.z = v == 0 ? X[0][2] : v == 1 ? X[1][2] : v == 2 ? X[2][2] : X[3][2];
            t.w = wpack(a, b, c, 6 - v - c - a, 6 - v - a - b, 6 - v - b - c);
            sh->bd[S.r0][v] = t;
        }
    }
    WV_SYNC();
    // density: gradient by Cramer's rule in FP64 on the corner data
    double e[3][3], dr[3];
    for (int k = 0; k < 3; ++k) {
        for (int d = 0; d < 3; ++d) e[k][d] = X[k + 1][d] - X[0][d];
        dr[k] = (double)L.v[k + 1].r - (double)L.v[0].r;
    }
    double cc[3][3];
    for (int k = 0; k < 3; ++k) {
        const double *a = e[(k + 1) % 3], *b = e[(k + 2) % 3];
        cc[k][0] = a[1] * b[2] - a[2] * b[1];
        cc[k][1] = a[2] * b[0] - a[0] * b[2];
        cc[k][2] = a[0] * b[1] - a[1] * b[0];
    }
    const double det = e[0][0] * cc[0][0] + e[0][1] * cc[0][1] + e[0][2] * cc[0][2];
    const double inv = det != 0.0 ? 1.0 / det : 0.0;
    for (int d = 0; d < 3; ++d) {
        S.gd[d] = (dr[0] * cc[0][d] + dr[1] * cc[1][d] + dr[2] * cc[2][d]) * inv;
        S.g[d] = (float)S.gd[d];
        S.v0[d] = X[0][d];
    }
    S.r0d = (double)L.v[0].r;
    S.rlo = fminf(fminf(L.v[0].r, L.v[1].r), fminf(L.v[2].r, L.v[3].r));
    S.rhi = fmaxf(fmaxf(L.v[0].r, L.v[1].r), fmaxf(L.v[2].r, L.v[3].r));
    S.phase = sb > 0 ? PH_TRIM : PH_SLAB;
}

// The density in the frame whose origin is the cell (fx, fy, fz) of the
// simplex's anchor frame.
SP_HD inline Dens frame_density(const Sweep &S, int fx, int fy, int fz)
{
    Dens d;
    d.r0 = (float)(S.r0d + S.gd[0] * ((double)fx - S.v0[0]) + S.gd[1] * ((double)fy - S.v0[1]) +
                   S.gd[2] * ((double)fz - S.v0[2]));
    d.g[0] = S.g[0], d.g[1] = S.g[1], d.g[2] = S.g[2];
    d.rlo = S.rlo, d.rhi = S.rhi;
    return d;
}

// Next column (or slab) after the current column is done.
SP_HD inline void next_column(Sweep &S)
{
    if (S.r1 >= 0 && S.n1 > 0 && S.iy < S.yhi) {
        ++S.iy;
        S.phase = PH_COL;
    } else {
        S.pd.give(S.r1);
        S.r1 = -1;
        S.n1 = 0;
        ++S.ix;
        S.phase = (S.ix < S.send && S.r0 >= 0 && S.n0 > 0) ? PH_SLAB : PH_IDLE;
    }
}

// One step of the sweep: one split, and at most one piece, handed to
// dep(ix, iy, iz, integral) (called by every lane of the group with the same
// values).  Returns false on a capacity failure: S.fail is then the first
// piece not deposited, in sweep order.
template <typename Dep>
SP_HD inline bool sweep_step(GroupLDS *sh, Sweep &S, Dep &dep)
{
    const Dens none = {0.0f, {0.0f, 0.0f, 0.0f}, 0.0f, 0.0f};
    SlotD *const nd = nullptr;
    switch (S.phase) {
    case PH_TRIM: {
        // an item starting inside the simplex: drop the part left of slab sb
        const int bu = S.pd.take();
        const SplitOut o = split(sh, sh->bd[S.r0], S.n0, 0, 0.0, nd, sh->bd[bu], 0.0, false, -1, 0, none);
        S.fail[0] = S.ix, S.fail[1] = 0, S.fail[2] = 0;
        if (o.fail) {
            S.pd.give(bu);
            return false;
        }
        S.pd.give(S.r0);
        S.r0 = bu;
        S.n0 = o.nu;
        S.phase = S.n0 > 0 ? PH_SLAB : PH_IDLE;
        return true;
    }
    case PH_SLAB: {
        // slab ix: the remainder's part below x = 1, moved to its first
        // column along y; the rest (if the item goes on) moved to x - 1
        S.fail[0] = S.ix, S.fail[1] = 0, S.fail[2] = 0;
        const bool last = S.ix + 1 >= S.sx;
        const bool more = !last && S.ix + 1 < S.send;
        const int bl = S.pd.take();
        const int bu = more ? S.pd.take() : -1;
        const SplitOut o = split(sh, sh->bd[S.r0], S.n0, 0, last ? (double)INFINITY : 1.0, sh->bd[bl],
                                 more ? sh->bd[bu] : nd, 1.0, false, 1, S.sy - 1, none);
        if (o.fail) {
            S.pd.give(bl);
            S.pd.give(bu);
            return false;
        }
        S.pd.give(S.r0);
        S.r0 = bu;
        S.n0 = more ? o.nu : 0;
        S.r1 = bl;
        S.n1 = o.nl;
        if (S.n1 == 0) {
            S.pd.give(S.r1);
            S.r1 = -1;
            ++S.ix;
            S.phase = (S.ix < S.send && S.r0 >= 0 && S.n0 > 0) ? PH_SLAB : PH_IDLE;
            return true;
        }
        int yhi = (int)floorf(o.lmax);
        yhi = yhi > S.sy - 1 ? S.sy - 1 : yhi;
        S.iy = o.lshift;
        S.yhi = yhi < S.iy ? S.iy : yhi;
        S.phase = PH_COL;
        return true;
    }
    case PH_COL: {
        // column iy: the slab's part below y = 1, in FP32, moved to its
        // first cell along z; the rest of the slab moved to y - 1
        S.fail[0] = S.ix, S.fail[1] = S.iy, S.fail[2] = 0;
        const bool last = S.iy >= S.yhi;
        const int bl = S.pf.take();
        const int bu = last ? -1 : S.pd.take();
        const SplitOut o = split(sh, sh->bd[S.r1], S.n1, 1, last ? (double)INFINITY : 1.0, sh->bf[bl],
                                 last ? nd : sh->bd[bu], 1.0, false, 2, S.sz - 1, none);
        if (o.fail) {
            S.pf.give(bl);
            S.pd.give(bu);
            return false;
        }
        S.pd.give(S.r1);
        S.r1 = bu;
        S.n1 = last ? 0 : o.nu;
        S.r2 = bl;
        S.n2 = o.nl;
        if (S.n2 == 0) {
            S.pf.give(S.r2);
            S.r2 = -1;
            next_column(S);
            return true;
        }
        int zhi = (int)floorf(o.lmax);
        zhi = zhi > S.sz - 1 ? S.sz - 1 : zhi;
        S.iz = o.lshift;
        S.zhi = zhi < S.iz ? S.iz : zhi;
        S.phase = PH_PIECE;
        return true;
    }
    case PH_PIECE: {
        // piece (ix, iy, iz): the column's part below z = 1, integrated; the
        // rest moved to z - 1
        S.fail[0] = S.ix, S.fail[1] = S.iy, S.fail[2] = S.iz;
        const Dens rho = frame_density(S, S.ix, S.iy, S.iz);
        const bool last = S.iz >= S.zhi;
        const int bu = last ? -1 : S.pf.take();
        Slot *const nf = nullptr;
        const SplitOut o = split(sh, sh->bf[S.r2], S.n2, 2, last ? INFINITY : 1.0f, nf, last ? nf : sh->bf[bu], 1.0f,
                                 true, -1, 0, rho);
        if (o.fail) {
            S.pf.give(bu);
            return false;
        }
        if (o.s24 != 0.0f) dep(S.ix, S.iy, S.iz, o.s24 / 24.0f);
        S.pf.give(S.r2);
        if (last || o.nu == 0) {
            S.pf.give(bu);
            S.r2 = -1;
            S.n2 = 0;
            next_column(S);
        } else {
            S.r2 = bu;
            S.n2 = o.nu;
            ++S.iz;
        }
        return true;
    }
    default:
        return true;
    }
}

} // namespace wv
} // namespace sp
