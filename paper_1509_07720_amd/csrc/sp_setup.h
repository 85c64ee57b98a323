// sp_setup.h -- per-simplex set-up and the slab/column/cell sweep.
//
// Set-up (gather, periodic unwrap, cell coordinates, orientation) and the
// sweep that cuts one simplex into its pieces, one per grid cell it meets:
// x-slabs, then y-columns inside a slab, then z-cells inside a column
// (2D: x-slabs then y-cells).  The piece integrals are handed to a deposit
// callback.  Everything here is plain arithmetic usable on host and device.
#pragma once
#include <math.h>
#include <stdint.h>

#include "sp_poly.h"

namespace sp {

// Grid parameters as the kernels see them.
struct GridDev {
    int dims[3];
    int periodic[3];
    // cell coordinate u = (x - origin) * scale, scale = dims / extent;
    // hi/lo float pairs for the FP32 path, doubles for the FP64 path
    float o_hi[3], o_lo[3], s_hi[3], s_lo[3];
    double origin[3], scale[3], extent[3];
    double out_scale;   // 1 for density output, cell volume for mass output
};

// Largest bounding-box extent, in cells, of one simplex along any axis,
// periodic or not: work items and the set-up record encode slab counts and
// indices in 16 bits (a periodic axis also needs the extent below half the
// box, checked separately).
constexpr int MAX_SPAN = 32768;

// Set-up record of one simplex for the binning kernels: cost class (4 bits),
// number of work items (12 bits) and the span of its outermost sweep axis
// (16 bits; MAX_SPAN keeps it below 2^15); 0 means no work items.  A work
// item holds the simplex index (32 bits), its first slab and its slab count
// (16 bits each).
constexpr int MAX_ITEMS = 4095;

SP_HD inline uint32_t pack_setup(int cls, int nit, int sx)
{
    return ((uint32_t)cls << 28) | ((uint32_t)nit << 16) | (uint32_t)sx;
}
SP_HD inline int setup_class(uint32_t r) { return (int)(r >> 28); }
SP_HD inline int setup_items(uint32_t r) { return (int)((r >> 16) & 0xfffu); }
SP_HD inline int setup_span(uint32_t r) { return (int)(r & 0xffffu); }

SP_HD inline uint64_t pack_item(uint32_t s, int sb, int sc)
{
    return (uint64_t)s | ((uint64_t)(uint32_t)sb << 32) | ((uint64_t)(uint32_t)sc << 48);
}
SP_HD inline uint32_t item_simplex(uint64_t it) { return (uint32_t)it; }
SP_HD inline int item_first(uint64_t it) { return (int)((it >> 32) & 0xffffu); }
SP_HD inline int item_count(uint64_t it) { return (int)(it >> 48); }

// The k-th of nit work items over sx slabs: first slab and slab count.
SP_HD inline void item_range(int sx, int nit, int k, int &sb, int &sc)
{
    const int per = (sx + nit - 1) / nit;
    sb = k * per;
    sc = sx - sb < per ? sx - sb : per;
    if (sc < 0) sc = 0;
}

enum SetupStatus : int {
    SETUP_OK = 0,
    SETUP_ZERO_VOLUME = 1,
    SETUP_BAD_INDEX = 2,
    SETUP_NONFINITE = 3,
    SETUP_BAD_SPAN = 4,
};

// Local description of one simplex: corner positions in cell units relative
// to its anchor cell (the lowest cell of its bounding box), positively
// oriented; span = number of cells of the bounding box per axis.
template <typename T>
struct Local {
    V4<T> v[4];
    int anchor[3];
    int span[3];
    T det;   // 6 * volume (2 * area in 2D), > 0, cell units
};

// Error-free split of x*scale into an integer cell and a fraction in [0,1):
// TwoSum for x - origin, TwoProduct (fma) for the product, so the fraction
// carries the exact value up to one final rounding (Dekker 1971; Ogita, Rump
// & Oishi 2005).
SP_HD inline void cell_split(float x, float o_hi, float o_lo, float s_hi, float s_lo, int &k, float &f)
{
    // (the product p must stay rounded where it is added: no multiply-add
    // contraction, or its rounding error would count twice)
#pragma clang fp contract(off)
    float dh = x - o_hi;
    float t = dh - x;
    float dl = (x - (dh - t)) + (-o_hi - t);
    dl -= o_lo;
    float p = dh * s_hi;
    float e = fmaf(dh, s_hi, -p);
    float corr = e + (dh * s_lo + dl * s_hi);
    float kf = floorf(p);
    f = (p - kf) + corr;
    k = (int)kf;
    if (f >= 1.0f) {
        f -= 1.0f;
        k += 1;
    }
    if (f < 0.0f) {
        f += 1.0f;
        k -= 1;
        if (f >= 1.0f) f = 0.0f, k += 1;
    }
}

SP_HD inline bool finite_f(float v) { return v - v == 0.0f; }
SP_HD inline bool finite_d(double v) { return v - v == 0.0; }

// 6*volume of the tetrahedron (a, b, c, d)
template <typename T>
SP_HD inline T det3(const V4<T> &a, const V4<T> &b, const V4<T> &c, const V4<T> &d)
{
    T e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    T e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    T e3x = d.x - a.x, e3y = d.y - a.y, e3z = d.z - a.z;
    return e1x * (e2y * e3z - e2z * e3y) - e1y * (e2x * e3z - e2z * e3x) + e1z * (e2x * e3y - e2y * e3x);
}

// Orientation in FP32 with a static error filter (Appendix E.1: the error of
// a 3x3 determinant is bounded by a constant times the product of the
// largest entry of each column; the constant is rescaled from the paper's
// double precision value to single precision).  When the filter cannot
// decide, the determinant is recomputed in FP64 from the same (exactly
// representable) differences.  Returns 6*volume with the decided sign.
SP_HD inline float orient3_f(const V4<float> *v)
{
    float d = det3(v[0], v[1], v[2], v[3]);
    float mx[3] = {0.f, 0.f, 0.f};
    for (int a = 1; a < 4; ++a) {
        float e[3] = {v[a].x - v[0].x, v[a].y - v[0].y, v[a].z - v[0].z};
        for (int k = 0; k < 3; ++k) mx[k] = fmaxf(mx[k], fabsf(e[k]));
    }
    const float alpha = 4.0e-6f;
    if (fabsf(d) > alpha * mx[0] * mx[1] * mx[2]) return d;
    double e[3][3];
    for (int a = 1; a < 4; ++a) {
        e[a - 1][0] = (double)v[a].x - (double)v[0].x;
        e[a - 1][1] = (double)v[a].y - (double)v[0].y;
        e[a - 1][2] = (double)v[a].z - (double)v[0].z;
    }
    double dd = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    if (dd == 0.0) return 0.0f;
    // keep the FP64 sign even when the rounded magnitude underflows to 0
    float r = (float)dd;
    if (r == 0.0f) r = dd > 0 ? 1e-38f : -1e-38f;
    return r;
}

SP_HD inline float orient2_f(const V4<float> *v)
{
    float ax = v[1].x - v[0].x, ay = v[1].y - v[0].y, bx = v[2].x - v[0].x, by = v[2].y - v[0].y;
    float d = ax * by - ay * bx;
    const float alpha = 2.0e-6f;
    if (fabsf(d) > alpha * fmaxf(fabsf(ax), fabsf(bx)) * fmaxf(fabsf(ay), fabsf(by))) return d;
    double dd = ((double)v[1].x - v[0].x) * ((double)v[2].y - v[0].y) - ((double)v[1].y - v[0].y) * ((double)v[2].x - v[0].x);
    if (dd == 0.0) return 0.0f;
    float r = (float)dd;
    if (r == 0.0f) r = dd > 0 ? 1e-38f : -1e-38f;
    return r;
}

// Set-up of simplex s in the FP32 path.  D = 2 or 3.  Every check runs
// whatever `validate` says (a bad index or a non-finite coordinate must never
// reach the sweep); the caller decides whether to report the status.
//
// ex (optional, D = 3): the corners' local coordinates without rounding,
// (k - anchor) + fraction in FP64, in the same corner order as L.
template <int D>
SP_HD inline int setup_f32(const float *xyz, int64_t n_vert, const int32_t *simp, int64_t s, const float *rho,
                           bool per_corner, const GridDev &g, bool validate, Local<float> &L,
                           double (*ex)[3] = nullptr)
{
    constexpr int K = D + 1;
    int k[4][3];
    float f[4][3];
    float r[4];
    for (int a = 0; a < K; ++a) {
        int64_t vi = simp[s * K + a];
        if (vi < 0 || vi >= n_vert) return SETUP_BAD_INDEX;
        for (int d = 0; d < D; ++d) {
            float x = xyz[vi * D + d];
            // cell coordinates must stay well inside the int range
            float u = (x - g.o_hi[d]) * g.s_hi[d];
            if (!finite_f(x) || !(fabsf(u) < 1.0e9f)) return SETUP_NONFINITE;
            cell_split(x, g.o_hi[d], g.o_lo[d], g.s_hi[d], g.s_lo[d], k[a][d], f[a][d]);
        }
        r[a] = per_corner ? rho[s * K + a] : rho[vi];
        if (!finite_f(r[a])) return SETUP_NONFINITE;
    }
    for (int d = 0; d < D; ++d) {
        int kmin = k[0][d];
        if (g.periodic[d]) {
            const int N = g.dims[d];
            for (int a = 1; a < K; ++a) {
                float delta = (float)(k[a][d] - k[0][d]) + (f[a][d] - f[0][d]);
                int sh = (int)rintf(delta / (float)N);
                k[a][d] -= sh * N;
            }
        }
        for (int a = 1; a < K; ++a) kmin = k[a][d] < kmin ? k[a][d] : kmin;
        float lmax = 0.0f;
        for (int a = 0; a < K; ++a) {
            float l = (float)(k[a][d] - kmin) + f[a][d];
            if (d == 0) L.v[a].x = l;
            else if (d == 1) L.v[a].y = l;
            else L.v[a].z = l;
            lmax = l > lmax ? l : lmax;
            if (ex) ex[a][d] = (double)(k[a][d] - kmin) + (double)f[a][d];
        }
        if (!(lmax < (float)MAX_SPAN) || (g.periodic[d] && !(lmax < 0.5f * (float)g.dims[d]))) return SETUP_BAD_SPAN;
        L.anchor[d] = kmin;
        L.span[d] = (int)floorf(lmax) + 1;
    }
    for (int a = 0; a < K; ++a) {
        if (D == 2) L.v[a].z = 0.0f;
        L.v[a].r = r[a];
    }
    if (D == 2) {
        L.anchor[2] = 0;
        L.span[2] = 1;
    }
    float det = D == 3 ? orient3_f(L.v) : orient2_f(L.v);
    if (det == 0.0f) return SETUP_ZERO_VOLUME;
    if (det < 0.0f) {
        V4<float> t = L.v[1];
        L.v[1] = L.v[2];
        L.v[2] = t;
        det = -det;
        if (ex)
            for (int d = 0; d < 3; ++d) {
                const double u = ex[1][d];
                ex[1][d] = ex[2][d];
                ex[2][d] = u;
            }
    }
    L.det = det;
    return SETUP_OK;
}

// Set-up of simplex s in the FP64 path: the same unwrap in box units and the
// same cell coordinates as a plain double-precision evaluation.  The inputs
// may be float (simplices of an FP32C problem clipped in double), upcast
// exactly.
//
// swapped (optional): set when corners 1 and 2 were exchanged to orient the
// simplex positively (L's corner a is then the input's corner 3 - a for a in
// {1, 2}).
template <int D, typename TI = double>
SP_HD inline int setup_f64(const TI *xyz, int64_t n_vert, const int32_t *simp, int64_t s, const TI *rho,
                           bool per_corner, const GridDev &g, bool validate, Local<double> &L,
                           bool *swapped = nullptr)
{
    constexpr int K = D + 1;
    double x[4][3];
    double r[4];
    for (int a = 0; a < K; ++a) {
        int64_t vi = simp[s * K + a];
        if (vi < 0 || vi >= n_vert) return SETUP_BAD_INDEX;
        for (int d = 0; d < D; ++d) {
            x[a][d] = (double)xyz[vi * D + d];
            double u = (x[a][d] - g.origin[d]) * g.scale[d];
            if (!finite_d(x[a][d]) || !(fabs(u) < 1.0e9)) return SETUP_NONFINITE;
        }
        r[a] = (double)(per_corner ? rho[s * K + a] : rho[vi]);
        if (!finite_d(r[a])) return SETUP_NONFINITE;
    }
    for (int d = 0; d < D; ++d) {
        if (g.periodic[d]) {
            const double Lb = g.extent[d];
            for (int a = 1; a < K; ++a) x[a][d] -= Lb * rint((x[a][d] - x[0][d]) / Lb);
        }
        double u[4];
        double umin = 0, umax = 0;
        for (int a = 0; a < K; ++a) {
            u[a] = (x[a][d] - g.origin[d]) * g.scale[d];
            umin = (a == 0 || u[a] < umin) ? u[a] : umin;
            umax = (a == 0 || u[a] > umax) ? u[a] : umax;
        }
        if (!((umax - umin) < (double)MAX_SPAN - 1.0) || (g.periodic[d] && !((umax - umin) < 0.5 * (double)g.dims[d])))
            return SETUP_BAD_SPAN;
        double kmin = floor(umin);
        for (int a = 0; a < K; ++a) {
            double l = u[a] - kmin;
            if (d == 0) L.v[a].x = l;
            else if (d == 1) L.v[a].y = l;
            else L.v[a].z = l;
        }
        L.anchor[d] = (int)kmin;
        L.span[d] = (int)floor(umax - kmin) + 1;
    }
    for (int a = 0; a < K; ++a) {
        if (D == 2) L.v[a].z = 0.0;
        L.v[a].r = r[a];
    }
    if (D == 2) {
        L.anchor[2] = 0;
        L.span[2] = 1;
    }
    double det;
    if (D == 3) {
        det = det3(L.v[0], L.v[1], L.v[2], L.v[3]);
    } else {
        det = (L.v[1].x - L.v[0].x) * (L.v[2].y - L.v[0].y) - (L.v[1].y - L.v[0].y) * (L.v[2].x - L.v[0].x);
    }
    if (det == 0.0) return SETUP_ZERO_VOLUME;
    if (swapped) *swapped = det < 0.0;
    if (det < 0.0) {
        V4<double> t = L.v[1];
        L.v[1] = L.v[2];
        L.v[2] = t;
        det = -det;
    }
    L.det = det;
    return SETUP_OK;
}

// Order in which a simplex is swept: outermost axis first, innermost last.
// The innermost axis is the one of largest extent, which makes the columns
// (and so the polytope rebuilds) fewest.  With outer_longest the largest
// extent goes outermost instead: more columns, but as many slabs as the
// simplex is long, so that a long simplex cut into one-slab work items
// spreads over many lanes.
struct SweepOrder {
    int ax[3];
};

template <typename T>
SP_HD inline SweepOrder sweep_order(const Local<T> &L, bool outer_longest = false)
{
    // sort axes by span, ascending; ties keep x, y, z order (written with
    // compares on values only, so nothing is indexed at run time)
    const int s0 = L.span[0], s1 = L.span[1], s2 = L.span[2];
    const bool l01 = s1 < s0, l02 = s2 < s0, l12 = s2 < s1;
    const int r0 = (int)l01 + (int)l02;            // rank of axis 0
    const int r1 = (int)!l01 + (int)l12;           // rank of axis 1
    SweepOrder o;
    o.ax[0] = r0 == 0 ? 0 : (r1 == 0 ? 1 : 2);
    o.ax[1] = r0 == 1 ? 0 : (r1 == 1 ? 1 : 2);
    o.ax[2] = r0 == 2 ? 0 : (r1 == 2 ? 1 : 2);
    if (outer_longest) {
        const int t = o.ax[0];
        o.ax[0] = o.ax[2];
        o.ax[2] = t;
    }
    return o;
}

// One of three values by a run-time index, as selects (a register array
// indexed at run time would go to scratch memory).
template <typename X>
SP_HD inline X sel3(const X &a, const X &b, const X &c, int i)
{
    return i == 0 ? a : (i == 1 ? b : c);
}

// The simplex with its axes relabelled so that sweep axis k becomes local
// axis k (orientation restored by a vertex swap when the relabelling is odd).
template <typename T>
SP_HD inline Local<T> permuted(const Local<T> &L, const SweepOrder &o)
{
    Local<T> M = L;
    for (int k = 0; k < 4; ++k) {
        M.v[k].x = sel3(L.v[k].x, L.v[k].y, L.v[k].z, o.ax[0]);
        M.v[k].y = sel3(L.v[k].x, L.v[k].y, L.v[k].z, o.ax[1]);
        M.v[k].z = sel3(L.v[k].x, L.v[k].y, L.v[k].z, o.ax[2]);
    }
    for (int d = 0; d < 3; ++d) {
        M.span[d] = sel3(L.span[0], L.span[1], L.span[2], o.ax[d]);
        M.anchor[d] = sel3(L.anchor[0], L.anchor[1], L.anchor[2], o.ax[d]);
    }
    // a transposition of two axes flips the orientation; the three cyclic
    // orders keep it
    const bool odd = !((o.ax[0] == 0 && o.ax[1] == 1) || (o.ax[0] == 1 && o.ax[1] == 2) || (o.ax[0] == 2 && o.ax[1] == 0));
    if (odd) {
        V4<T> t = M.v[1];
        M.v[1] = M.v[2];
        M.v[2] = t;
    }
    return M;
}

// Exact corners relabelled as permuted() relabels the set-up.
SP_HD inline void permuted_exact(const double (*ex)[3], const SweepOrder &o, double (*out)[3])
{
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) out[k][d] = sel3(ex[k][0], ex[k][1], ex[k][2], o.ax[d]);
    const bool odd = !((o.ax[0] == 0 && o.ax[1] == 1) || (o.ax[0] == 1 && o.ax[1] == 2) || (o.ax[0] == 2 && o.ax[1] == 0));
    if (odd)
        for (int d = 0; d < 3; ++d) {
            const double u = out[1][d];
            out[1][d] = out[2][d];
            out[2][d] = u;
        }
}

// y range of a simplex's part in slab ix of its sweep (x in [ix, ix + 1),
// unbounded below for the first slab and above for the last), in its anchor
// frame: over its corners inside the slab and the points where its edges
// cross the slab's planes.  mn > mx: the slab is empty.  Rounding can put a
// bound a hair off; the sweep leaves its first column open below and its
// last open above, so a sliver beyond a bound still lands in a column.
template <typename T>
SP_HD inline void slab_y_range(const V4<T> *v, int ix, int sx, T &mn, T &mx)
{
    const bool lo = ix > 0, hi = ix < sx - 1;
    const T xl = (T)ix, xu = (T)(ix + 1);
    mn = T(INFINITY);
    mx = T(-INFINITY);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = (!lo || v[k].x >= xl) && (!hi || v[k].x <= xu);
        mn = in ? sp_fmin(mn, v[k].y) : mn;
        mx = in ? sp_fmax(mx, v[k].y) : mx;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int a = e < 3 ? 0 : (e < 5 ? 1 : 2);
        const int b = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
        const T xa = v[a].x, xb = v[b].x, ya = v[a].y, yb = v[b].y;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const T c = side ? xu : xl;
            const bool on = side ? hi : lo;
            // (the hardware reciprocal: a bound only needs to be near)
            const bool cut = on && ((xa < c) != (xb < c));
            const T y = ya + (c - xa) * sp_rcp(cut ? xb - xa : T(1)) * (yb - ya);
            mn = cut ? sp_fmin(mn, y) : mn;
            mx = cut ? sp_fmax(mx, y) : mx;
        }
    }
}

// Sweep of one 3D simplex over the slabs [sb, sb+sc) of its outermost axis,
// starting at column ry of the first slab.  The deposit receives each
// piece's integral of rho in cell-volume units at its local cell indices
// along the sweep axes.
//
// The sweep is resumable: step() first builds the next column polytope if
// the previous one is finished (the simplex cut by the planes of slab i0 and
// column i1) and then cuts off and integrates one piece.  A GPU lane calls
// step() once per loop iteration and takes a new simplex as soon as its
// current one is done, so the lanes of a wave stay busy whatever their
// slab, column and cell counts.  On a capacity failure, fail = (i0, i1, i2)
// is the first piece not yet deposited, in sweep order.
//
// Each column is cut out of the simplex afresh, in a frame local to it: the
// tetrahedron is moved by (-i0, -i1) and clipped by the slab's and the
// column's planes (the slab's y range comes from the corners, not from a
// clipped slab), and the column is moved by -(its lowest cell) along z once
// its z range is known.  The cut points then carry the rounding of
// coordinates of a few cells instead of the simplex's span, which for
// simplices tens of cells across is the difference between meeting the
// FP32 bound per cell and missing it.
struct Sweep3 {
    int sb, send, ry;
    int ix, iy, ylo, yhi, iz, zhi, cx, cy, zo;
    int fail[3];

    SP_HD void start(int sb_, int sc_, int ry_)
    {
        sb = sb_;
        send = sb_ + sc_;
        ry = ry_;
        ix = sb;
        iy = -1;
        ylo = 0;
        yhi = -1;
        iz = 0;
        zhi = -1;
        cx = sb;
        cy = 0;
        zo = 0;
        fail[0] = ix;
        fail[1] = ry;
        fail[2] = 0;
    }

    // The next step starts by building a column (the current one is done and
    // slabs remain).
    SP_HD bool needs_build() const { return iz > zhi && ix < send; }

    // One step.  Returns 1 when a piece was processed and more may follow,
    // 0 when the sweep is finished, -1 on a capacity failure.
    template <typename T, int MAXV, int STRIDE, typename Dep>
    SP_HD int step(Poly3<T, MAXV, STRIDE> &P, const Local<T> &L, Dep &dep)
    {
        const int sx = L.span[0], sy = L.span[1], sz = L.span[2];
        // build the next non-empty column (in its own frame)
        while (iz > zhi && ix < send) {
            if (iy < 0) {
                // a new slab: its columns
                T mn, mx;
                slab_y_range(L.v, ix, sx, mn, mx);
                if (mn <= mx) {
                    ylo = (int)floor(mn);
                    yhi = (int)floor(mx);
                    ylo = ylo < 0 ? 0 : (ylo > sy - 1 ? sy - 1 : ylo);
                    yhi = yhi > sy - 1 ? sy - 1 : (yhi < ylo ? ylo : yhi);
                    iy = ylo;
                    if (ix == sb && ry > iy) iy = ry;
                }
                if (mn > mx || iy > yhi) {
                    ++ix;
                    iy = -1;
                    fail[0] = ix;
                    fail[1] = 0;
                    fail[2] = 0;
                    continue;
                }
            }
            fail[0] = ix;
            fail[1] = iy;
            fail[2] = 0;
            P.init_tet_at(L.v, (T)ix, (T)iy);
            // the slab's and the column's planes, those that cut: one clip
            // call in a loop, so that lanes needing different planes cut
            // together
            for (uint32_t cuts = (ix > 0 ? 1u : 0u) | (ix < sx - 1 ? 2u : 0u) | (iy > ylo ? 4u : 0u) |
                                 (iy < yhi ? 8u : 0u);
                 cuts; cuts &= cuts - 1u) {
                const int k = __builtin_ctz(cuts);
                const bool lower = (k & 1) == 0;  // a lower plane keeps what is above it
                if (!P.clip(k >> 1, lower ? T(0) : T(1), lower)) return -1;
            }
            if (!P.empty()) {
                T mn, mx;
                P.range(2, mn, mx);
                iz = (int)floor(mn);
                zhi = (int)floor(mx);
                iz = iz < 0 ? 0 : iz;
                zhi = zhi > sz - 1 ? sz - 1 : zhi;
                cx = ix;
                cy = iy;
                zo = iz;
                if (zo != 0) P.shift(2, (T)zo);
            }
            // next column (or slab) for the following build
            if (iy >= yhi) {
                ++ix;
                iy = -1;
            } else {
                ++iy;
            }
        }
        if (iz > zhi) return 0;  // nothing left
        // one piece: the part of the column below z = iz + 1
        T s6, s24;
        const bool last = iz == zhi;
        fail[0] = cx;
        fail[1] = cy;
        fail[2] = iz;
        uint32_t below = 0u;
        if (!P.integrate_below(2, (T)(iz + 1 - zo), last, s6, s24, &below)) return -1;
        if (s24 != T(0)) dep(cx, cy, iz, s24 / T(24));
        if (!last) {
            fail[2] = iz + 1;
            // (the integral classified the vertices against the same plane)
            if (!P.clip_classified(2, (T)(iz + 1 - zo), true, below)) return -1;
            ++iz;
            if (P.empty()) zhi = iz - 1;
        } else {
            ++iz;
        }
        return 1;
    }
};

// The whole sweep of one simplex in one call (host-side tools and tests).
template <typename T, int MAXV, int STRIDE, typename Dep>
SP_HD inline bool sweep3(Poly3<T, MAXV, STRIDE> &P, const Local<T> &L, int sb, int sc, Dep &dep, int ry, int *fail)
{
    Sweep3 S;
    S.start(sb, sc, ry);
    P.set_density(L.v);
    int r;
    while ((r = S.step(P, L, dep)) > 0) {
    }
    fail[0] = S.fail[0];
    fail[1] = S.fail[1];
    fail[2] = S.fail[2];
    return r == 0;
}

// Convex polygon (2D pieces): an ordered, counter-clockwise vertex list in two
// ping-pong buffers.  Cuts follow Sutherland-Hodgman with the same
// classification and intersection rule as the 3D polytopes.
template <typename T, int MAXP, int STRIDE>
struct Poly2 {
    V4<T> *a;
    V4<T> *b;
    int n;

    SP_HD V4<T> P(int v) const { return a[v * STRIDE]; }

    SP_HD void init_tri(const V4<T> *v)
    {
        for (int i = 0; i < 3; ++i) a[i * STRIDE] = v[i];
        n = 3;
    }

    SP_HD bool clip(int ax, T c, bool keep_upper)
    {
        int m = 0;
        for (int v = 0; v < n; ++v) {
            V4<T> p = a[v * STRIDE];
            V4<T> q = a[((v + 1) % n) * STRIDE];
            bool bp = comp(p, ax) < c, bq = comp(q, ax) < c;
            bool kp = keep_upper ? !bp : bp;
            if (kp) {
                if (m >= MAXP) return false;
                b[m++ * STRIDE] = p;
            }
            if (bp != bq) {
                if (m >= MAXP) return false;
                b[m++ * STRIDE] = bp ? isect(p, q, ax, c) : isect(q, p, ax, c);
            }
        }
        V4<T> *t = a;
        a = b;
        b = t;
        n = m >= 3 ? m : 0;
        return true;
    }

    // 2*area and 6*integral of the part below x_ax = c (or of the whole
    // polygon), as triangles from an apex on the cutting line.
    SP_HD void integrate_below(int ax, T c, bool whole, T &s2, T &s6) const
    {
        s2 = T(0);
        s6 = T(0);
        if (n == 0) return;
        V4<T> A = a[0];
        if (!whole) {
            bool any = false, all = true;
            for (int v = 0; v < n; ++v) {
                bool bv = comp(a[v * STRIDE], ax) < c;
                any = any || bv;
                all = all && bv;
            }
            if (!any) return;
            if (all) {
                whole = true;
            } else {
                // apex: the first crossing point (on the cutting line)
                for (int v = 0; v < n; ++v) {
                    V4<T> p = a[v * STRIDE];
                    V4<T> q = a[((v + 1) % n) * STRIDE];
                    bool bp = comp(p, ax) < c, bq = comp(q, ax) < c;
                    if (bp != bq) {
                        A = bp ? isect(p, q, ax, c) : isect(q, p, ax, c);
                        break;
                    }
                }
            }
        }
        V4<T> q0, qp;
        int cnt = 0;
        for (int v = 0; v < n; ++v) {
            V4<T> p = a[v * STRIDE];
            V4<T> q = a[((v + 1) % n) * STRIDE];
            bool bp = whole || comp(p, ax) < c, bq = whole || comp(q, ax) < c;
            for (int e = 0; e < 2; ++e) {
                V4<T> w;
                if (e == 0) {
                    if (!bp) continue;
                    w = p;
                } else {
                    if (bp == bq) continue;
                    w = bp ? isect(p, q, ax, c) : isect(q, p, ax, c);
                }
                if (cnt == 0) q0 = w;
                else {
                    T d = (qp.x - A.x) * (w.y - A.y) - (qp.y - A.y) * (w.x - A.x);
                    s2 += d;
                    s6 += d * (A.r + qp.r + w.r);
                }
                qp = w;
                ++cnt;
            }
        }
        if (cnt >= 2) {
            T d = (qp.x - A.x) * (q0.y - A.y) - (qp.y - A.y) * (q0.x - A.x);
            s2 += d;
            s6 += d * (A.r + qp.r + q0.r);
        }
    }
};

// Sweep of one triangle over x-slabs [sb, sb+sc) of its bounding box; the
// deposit receives (ix, iy, 0, integral of rho in cell-area units).
template <typename T, int MAXP, int STRIDE, typename Dep>
SP_HD inline bool sweep2(Poly2<T, MAXP, STRIDE> &P, const Local<T> &L, int sb, int sc, Dep &dep, int *fail)
{
    const int sx = L.span[0], sy = L.span[1];
    for (int ix = sb; ix < sb + sc; ++ix) {
        fail[0] = ix;
        fail[1] = 0;
        fail[2] = 0;
        P.init_tri(L.v);
        if (ix > 0 && !P.clip(0, (T)ix, true)) return false;
        if (ix < sx - 1 && !P.clip(0, (T)(ix + 1), false)) return false;
        if (P.n == 0) continue;
        T mn = P.P(0).y, mx = mn;
        for (int v = 1; v < P.n; ++v) {
            T c = P.P(v).y;
            mn = c < mn ? c : mn;
            mx = c > mx ? c : mx;
        }
        int ylo = (int)floor(mn), yhi = (int)floor(mx);
        ylo = ylo < 0 ? 0 : ylo;
        yhi = yhi > sy - 1 ? sy - 1 : yhi;
        for (int iy = ylo; iy <= yhi; ++iy) {
            bool last = iy == yhi;
            T s2, s6;
            P.integrate_below(1, (T)(iy + 1), last, s2, s6);
            if (s6 != T(0)) dep(ix, iy, 0, s6 / T(6));
            if (!last) {
                fail[1] = iy + 1;
                if (!P.clip(1, (T)(iy + 1), true)) return false;
                if (P.n == 0) break;
            }
        }
    }
    return true;
}

} // namespace sp
