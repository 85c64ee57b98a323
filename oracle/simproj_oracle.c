/*
 * simproj_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 reference for the exact projection of a piecewise-linear
 * density defined on a simplicial mesh onto a regular grid (Sousbie & Colombi,
 * "ColDICE", Section 3, eq. eq_firstOrder):
 *
 *     P_j = sum_i  integral over (S_i intersect G_j) of rho_i(x) dx
 *
 * where rho_i is the linear interpolant of simplex i's vertex (or corner)
 * densities (Section 3.1, last paragraph).  Only tests/, the smoke check and
 * the CPU-baseline leg of the benchmark use this file; the projection library
 * shares no code with it.
 *
 * Method (brute force, one candidate cell at a time):
 *   1. gather the simplex, unwrap it on periodic axes (minimum image relative
 *      to its first vertex) and move to cell units;
 *   2. for every cell of its integer bounding box, collect the boundary of the
 *      convex piece P = S intersect G as polygons: each simplex facet clipped
 *      to the closed cell, and each cell facet clipped to the closed simplex
 *      (Sutherland-Hodgman, one half-space at a time);
 *   3. integrate rho over P by cones from a point O inside P to every
 *      boundary facet, each cone split into tetrahedra along a fan of its
 *      facet (the decomposition used in Appendix C); the integral of a linear
 *      function over a tetrahedron is its volume times the mean of its four
 *      vertex values, and the rho-weighted first moment uses
 *      int lambda_a lambda_b = V (1 + delta_ab) / 20 (3D), / 12 (2D);
 *   4. add the piece to its cell in a double-double (TwoSum) accumulator.
 *
 * Threads own disjoint z-planes (y-rows in 2D) of the grid, so every cell sum
 * is formed in a fixed order and the result is deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dim;                 /* 2 or 3 */
    const double *xyz;       /* [n_vert][dim] */
    int64_t n_vert;
    const int32_t *simp;     /* [n_simplex][dim+1] */
    int64_t n_simplex;
    const double *rho;       /* [n_vert] or [n_simplex][dim+1] */
    int rho_per_corner;
    double origin[3], extent[3];
    int64_t dims[3];
    int periodic[3];
    const uint8_t *cell_mask; /* optional: only cells with mask != 0 are computed */
} or_problem;

typedef struct {
    int64_t n_zero_volume;   /* skipped: zero volume */
    int64_t n_bad_span;      /* skipped: periodic extent >= L/2 */
    int64_t n_bad_index;     /* skipped: vertex index out of range */
    int64_t n_candidates;    /* candidate cells visited */
    int64_t n_pieces;        /* candidates with a piece of positive volume */
} or_stats;

/* ------------------------------------------------------------------------ */
/* small vector helpers */

typedef struct { double x[3]; double r; } pt; /* position (cell-local) + rho */

#define MAXP 24

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Sutherland-Hodgman: keep the part of polygon (in,n) where s(p) >= 0, with
 * s(p) = dot(nrm, p) + off.  rho is interpolated along the clipped edges. */
static int clip_poly(const pt *in, int n, const double *nrm, double off, pt *out)
{
    int m = 0;
    if (n == 0) return 0;
    for (int i = 0; i < n; ++i) {
        const pt *a = &in[i];
        const pt *b = &in[(i + 1) % n];
        double sa = dot3(nrm, a->x) + off;
        double sb = dot3(nrm, b->x) + off;
        if (sa >= 0) out[m++] = *a;
        if ((sa >= 0) != (sb >= 0)) {
            /* canonical direction: interpolate from the kept end */
            const pt *p = sa >= 0 ? a : b, *q = sa >= 0 ? b : a;
            double sp = sa >= 0 ? sa : sb, sq = sa >= 0 ? sb : sa;
            double t = sp / (sp - sq);
            pt r;
            for (int d = 0; d < 3; ++d) r.x[d] = p->x[d] + t * (q->x[d] - p->x[d]);
            r.r = p->r + t * (q->r - p->r);
            out[m++] = r;
        }
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* one piece: S (vertices v[0..dim], positively oriented, cell-local) against
 * the closed unit cell.  Returns volume; adds integral of rho and the
 * rho-weighted first moment (in the caller's global cell coordinates, i.e.
 * local + shift). */

typedef struct {
    int npoly;
    int len[16];
    double nrm[16][3];       /* outward unit normal of each facet / edge */
    pt poly[16][MAXP];
} boundary;

static double rho_at(const double *x, const double *x0, double r0, const double *g)
{
    return r0 + g[0] * (x[0] - x0[0]) + g[1] * (x[1] - x0[1]) + g[2] * (x[2] - x0[2]);
}

static double piece3(const pt *v, const double *nrmf /* [4][3] outward unit */, const double *g,
                     const double *shift, double *mass, double *mom)
{
    boundary B;
    B.npoly = 0;
    /* (a) simplex facets clipped to the cell: facet k is opposite vertex k */
    for (int k = 0; k < 4; ++k) {
        pt a[MAXP], b[MAXP];
        int n = 0;
        for (int i = 0; i < 4; ++i)
            if (i != k) a[n++] = v[i];
        for (int d = 0; d < 3 && n; ++d) {
            double e[3] = {0, 0, 0};
            e[d] = 1.0;
            n = clip_poly(a, n, e, 0.0, b);      /* x_d >= 0 */
            e[d] = -1.0;
            n = clip_poly(b, n, e, 1.0, a);      /* x_d <= 1 */
        }
        if (n >= 3) {
            memcpy(B.poly[B.npoly], a, sizeof(pt) * n);
            B.len[B.npoly] = n;
            memcpy(B.nrm[B.npoly], &nrmf[3 * k], sizeof(double) * 3);
            B.npoly++;
        }
    }
    /* (b) cell facets clipped to the simplex */
    for (int d = 0; d < 3; ++d) {
        for (int side = 0; side < 2; ++side) {
            double on[3] = {0, 0, 0};
            on[d] = side ? 1.0 : -1.0;
            /* a simplex facet lying in this cell facet with the same outward
             * normal already covers it */
            int skip = 0;
            for (int k = 0; k < 4 && !skip; ++k) {
                int inplane = 1;
                for (int i = 0; i < 4; ++i)
                    if (i != k && v[i].x[d] != (double)side) inplane = 0;
                if (inplane && nrmf[3 * k + d] * on[d] > 0) skip = 1;
            }
            if (skip) continue;
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            pt a[MAXP], b[MAXP];
            double sq[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int i = 0; i < 4; ++i) {
                a[i].x[d] = side;
                a[i].x[d1] = sq[i][0];
                a[i].x[d2] = sq[i][1];
                a[i].r = 0;
            }
            int n = 4;
            for (int k = 0; k < 4 && n; ++k) {
                /* inside the simplex: dot(n_k, p - p_k) <= 0 */
                const double *nk = &nrmf[3 * k];
                const double *pk = v[(k + 1) % 4].x;
                double neg[3] = {-nk[0], -nk[1], -nk[2]};
                n = clip_poly(a, n, neg, dot3(nk, pk), b);
                memcpy(a, b, sizeof(pt) * n);
            }
            if (n >= 3) {
                for (int i = 0; i < n; ++i) a[i].r = rho_at(a[i].x, v[0].x, v[0].r, g);
                memcpy(B.poly[B.npoly], a, sizeof(pt) * n);
                B.len[B.npoly] = n;
                memcpy(B.nrm[B.npoly], on, sizeof(on));
                B.npoly++;
            }
        }
    }
    if (B.npoly == 0) return 0.0;
    /* interior point: mean of all boundary polygon vertices */
    double O[3] = {0, 0, 0};
    int cnt = 0;
    for (int f = 0; f < B.npoly; ++f)
        for (int i = 0; i < B.len[f]; ++i) {
            for (int d = 0; d < 3; ++d) O[d] += B.poly[f][i].x[d];
            cnt++;
        }
    for (int d = 0; d < 3; ++d) O[d] /= cnt;
    double rO = rho_at(O, v[0].x, v[0].r, g);
    double vol = 0, ms = 0, m3[3] = {0, 0, 0};
    for (int f = 0; f < B.npoly; ++f) {
        const pt *P = B.poly[f];
        double dv[3];
        sub3(P[0].x, O, dv);
        double h = dot3(B.nrm[f], dv);
        for (int i = 1; i + 1 < B.len[f]; ++i) {
            double e1[3], e2[3], c[3];
            sub3(P[i].x, P[0].x, e1);
            sub3(P[i + 1].x, P[0].x, e2);
            cross3(e1, e2, c);
            double area = 0.5 * sqrt(dot3(c, c));
            double Vt = h * area / 3.0;
            double r4[4] = {rO, P[0].r, P[i].r, P[i + 1].r};
            const double *x4[4] = {O, P[0].x, P[i].x, P[i + 1].x};
            double rs = r4[0] + r4[1] + r4[2] + r4[3];
            vol += Vt;
            ms += Vt * rs / 4.0;
            for (int d = 0; d < 3; ++d) {
                double xs = 0, rx = 0;
                for (int a2 = 0; a2 < 4; ++a2) {
                    double xg = x4[a2][d] + shift[d];
                    xs += xg;
                    rx += r4[a2] * xg;
                }
                m3[d] += Vt / 20.0 * (rs * xs + rx);
            }
        }
    }
    *mass = ms;
    for (int d = 0; d < 3; ++d) mom[d] = m3[d];
    return vol;
}

/* 2D: v[0..2] (x[2] unused), positively oriented triangle, against the
 * closed unit square. */
static void clip_seg(const pt *a, const pt *b, const double *nrm, double off, pt *oa, pt *ob, int *ok)
{
    double sa = dot3(nrm, a->x) + off, sb = dot3(nrm, b->x) + off;
    *oa = *a;
    *ob = *b;
    if (sa < 0 && sb < 0) { *ok = 0; return; }
    if (sa >= 0 && sb >= 0) { *ok = 1; return; }
    const pt *p = sa >= 0 ? a : b, *q = sa >= 0 ? b : a;
    double sp = sa >= 0 ? sa : sb, sq = sa >= 0 ? sb : sa;
    double t = sp / (sp - sq);
    pt r;
    for (int d = 0; d < 3; ++d) r.x[d] = p->x[d] + t * (q->x[d] - p->x[d]);
    r.r = p->r + t * (q->r - p->r);
    if (sa >= 0) *ob = r; else *oa = r;
    *ok = 1;
}

static double piece2(const pt *v, const double *nrme /* [3][3] outward unit, edge k opposite vertex k */,
                     const double *g, const double *shift, double *mass, double *mom)
{
    pt seg[16][2];
    double nrm[16][3];
    int ns = 0;
    for (int k = 0; k < 3; ++k) {
        pt a = v[(k + 1) % 3], b = v[(k + 2) % 3];
        int ok = 1;
        for (int d = 0; d < 2 && ok; ++d) {
            double e[3] = {0, 0, 0};
            e[d] = 1.0;
            clip_seg(&a, &b, e, 0.0, &a, &b, &ok);
            if (!ok) break;
            e[d] = -1.0;
            clip_seg(&a, &b, e, 1.0, &a, &b, &ok);
        }
        if (ok) {
            seg[ns][0] = a;
            seg[ns][1] = b;
            memcpy(nrm[ns], &nrme[3 * k], sizeof(double) * 3);
            ns++;
        }
    }
    for (int d = 0; d < 2; ++d) {
        for (int side = 0; side < 2; ++side) {
            double on[3] = {0, 0, 0};
            on[d] = side ? 1.0 : -1.0;
            int skip = 0;
            for (int k = 0; k < 3 && !skip; ++k) {
                int inl = 1;
                for (int i = 0; i < 3; ++i)
                    if (i != k && v[i].x[d] != (double)side) inl = 0;
                if (inl && nrme[3 * k + d] * on[d] > 0) skip = 1;
            }
            if (skip) continue;
            int d1 = 1 - d;
            pt a, b;
            memset(&a, 0, sizeof a);
            memset(&b, 0, sizeof b);
            a.x[d] = side; a.x[d1] = 0;
            b.x[d] = side; b.x[d1] = 1;
            int ok = 1;
            for (int k = 0; k < 3 && ok; ++k) {
                const double *nk = &nrme[3 * k];
                const double *pk = v[(k + 1) % 3].x;
                double neg[3] = {-nk[0], -nk[1], 0};
                clip_seg(&a, &b, neg, nk[0] * pk[0] + nk[1] * pk[1], &a, &b, &ok);
            }
            if (ok) {
                a.r = rho_at(a.x, v[0].x, v[0].r, g);
                b.r = rho_at(b.x, v[0].x, v[0].r, g);
                seg[ns][0] = a;
                seg[ns][1] = b;
                memcpy(nrm[ns], on, sizeof on);
                ns++;
            }
        }
    }
    if (ns == 0) return 0.0;
    double O[3] = {0, 0, 0};
    for (int s = 0; s < ns; ++s)
        for (int e = 0; e < 2; ++e)
            for (int d = 0; d < 2; ++d) O[d] += seg[s][e].x[d];
    O[0] /= 2 * ns;
    O[1] /= 2 * ns;
    double rO = rho_at(O, v[0].x, v[0].r, g);
    double area = 0, ms = 0, m2[2] = {0, 0};
    for (int s = 0; s < ns; ++s) {
        const pt *a = &seg[s][0], *b = &seg[s][1];
        double h = nrm[s][0] * (a->x[0] - O[0]) + nrm[s][1] * (a->x[1] - O[1]);
        double len = hypot(b->x[0] - a->x[0], b->x[1] - a->x[1]);
        double At = 0.5 * h * len;
        double r3[3] = {rO, a->r, b->r};
        const double *x3[3] = {O, a->x, b->x};
        double rs = r3[0] + r3[1] + r3[2];
        area += At;
        ms += At * rs / 3.0;
        for (int d = 0; d < 2; ++d) {
            double xs = 0, rx = 0;
            for (int i = 0; i < 3; ++i) {
                double xg = x3[i][d] + shift[d];
                xs += xg;
                rx += r3[i] * xg;
            }
            m2[d] += At / 12.0 * (rs * xs + rx);
        }
    }
    *mass = ms;
    mom[0] = m2[0];
    mom[1] = m2[1];
    mom[2] = 0;
    return area;
}

/* ------------------------------------------------------------------------ */
/* per-simplex preparation */

typedef struct {
    pt v[4];                 /* cell units, unwrapped, positively oriented */
    double nrm[4][3];        /* outward unit normals of facets (3D) / edges (2D) */
    double g[3];             /* gradient of rho in cell units */
    int64_t lo[3], hi[3];    /* integer bounding box (unwrapped cell indices) */
    double vol;              /* |volume| in cell units */
    double rmax;             /* max |rho_a| */
} prep;

/* returns 0 ok, 1 zero volume, 2 bad span, 3 bad index */
static int prepare(const or_problem *p, int64_t s, prep *o)
{
    int D = p->dim, K = D + 1;
    double x[4][3];
    double r[4];
    for (int a = 0; a < K; ++a) {
        int64_t vi = p->simp[s * K + a];
        if (vi < 0 || vi >= p->n_vert) return 3;
        for (int d = 0; d < D; ++d) x[a][d] = p->xyz[vi * D + d];
        for (int d = D; d < 3; ++d) x[a][d] = 0;
        r[a] = p->rho_per_corner ? p->rho[s * K + a] : p->rho[vi];
    }
    for (int d = 0; d < D; ++d) {
        if (!p->periodic[d]) continue;
        double L = p->extent[d];
        double mn = x[0][d], mx = x[0][d];
        for (int a = 1; a < K; ++a) {
            x[a][d] -= L * rint((x[a][d] - x[0][d]) / L);
            if (x[a][d] < mn) mn = x[a][d];
            if (x[a][d] > mx) mx = x[a][d];
        }
        if (!(mx - mn < 0.5 * L)) return 2;
    }
    for (int a = 0; a < K; ++a) {
        for (int d = 0; d < D; ++d) o->v[a].x[d] = (x[a][d] - p->origin[d]) * ((double)p->dims[d] / p->extent[d]);
        for (int d = D; d < 3; ++d) o->v[a].x[d] = 0;
        o->v[a].r = r[a];
    }
    double e[3][3];
    for (int a = 1; a < K; ++a) sub3(o->v[a].x, o->v[0].x, e[a - 1]);
    double det;
    if (D == 3) {
        double c[3];
        cross3(e[1], e[2], c);
        det = dot3(e[0], c);
    } else {
        det = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    }
    if (det == 0.0) return 1;
    if (det < 0) {
        pt t = o->v[1];
        o->v[1] = o->v[2];
        o->v[2] = t;
        for (int a = 1; a < K; ++a) sub3(o->v[a].x, o->v[0].x, e[a - 1]);
        det = -det;
    }
    o->vol = det / (D == 3 ? 6.0 : 2.0);
    /* gradient: solve E g = drho with E rows e_a (Section 3.1: M grad = drho) */
    double dr[3] = {0, 0, 0};
    for (int a = 1; a < K; ++a) dr[a - 1] = o->v[a].r - o->v[0].r;
    o->g[0] = o->g[1] = o->g[2] = 0;
    if (D == 3) {
        double c0[3], c1[3], c2[3];
        cross3(e[1], e[2], c0);
        cross3(e[2], e[0], c1);
        cross3(e[0], e[1], c2);
        for (int d = 0; d < 3; ++d) o->g[d] = (dr[0] * c0[d] + dr[1] * c1[d] + dr[2] * c2[d]) / det;
    } else {
        o->g[0] = (dr[0] * e[1][1] - dr[1] * e[0][1]) / det;
        o->g[1] = (e[0][0] * dr[1] - e[1][0] * dr[0]) / det;
    }
    /* outward unit normals: facet k opposite vertex k */
    for (int k = 0; k < K; ++k) {
        double n[3] = {0, 0, 0};
        if (D == 3) {
            int i0 = (k + 1) % 4, i1 = (k + 2) % 4, i2 = (k + 3) % 4;
            double a1[3], a2[3];
            sub3(o->v[i1].x, o->v[i0].x, a1);
            sub3(o->v[i2].x, o->v[i0].x, a2);
            cross3(a1, a2, n);
            double w[3];
            sub3(o->v[k].x, o->v[i0].x, w);
            if (dot3(n, w) > 0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
        } else {
            int i0 = (k + 1) % 3, i1 = (k + 2) % 3;
            double t0 = o->v[i1].x[0] - o->v[i0].x[0], t1 = o->v[i1].x[1] - o->v[i0].x[1];
            n[0] = t1;
            n[1] = -t0;
            double w0 = o->v[k].x[0] - o->v[i0].x[0], w1 = o->v[k].x[1] - o->v[i0].x[1];
            if (n[0] * w0 + n[1] * w1 > 0) { n[0] = -n[0]; n[1] = -n[1]; }
        }
        double l = sqrt(dot3(n, n));
        for (int d = 0; d < 3; ++d) o->nrm[k][d] = n[d] / l;
    }
    o->rmax = 0;
    for (int a = 0; a < K; ++a)
        if (fabs(o->v[a].r) > o->rmax) o->rmax = fabs(o->v[a].r);
    for (int d = 0; d < 3; ++d) {
        if (d >= D) { o->lo[d] = o->hi[d] = 0; continue; }
        double mn = o->v[0].x[d], mx = mn;
        for (int a = 1; a < K; ++a) {
            if (o->v[a].x[d] < mn) mn = o->v[a].x[d];
            if (o->v[a].x[d] > mx) mx = o->v[a].x[d];
        }
        o->lo[d] = (int64_t)floor(mn);
        o->hi[d] = (int64_t)floor(mx);
    }
    return 0;
}

static int64_t wrap_index(int64_t c, int64_t n, int periodic, int *ok)
{
    if (periodic) {
        c %= n;
        if (c < 0) c += n;
        *ok = 1;
        return c;
    }
    *ok = (c >= 0 && c < n);
    return c;
}

static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* ------------------------------------------------------------------------ */

/*
 * or_project: project every simplex; out_mass receives the mass per cell
 * (grid x fastest, [dims2][dims1][dims0]); out_cov (optional) the coverage
 * scale |G_j| * max over simplices with a piece in j of max_a |rho_a|;
 * simplex_mass / simplex_moment (optional) the sum over cells of each
 * simplex's pieces and of their rho-weighted first moments (in box units,
 * unwrapped relative to the simplex's first vertex).  Returns 0.
 */
int or_project(const or_problem *p, double *out_mass, double *out_cov, double *simplex_mass,
               double *simplex_moment, or_stats *st, int nthreads)
{
    const int D = p->dim;
    const int Dz = D - 1; /* partition axis */
    const int64_t nx = p->dims[0], ny = p->dims[1], nz = D == 3 ? p->dims[2] : 1;
    const int64_t ncell = nx * ny * nz;
    const int64_t nplanes = p->dims[Dz];
    double cellvol = 1.0;
    for (int d = 0; d < D; ++d) cellvol *= p->extent[d] / (double)p->dims[d];
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = d < D ? p->extent[d] / (double)p->dims[d] : 1.0;

    memset(st, 0, sizeof *st);
    prep *pr = (prep *)malloc(sizeof(prep) * (p->n_simplex > 0 ? p->n_simplex : 1));
    int *status = (int *)malloc(sizeof(int) * (p->n_simplex > 0 ? p->n_simplex : 1));
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t s = 0; s < p->n_simplex; ++s) status[s] = prepare(p, s, &pr[s]);
    for (int64_t s = 0; s < p->n_simplex; ++s) {
        if (status[s] == 1) st->n_zero_volume++;
        if (status[s] == 2) st->n_bad_span++;
        if (status[s] == 3) st->n_bad_index++;
    }
    /* CSR: partition plane -> (simplex, unwrapped plane index) */
    int64_t *cnt = (int64_t *)calloc(nplanes + 1, sizeof(int64_t));
    for (int64_t s = 0; s < p->n_simplex; ++s) {
        if (status[s]) continue;
        for (int64_t c = pr[s].lo[Dz]; c <= pr[s].hi[Dz]; ++c) {
            int ok;
            int64_t w = wrap_index(c, nplanes, p->periodic[Dz], &ok);
            if (ok) cnt[w + 1]++;
        }
    }
    for (int64_t i = 0; i < nplanes; ++i) cnt[i + 1] += cnt[i];
    int64_t nent = cnt[nplanes];
    int64_t *es = (int64_t *)malloc(sizeof(int64_t) * (nent > 0 ? nent : 1));
    int64_t *ec = (int64_t *)malloc(sizeof(int64_t) * (nent > 0 ? nent : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (nplanes > 0 ? nplanes : 1));
    memcpy(fill, cnt, sizeof(int64_t) * nplanes);
    for (int64_t s = 0; s < p->n_simplex; ++s) {
        if (status[s]) continue;
        for (int64_t c = pr[s].lo[Dz]; c <= pr[s].hi[Dz]; ++c) {
            int ok;
            int64_t w = wrap_index(c, nplanes, p->periodic[Dz], &ok);
            if (ok) {
                es[fill[w]] = s;
                ec[fill[w]] = c;
                fill[w]++;
            }
        }
    }
    double *lo = (double *)calloc(ncell, sizeof(double));
    double *ent_mass = simplex_mass ? (double *)calloc(nent > 0 ? nent : 1, sizeof(double)) : NULL;
    double *ent_mom = simplex_moment ? (double *)calloc(3 * (nent > 0 ? nent : 1), sizeof(double)) : NULL;
    memset(out_mass, 0, sizeof(double) * ncell);
    if (out_cov) memset(out_cov, 0, sizeof(double) * ncell);
    int64_t ncand = 0, npiece = 0;

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : ncand, npiece)
    for (int64_t w = 0; w < nplanes; ++w) {
        for (int64_t e = cnt[w]; e < cnt[w + 1]; ++e) {
            const prep *P = &pr[es[e]];
            int64_t cz = ec[e];
            int64_t ylo = D == 3 ? P->lo[1] : cz, yhi = D == 3 ? P->hi[1] : cz;
            int64_t zz = D == 3 ? cz : 0;
            for (int64_t cy = ylo; cy <= yhi; ++cy) {
                int oky;
                int64_t wy = wrap_index(cy, ny, p->periodic[1], &oky);
                if (!oky) continue;
                for (int64_t cx = P->lo[0]; cx <= P->hi[0]; ++cx) {
                    int okx;
                    int64_t wx = wrap_index(cx, nx, p->periodic[0], &okx);
                    if (!okx) continue;
                    int64_t wz = D == 3 ? w : 0;
                    int64_t cell = wx + nx * (wy + ny * wz);
                    if (p->cell_mask && !p->cell_mask[cell]) continue;
                    ncand++;
                    double sh[3] = {(double)cx, (double)cy, (double)zz};
                    pt lv[4];
                    for (int a = 0; a <= D; ++a) {
                        lv[a] = P->v[a];
                        for (int d = 0; d < D; ++d) lv[a].x[d] -= sh[d];
                    }
                    double ms = 0, mom[3] = {0, 0, 0}, vol;
                    if (D == 3)
                        vol = piece3(lv, &P->nrm[0][0], P->g, sh, &ms, mom);
                    else
                        vol = piece2(lv, &P->nrm[0][0], P->g, sh, &ms, mom);
                    if (!(vol > 0)) continue;
                    npiece++;
                    double mass = ms * cellvol;
                    double s2, e2;
                    two_sum(out_mass[cell], mass, &s2, &e2);
                    out_mass[cell] = s2;
                    lo[cell] += e2;
                    if (out_cov) {
                        double c = P->rmax * cellvol;
                        if (c > out_cov[cell]) out_cov[cell] = c;
                    }
                    if (ent_mass) ent_mass[e] += mass;
                    if (ent_mom)
                        for (int d = 0; d < D; ++d) ent_mom[3 * e + d] += mom[d] * cellvol * h[d];
                }
            }
        }
    }
    for (int64_t c = 0; c < ncell; ++c) out_mass[c] += lo[c];
    st->n_candidates = ncand;
    st->n_pieces = npiece;
    if (simplex_mass) {
        memset(simplex_mass, 0, sizeof(double) * p->n_simplex);
        for (int64_t e = 0; e < nent; ++e) simplex_mass[es[e]] += ent_mass[e];
    }
    if (simplex_moment) {
        memset(simplex_moment, 0, sizeof(double) * 3 * p->n_simplex);
        for (int64_t e = 0; e < nent; ++e) {
            /* moments were accumulated in unwrapped cell units; convert to box
             * units by adding the origin times the mass */
            for (int d = 0; d < D; ++d)
                simplex_moment[3 * es[e] + d] += ent_mom[3 * e + d] + p->origin[d] * ent_mass[e];
        }
    }
    free(lo);
    free(ent_mass);
    free(ent_mom);
    free(es);
    free(ec);
    free(fill);
    free(cnt);
    free(pr);
    free(status);
    return 0;
}

/* Per-simplex exact mass |V| * mean(rho) in box units (Section 3.1: the
 * integral of a linear function over a simplex is its volume times the mean
 * of its vertex values).  Skipped simplices get 0. */
void or_simplex_mass(const or_problem *p, double *out)
{
    double cellvol = 1.0;
    for (int d = 0; d < p->dim; ++d) cellvol *= p->extent[d] / (double)p->dims[d];
    for (int64_t s = 0; s < p->n_simplex; ++s) {
        prep P;
        if (prepare(p, s, &P)) { out[s] = 0; continue; }
        double rs = 0;
        for (int a = 0; a <= p->dim; ++a) rs += P.v[a].r;
        out[s] = P.vol * cellvol * rs / (p->dim + 1);
    }
}

int or_version(void) { return 1; }
