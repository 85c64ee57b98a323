// Host build of the projection's per-simplex set-up and sweep (the headers
// the clip kernel uses), for CPU tests of their logic against the oracle:
// the sweep over slab groups, and the overflow protocol (a sweep that runs
// out of polytope slots reports the first piece it did not deposit; a
// second sweep with more slots resumes there, skipping the pieces before
// it).  Grid: origin 0, unit box, dims[d] cells, so the cell coordinate of
// x is x * dims exactly when dims is a power of two.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "sp_setup.h"

using namespace sp;

namespace {

struct HostDep {
    double *grid;
    int anchor[3], dims[3], periodic[3];
    long stride[3];
    int suppress_ix = -1, suppress_iy = 0, suppress_iz = 0;
    long count = 0;
    void operator()(int ix, int iy, int iz, float v)
    {
        if (ix == suppress_ix && (iy < suppress_iy || (iy == suppress_iy && iz < suppress_iz))) return;
        ++count;
        int c[3] = {anchor[0] + ix, anchor[1] + iy, anchor[2] + iz};
        for (int d = 0; d < 3; ++d) {
            if (periodic[d]) {
                c[d] %= dims[d];
                if (c[d] < 0) c[d] += dims[d];
            } else if (c[d] < 0 || c[d] >= dims[d]) {
                return;
            }
        }
        grid[c[0] * stride[0] + c[1] * stride[1] + c[2] * stride[2]] += v;
    }
};

template <int MAXV>
bool sweep_from(const Local<float> &L, int sb, int sc, int ry, HostDep &dep, int *fail)
{
    static P3T<float> pos[MAXV];
    static uint16_t nbw[MAXV];
    Poly3<float, MAXV, 1> P;
    P.pp = pos;
    P.pn = nbw;
    P.live = 0u;
    return sweep3<float, MAXV, 1>(P, L, sb, sc, dep, ry, fail);
}

}  // namespace

// stats: [0] skipped at set-up, [1] single-cell, [2] items, [3] items that
// overflowed the small polytope and were resumed, [4] resumes that failed,
// [5] pieces deposited
extern "C" int sweep_host(const float *xyz, int64_t n_vert, const int32_t *simp, int64_t n, const float *rho,
                          int per_corner, const int *dims, const int *periodic, int slab_group, int small_slots,
                          double *out, long *stats)
{
    GridDev g;
    memset(&g, 0, sizeof g);
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = dims[d];
        g.periodic[d] = periodic[d];
        g.s_hi[d] = (float)dims[d];
        g.scale[d] = dims[d];
        g.extent[d] = 1.0;
    }
    const long stride[3] = {1, (long)dims[0], (long)dims[0] * dims[1]};
    for (int k = 0; k < 6; ++k) stats[k] = 0;
    for (int64_t s = 0; s < n; ++s) {
        Local<float> L0;
        if (setup_f32<3>(xyz, n_vert, simp, s, rho, per_corner != 0, g, true, L0) != SETUP_OK) {
            stats[0]++;
            continue;
        }
        const SweepOrder o = sweep_order(L0);
        const Local<float> L = permuted(L0, o);
        HostDep dep;
        dep.grid = out;
        for (int d = 0; d < 3; ++d) {
            dep.anchor[d] = L.anchor[d];
            dep.dims[d] = dims[o.ax[d]];
            dep.periodic[d] = periodic[o.ax[d]];
            dep.stride[d] = stride[o.ax[d]];
        }
        if (L0.span[0] == 1 && L0.span[1] == 1 && L0.span[2] == 1) {
            stats[1]++;
            HostDep d0 = dep;
            for (int d = 0; d < 3; ++d) {
                d0.anchor[d] = L0.anchor[d];
                d0.dims[d] = dims[d];
                d0.periodic[d] = periodic[d];
                d0.stride[d] = stride[d];
            }
            d0(0, 0, 0, L0.det * (L0.v[0].r + L0.v[1].r + L0.v[2].r + L0.v[3].r) / 24.0f);
            stats[5]++;
            continue;
        }
        const int sx = L.span[0];
        const int nit = (sx + slab_group - 1) / slab_group, per = (sx + nit - 1) / nit;
        for (int k = 0; k < nit; ++k) {
            const int sb = k * per, sc = sx - sb < per ? sx - sb : per;
            if (sc <= 0) continue;
            stats[2]++;
            int fail[3];
            HostDep d1 = dep;
            const bool ok = small_slots ? sweep_from<10>(L, sb, sc, 0, d1, fail) : sweep_from<18>(L, sb, sc, 0, d1, fail);
            stats[5] += d1.count;
            if (ok) continue;
            // resume with room to spare from the first piece not deposited
            stats[3]++;
            HostDep d2 = dep;
            d2.suppress_ix = fail[0];
            d2.suppress_iy = fail[1];
            d2.suppress_iz = fail[2];
            int fail2[3];
            if (!sweep_from<32>(L, fail[0], sb + sc - fail[0], fail[1], d2, fail2)) stats[4]++;
            stats[5] += d2.count;
        }
    }
    return 0;
}

// Set-up status and outermost span of one triangle (corners in cell units)
// on a periodic dims[0] x dims[1] grid over the unit box: the 2D case whose
// x-span has to fit the 16-bit fields of the binning records.
extern "C" int setup_tri_host(const float *corners, const int *dims, int *span_out)
{
    GridDev g;
    memset(&g, 0, sizeof g);
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = d < 2 ? dims[d] : 1;
        g.periodic[d] = 1;
        g.s_hi[d] = (float)g.dims[d];
        g.scale[d] = g.dims[d];
        g.extent[d] = 1.0;
    }
    float xyz[6];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 2; ++d) xyz[2 * a + d] = corners[2 * a + d] / (float)dims[d];
    const int32_t simp[3] = {0, 1, 2};
    const float rho[3] = {1.f, 1.f, 1.f};
    Local<float> L;
    const int st = setup_f32<2>(xyz, 3, simp, 0, rho, false, g, true, L);
    span_out[0] = L.span[0];
    span_out[1] = L.span[1];
    return st;
}

// Round trip of the binning records for a simplex of outer span sx cut into
// nit work items: 0 when the set-up record decodes to (cls, nit, sx) and the
// items, decoded, cover slabs [0, sx) once each in order; else a code.
extern "C" int pack_roundtrip_host(int cls, int nit, int sx, uint32_t simplex)
{
    const uint32_t r = pack_setup(cls, nit, sx);
    if (setup_class(r) != cls || setup_items(r) != nit || setup_span(r) != sx) return 1;
    int next = 0;
    for (int k = 0; k < nit; ++k) {
        int sb, sc;
        item_range(sx, nit, k, sb, sc);
        const uint64_t it = pack_item(simplex, sb, sc);
        if (item_simplex(it) != simplex || item_first(it) != sb || item_count(it) != sc) return 2;
        if (sc > 0 && sb != next) return 3;
        next = sc > 0 ? sb + sc : next;
    }
    return next == sx ? 0 : 4;
}
