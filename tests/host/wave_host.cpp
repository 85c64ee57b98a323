// Host build of the group sweep (sp_wave.h: one polytope per 16 lanes,
// emulated here one lane after the other), for CPU tests against the oracle:
// the same set-up, item split and overflow protocol as the clip kernel (an
// item that runs out of slots is finished by the one-polytope-per-lane sweep
// from its first undeposited piece, skipping the pieces before it).
#include <cmath>
#include <cstdint>
#include <cstring>

#include "sp_wave.h"

using namespace sp;

namespace sp {
namespace wv {
thread_local int wv_cur_lane = 0;
}
}  // namespace sp

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

}  // namespace

// stats: [0] skipped at set-up, [1] single-cell, [2] items, [3] items handed
// to the per-lane sweep after a failure, [4] per-lane resumes that failed,
// [5] pieces deposited, [6] group steps
extern "C" int wave_host(const float *xyz, int64_t n_vert, const int32_t *simp, int64_t n, const float *rho,
                         int per_corner, const int *dims, const int *periodic, int slab_group, double *out, long *stats)
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
    for (int k = 0; k < 7; ++k) stats[k] = 0;
    static wv::GroupLDS sh;
    static P3T<float> pos[32];
    static uint16_t nbw[32];
    for (int64_t s = 0; s < n; ++s) {
        Local<float> L0;
        double ex0[4][3], ex[4][3];
        if (setup_f32<3>(xyz, n_vert, simp, s, rho, per_corner != 0, g, true, L0, ex0) != SETUP_OK) {
            stats[0]++;
            continue;
        }
        const SweepOrder o = sweep_order(L0);
        const Local<float> L = permuted(L0, o);
        permuted_exact(ex0, o, ex);
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
        const int nit = (sx + slab_group - 1) / slab_group;
        for (int k = 0; k < nit; ++k) {
            int sb, sc;
            item_range(sx, nit, k, sb, sc);
            if (sc <= 0) continue;
            stats[2]++;
            HostDep d1 = dep;
            wv::Sweep S;
            wv::sweep_start(&sh, S, L, ex, sb, sc);
            bool ok = true;
            while (S.phase != wv::PH_IDLE) {
                stats[6]++;
                if (!wv::sweep_step(&sh, S, d1)) {
                    ok = false;
                    break;
                }
            }
            stats[5] += d1.count;
            if (ok) continue;
            // finish with the per-lane sweep from the first piece not deposited
            stats[3]++;
            HostDep d2 = dep;
            d2.suppress_ix = S.fail[0];
            d2.suppress_iy = S.fail[1];
            d2.suppress_iz = S.fail[2];
            Poly3<float, 32, 1> P;
            P.pp = pos;
            P.pn = nbw;
            P.live = 0u;
            int fail2[3];
            if (!sweep3<float, 32, 1>(P, L, S.fail[0], sb + sc - S.fail[0], d2, S.fail[1], fail2)) stats[4]++;
            stats[5] += d2.count;
        }
    }
    return 0;
}
