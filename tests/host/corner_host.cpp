// Host build of the corner-sum projection (the header the corner kernel
// uses), for CPU tests of its logic against the oracle.  Grid: origin 0,
// unit box, dims[d] cells; mass per cell out.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "sp_corner.h"

using namespace sp;

namespace {

struct HostDep {
    double *grid;
    int anchor[3], dims[3], periodic[3];
    long stride[3];
    long count = 0;
    void operator()(int ix, int iy, int iz, double v)
    {
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

// stats: [0] skipped at set-up, [1] simplices summed, [2] degenerate
// configurations met, [3] terms deposited
extern "C" int corner_host(const double *xyz, int64_t n_vert, const int32_t *simp, int64_t n, const double *rho,
                           int per_corner, const int *dims, const int *periodic, double *out, long *stats)
{
    GridDev g;
    memset(&g, 0, sizeof g);
    double cellvol = 1.0;
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = dims[d];
        g.periodic[d] = periodic[d];
        g.scale[d] = dims[d];
        g.extent[d] = 1.0;
        cellvol /= dims[d];
    }
    const long stride[3] = {1, (long)dims[0], (long)dims[0] * dims[1]};
    for (int k = 0; k < 4; ++k) stats[k] = 0;
    for (int64_t s = 0; s < n; ++s) {
        Local<double> L;
        if (setup_f64<3>(xyz, n_vert, simp, s, rho, per_corner != 0, g, true, L) != SETUP_OK) {
            stats[0]++;
            continue;
        }
        HostDep dep;
        dep.grid = out;
        for (int d = 0; d < 3; ++d) {
            dep.anchor[d] = L.anchor[d];
            dep.dims[d] = dims[d];
            dep.periodic[d] = periodic[d];
            dep.stride[d] = stride[d];
        }
        stats[1]++;
        stats[2] += corner_project(L, dep);
        stats[3] += dep.count;
    }
    for (long i = 0; i < (long)dims[0] * dims[1] * dims[2]; ++i) out[i] *= cellvol;
    return 0;
}

#include <algorithm>
#include <array>
#include <map>
#include <vector>

// The same projection with the fused facet contributions: facets shared by
// two summed simplices (matched by their vertex ids) are summed once, by the
// simplex of lower index.  stats as above, plus [4] facets paired and [5]
// simplices left out of the fusion (slivers).
extern "C" int corner_host_fused(const double *xyz, int64_t n_vert, const int32_t *simp, int64_t n, const double *rho,
                                 int per_corner, const int *dims, const int *periodic, double *out, long *stats)
{
    GridDev g;
    memset(&g, 0, sizeof g);
    double cellvol = 1.0;
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = dims[d];
        g.periodic[d] = periodic[d];
        g.scale[d] = dims[d];
        g.extent[d] = 1.0;
        cellvol /= dims[d];
    }
    const long stride[3] = {1, (long)dims[0], (long)dims[0] * dims[1]};
    for (int k = 0; k < 6; ++k) stats[k] = 0;
    std::vector<Local<double>> L(n);
    std::vector<char> ok(n, 0);
    std::vector<std::array<int64_t, 4>> vid(n);
    std::vector<D3> grad(n);
    std::vector<std::array<int, 4>> side(n);
    std::map<std::array<int64_t, 3>, std::vector<int64_t>> facets;  // sorted vertex ids -> facet ids s * 4 + m
    for (int64_t s = 0; s < n; ++s) {
        bool sw = false;
        if (setup_f64<3>(xyz, n_vert, simp, s, rho, per_corner != 0, g, true, L[s], &sw) != SETUP_OK) continue;
        for (int a = 0; a < 4; ++a) vid[s][a] = simp[s * 4 + (sw && (a == 1 || a == 2) ? 3 - a : a)];
        ok[s] = 1;
        grad[s] = corner_gradient(L[s]);
        if (!corner_fusable(L[s], grad[s])) {
            stats[5]++;
            continue;
        }
        for (int m = 0; m < 4; ++m) {
            side[s][m] = facet_side(L[s], vid[s].data(), m);
            std::array<int64_t, 3> key;
            int c = 0;
            for (int a = 0; a < 4; ++a)
                if (a != m) key[c++] = vid[s][a];
            std::sort(key.begin(), key.end());
            if (side[s][m] != 0) facets[key].push_back(s * 4 + m);
        }
    }
    std::vector<int64_t> mate(4 * n, -1);
    for (auto &kv : facets)
        if (kv.second.size() == 2) {
            mate[kv.second[0]] = kv.second[1];
            mate[kv.second[1]] = kv.second[0];
            stats[4]++;
        }
    for (int64_t s = 0; s < n; ++s) {
        if (!ok[s]) {
            stats[0]++;
            continue;
        }
        FacetFuse fz;
        fz.cell_origin = false;
        for (int m = 0; m < 4; ++m) {
            fz.mode[m] = FACET_PLAIN;
            const int64_t f = mate[s * 4 + m];
            if (f < 0) continue;
            fz.cell_origin = true;
            const int64_t j = f / 4;
            const int mj = (int)(f % 4);
            if (j < s) {
                fz.mode[m] = FACET_SKIP;
                continue;
            }
            const int a = m == 0 ? 1 : 0;  // a corner of the facet
            double rj = rho[vid[s][a]];
            if (per_corner)
                for (int k = 0; k < 4; ++k)
                    if (simp[j * 4 + k] == vid[s][a]) rj = rho[j * 4 + k];
            fuse_facet(fz, m, L[s], grad[s], a, grad[j], rj, side[s][m] * side[j][mj]);
        }
        HostDep dep;
        dep.grid = out;
        for (int d = 0; d < 3; ++d) {
            dep.anchor[d] = L[s].anchor[d];
            dep.dims[d] = dims[d];
            dep.periodic[d] = periodic[d];
            dep.stride[d] = stride[d];
        }
        stats[1]++;
        stats[2] += corner_project(L[s], dep, &fz);
        stats[3] += dep.count;
    }
    for (long i = 0; i < (long)dims[0] * dims[1] * dims[2]; ++i) out[i] *= cellvol;
    return 0;
}
