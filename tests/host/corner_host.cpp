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
