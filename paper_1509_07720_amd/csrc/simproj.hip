// simproj.hip -- MI355X (gfx950) kernels and C-ABI runtime for the exact
// projection of a piecewise-linear density on a simplicial mesh onto a
// regular grid (Section 3.1, eq. eq_firstOrder).
//
// Path of one call (sp_project_tets / sp_project_tris):
//   k_fill      zero the output (unless SP_ACCUMULATE) and the per-call state
//   k_setup     per simplex: gather, unwrap, cell coordinates, orientation;
//               a simplex inside one cell deposits its whole mass at once
//               (Appendix D, first step; merged per cell and block first);
//               the others are binned into cost classes, big ones cut into
//               work items of consecutive x-slabs sized by expected pieces
//   k_scan      class offsets, most expensive class first
//   k_scatter   the work items in class order
//   k_clip      persistent waves pull 64 items at a time; each lane sweeps
//               its simplex through slabs, columns and cells, clipping a
//               polytope held in LDS and depositing each piece
//   k_clip(big) items whose polytope overflowed, resumed with more room
//   k_finalize  hi+lo -> out, FP64 total mass
// Other entry points: sp_vertex_density (k_vd_accum, k_vd_finish), the
// accuracy-controlled projection (k_flag, k_tag, k_widen, k_gather_tagged,
// k_patch), the adaptive-grid projection (k_amr_level, k_amr_mark, k_amr_refine,
// k_amr_plevel, k_amr_scatter, k_amr_restrict, k_amr_gather),
// the corner-sum projection (k_corner) and the batched launch (the same
// kernels over many problems, captured in a graph).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "simproj.h"
#include "sp_corner.h"
#include "sp_setup.h"
#include "sp_wave.h"

using namespace sp;

namespace {

constexpr int WG = 64;       // lanes per block in the clip kernels (one wave)
constexpr int NCLS = 16;     // cost classes
// Precision route of FP32C problems: a simplex whose bounding box spans
// WIDE_SPAN cells or more along some axis is clipped and integrated in FP64
// (its pieces deposited compensated into the FP32 grids).  Positions local
// to a simplex carry a rounding of half an ulp of its span (u times the span),
// and at 64 cells that is 3.8e-6 of a cell, the most the per-cell bound of
// 1e-5 leaves room for.  Such simplices get the class CLS_WIDE, which no
// other simplex uses; their work items come first in the list.
constexpr int WIDE_SPAN = 64;
constexpr int CLS_WIDE = NCLS - 1;
// Polytope vertex slots per lane.  A cut frees the removed vertices it no
// longer reads before it places new ones, so its peak stays near the larger
// of the two polytopes.  FP32: 14 slots (12.3 KB of LDS per wave) let 12 waves
// share a CU when the kernel keeps to 168 VGPRs (3 waves per SIMD); the
// kernel is latency bound, and every wave counts (9 waves ran 9 % faster
// than 8).  No 10M-tet soup item needed more than 14; one that does is
// finished by the 32-slot kernel.  FP64: 15 slots, 6 waves.  (A slot is
// 12 + 2 bytes in FP32 and 24 + 4 in FP64: positions and neighbour words
// in separate arrays.)
template <typename T>
constexpr int maxv3() { return sizeof(T) == 4 ? 14 : 15; }
constexpr int MAXV3_BIG = 32;
constexpr int MAXP2 = 12;    // polygon vertices per lane and buffer (peak 8)
constexpr int OVF_CAP = 1 << 20;  // overflow records per launch (24 MB of scratch)
// Lanes of a wave that build their next columns together (see k_clip):
// on the 10M-tet soup 40 measured best among 16..48 and among thresholds
// relative to the busy lanes (the clip 10 % faster than building at once).
constexpr int BUILD_MIN = 40;
// Cells in a wave's deposit tile (the opt-in tiled FP32 clip kernel).
constexpr int DEP_TILE = 64;

// Per-call device state, cleared at the start of every call.
struct CallState {
    unsigned hist[NCLS];
    unsigned cursor[NCLS];
    unsigned total;
    unsigned head;
    unsigned head_wide;
    unsigned extra;
    unsigned ovf_count;
    unsigned ovf_head;
    unsigned pad;
    unsigned long long pieces;
};

// Error state, kept until sp_sync_status reads and clears it.
struct ErrState {
    int first;
    int n_bad_index;
    int n_nonfinite;
    int n_bad_span;
    int n_overflow;
    int n_internal;
    int n_degenerate;  // corner sums: simplices not summed (bounding box over 2^24 cells)
};

struct Ovf {
    int s, ix, iy, iz, end, pid;
};

struct Tuning {
    int slab_group;   // at most this many x-slabs per work item
    int chunks_per_cu; // persistent blocks per CU in the clip kernel (0: occupancy)
    int item_pieces;  // expected pieces a work item is cut down to (0: from the launch size)
};

// Expected pieces per work item: one lane's expected share of the launch
// (16 pieces per simplex assumed, a nominal 9 waves of 64 lanes per CU: the
// sizes for the waves that actually run, 11 when measured, gave the same
// times), within
// [16, 1024].  Few simplices (big ones, as a rule) are cut into many items
// so that every lane has work; many small ones stay whole, which saves the
// per-item set-up and column rebuilds.
static int auto_item_pieces(int64_t nsimplex, int num_cu)
{
    const double lanes = (double)num_cu * 9.0 * 64.0;
    const double b = 16.0 * (double)nsimplex / lanes;
    return b < 16.0 ? 16 : (b > 1024.0 ? 1024 : (int)b);
}

__device__ inline void record_error(ErrState *e, int code)
{
    atomicCAS(&e->first, 0, code);
}

// ---------------------------------------------------------------------------
// deposits

// Compensated FP32 deposit: the returning atomic gives the value the add was
// applied to; TwoSum recovers its exact rounding error, which goes to the
// low grid, so hi + lo keeps the exact sum up to the rounding of the low
// parts (Knuth's TwoSum; requires round-to-nearest atomics).
struct DepF32 {
    float *hi;
    float *lo;
    uint32_t *cmax;  // optional: largest |contribution| per cell, as float bits
    int anchor[3];   // along the sweep axes
    int dims[3];
    int periodic[3];
    size_t stride[3];
    float scale;
    int suppress_iy, suppress_iz, suppress_ix;  // resume: skip pieces before this one
    int count;
    // Optional per-wave deposit tile in LDS (the tiled instance of the FP32
    // clip kernel; null otherwise): DEP_TILE cells of (key, hi, lo) in
    // which pieces of one cell merge before one compensated grid deposit.
    uint32_t *tkey;
    float *thi, *tlo;
    static constexpr uint32_t TILE_EMPTY = 0xffffffffu;

    // a piece computed in FP64 (a simplex routed to FP64)
    __device__ void operator()(int ix, int iy, int iz, double v)
    {
        if (ix == suppress_ix && (iy < suppress_iy || (iy == suppress_iy && iz < suppress_iz))) return;
        ++count;
        size_t idx;
        if (cell(ix, iy, iz, idx)) add(idx, v);
    }

    __device__ void operator()(int ix, int iy, int iz, float v)
    {
#pragma clang fp contract(off)
        if (ix == suppress_ix && (iy < suppress_iy || (iy == suppress_iy && iz < suppress_iz))) return;
        ++count;
        size_t idx;
        if (!cell(ix, iy, iz, idx)) return;
        float x = v * scale;
        if (cmax) atomicMax(cmax + idx, __float_as_uint(fabsf(x)));
        if (tkey && tile_add(idx, x)) return;
        float old = unsafeAtomicAdd(hi + idx, x);
        float s = old + x;
        float bb = s - old;
        float err = (old - (s - bb)) + (x - bb);
        if (err != 0.0f) unsafeAtomicAdd(lo + idx, err);
    }

    // Grid deposit of a merged cell: its high part with the compensated
    // add; the rounding error and its low part go to the low grid.
    static __device__ void flush(float *hi, float *lo, size_t idx, float h, float l)
    {
#pragma clang fp contract(off)
        float old = unsafeAtomicAdd(hi + idx, h);
        float s = old + h;
        float bb = s - old;
        float err = (old - (s - bb)) + (h - bb) + l;
        if (err != 0.0f) unsafeAtomicAdd(lo + idx, err);
    }

    // Piece x of cell idx (< TILE_EMPTY) into the wave's tile: added there
    // (LDS atomics, with TwoSum into the entry's low part) when the cell
    // holds its hashed slot, else the lane tries to take the slot over,
    // flushing the cell it evicts.  False when another lane took the slot
    // first: the caller deposits directly.  The lanes of the wave run this
    // in lockstep; every add into a cell already in the tile is issued
    // before any take-over, and LDS operations of a wave complete in order.
    __device__ bool tile_add(size_t idx, float x) const
    {
#pragma clang fp contract(off)
        const uint32_t key = (uint32_t)idx;
        const uint32_t t = (key * 2654435761u) >> 26;  // multiplicative hash onto 64 slots
        const uint32_t k = tkey[t];
        const bool match = k == key;
        if (match) {
            float old = atomicAdd(thi + t, x);
            float s = old + x;
            float bb = s - old;
            float err = (old - (s - bb)) + (x - bb);
            if (err != 0.0f) atomicAdd(tlo + t, err);
        }
        __builtin_amdgcn_wave_barrier();
        if (match) return true;
        if (atomicCAS(tkey + t, k, key) != k) return false;
        const float oh = atomicExch(thi + t, x);
        const float ol = atomicExch(tlo + t, 0.0f);
        if (k != TILE_EMPTY) flush(hi, lo, (size_t)k, oh, ol);
        return true;
    }

    // Global index of local cell (ix, iy, iz); false outside a non-periodic
    // grid.  With add(), the two halves of operator() for callers that merge
    // contributions to one cell first.
    __device__ bool cell(int ix, int iy, int iz, size_t &idx) const
    {
        // periodic anchors are reduced to [0, dims) and local indices lie
        // within a span of at most half the box (one below it at worst), so
        // one conditional step wraps a periodic index
        int c[3] = {anchor[0] + ix, anchor[1] + iy, anchor[2] + iz};
        for (int d = 0; d < 3; ++d) {
            if (periodic[d]) {
                c[d] = c[d] >= dims[d] ? c[d] - dims[d] : (c[d] < 0 ? c[d] + dims[d] : c[d]);
            } else if ((unsigned)c[d] >= (unsigned)dims[d]) {
                return false;
            }
        }
        idx = (size_t)c[0] * stride[0] + (size_t)c[1] * stride[1] + (size_t)c[2] * stride[2];
        return true;
    }
    __device__ void add(size_t idx, double v) const
    {
#pragma clang fp contract(off)
        // the FP64 value as a float and the float remainder: the remainder
        // joins the low grid with the rounding error of the high sum
        const double w = v * (double)scale;
        const float x = (float)w;
        const float rem = (float)(w - (double)x);
        if (cmax) atomicMax(cmax + idx, __float_as_uint(fabsf(x)));
        float old = unsafeAtomicAdd(hi + idx, x);
        float s = old + x;
        float bb = s - old;
        float err = (old - (s - bb)) + (x - bb) + rem;
        if (err != 0.0f) unsafeAtomicAdd(lo + idx, err);
    }
};

struct DepF64 {
    double *out;
    int anchor[3];   // along the sweep axes
    int dims[3];
    int periodic[3];
    size_t stride[3];
    double scale;
    int suppress_iy, suppress_iz, suppress_ix;
    int count;

    __device__ void operator()(int ix, int iy, int iz, double v)
    {
        if (ix == suppress_ix && (iy < suppress_iy || (iy == suppress_iy && iz < suppress_iz))) return;
        ++count;
        // periodic anchors are reduced to [0, dims) and local indices lie
        // within a span of at most half the box (one below it at worst), so
        // one conditional step wraps a periodic index
        int c[3] = {anchor[0] + ix, anchor[1] + iy, anchor[2] + iz};
        for (int d = 0; d < 3; ++d) {
            if (periodic[d]) {
                c[d] = c[d] >= dims[d] ? c[d] - dims[d] : (c[d] < 0 ? c[d] + dims[d] : c[d]);
            } else if ((unsigned)c[d] >= (unsigned)dims[d]) {
                return;
            }
        }
        size_t idx = (size_t)c[0] * stride[0] + (size_t)c[1] * stride[1] + (size_t)c[2] * stride[2];
        unsafeAtomicAdd(out + idx, v * scale);
    }

    __device__ bool cell(int ix, int iy, int iz, size_t &idx) const
    {
        int c[3] = {anchor[0] + ix, anchor[1] + iy, anchor[2] + iz};
        for (int d = 0; d < 3; ++d) {
            if (periodic[d]) {
                c[d] = c[d] >= dims[d] ? c[d] - dims[d] : (c[d] < 0 ? c[d] + dims[d] : c[d]);
            } else if ((unsigned)c[d] >= (unsigned)dims[d]) {
                return false;
            }
        }
        idx = (size_t)c[0] * stride[0] + (size_t)c[1] * stride[1] + (size_t)c[2] * stride[2];
        return true;
    }
    __device__ void add(size_t idx, double v) const { unsafeAtomicAdd(out + idx, v * scale); }
};

template <typename T>
struct DepFor;
template <>
struct DepFor<float> {
    using type = DepF32;
};
template <>
struct DepFor<double> {
    using type = DepF64;
};

// ---------------------------------------------------------------------------
// problem description as the kernels see it

// Per-simplex set-up handed from k_setup to the 3D clip kernels: the local
// frame relabelled to the sweep order, that order and the density gradient
// (the FP64 solve through the corner values), so that a clip lane starting
// a simplex loads one record instead of repeating the set-up.  Written for
// every simplex that gets work items, except those routed to FP64.
template <typename T>
struct SimplexRec {
    V4<T> v[4];
    int anchor[3];
    int span[3];
    T det;
    int order;  // sweep axes: ax[0] | ax[1] << 2 | ax[2] << 4
    double gd[3];
};

SP_HD inline int pack_order(const SweepOrder &o) { return o.ax[0] | (o.ax[1] << 2) | (o.ax[2] << 4); }
SP_HD inline SweepOrder unpack_order(int w)
{
    SweepOrder o;
    o.ax[0] = w & 3;
    o.ax[1] = (w >> 2) & 3;
    o.ax[2] = (w >> 4) & 3;
    return o;
}

template <typename T>
struct ProbDev {
    const T *xyz;
    int64_t n_vert;
    const int32_t *simp;
    int64_t n;
    const T *rho;
    int per_corner;
    int validate;
    GridDev g;
    T *out;        // hi (FP32C) or the grid (FP64)
    float *lo;     // FP32C low grid
    uint32_t *tinfo;        // this problem's slice
    SimplexRec<T> *rec;     // this problem's slice (3D)
    uint64_t *items;        // shared by all problems of a launch
    uint16_t *item_prob;    // problem of each item (batches only)
    unsigned extra_cap;
    Ovf *ovf;
    CallState *cs;
    ErrState *es;
    int slab_group;
    float item_pieces;
    int count_pieces;
    uint32_t *cmax;  // FP32C: per-cell largest contribution (accuracy control), or NULL
};

// Several problems in one launch: their descriptors in device memory and,
// for the per-simplex kernels, the first 256-thread block of each problem
// (the blocks of a problem are contiguous, so the problem is uniform per
// block; boffs[nprob] = all blocks).  nprob == 0 means a single problem
// passed by value.
struct Batch {
    const void *probs;
    const int32_t *boffs;
    int nprob;
};

// Problem of this block and the index of its first simplex.
template <typename T>
__device__ inline void block_problem(const Batch &b, ProbDev<T> &p, int64_t &s0, int &pi)
{
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = b.nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.boffs[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    pi = lo;
    p = static_cast<const ProbDev<T> *>(b.probs)[lo];
    s0 = (int64_t)(blk - b.boffs[lo]) * blockDim.x;
}

template <int D>
__device__ inline int setup_any(const ProbDev<float> &p, int64_t s, bool validate, Local<float> &L)
{
    return setup_f32<D>(p.xyz, p.n_vert, p.simp, s, p.rho, p.per_corner != 0, p.g, validate, L);
}
template <int D>
__device__ inline int setup_any(const ProbDev<double> &p, int64_t s, bool validate, Local<double> &L)
{
    return setup_f64<D>(p.xyz, p.n_vert, p.simp, s, p.rho, p.per_corner != 0, p.g, validate, L);
}
// a simplex of an FP32C problem routed to FP64 (float inputs, double set-up)
template <int D>
__device__ inline int setup_any(const ProbDev<float> &p, int64_t s, bool validate, Local<double> &L)
{
    return setup_f64<D, float>(p.xyz, p.n_vert, p.simp, s, p.rho, p.per_corner != 0, p.g, validate, L);
}

constexpr SweepOrder kIdentity = {{0, 1, 2}};

__device__ inline int wrap_index(int k, int n)
{
    k %= n;
    return k < 0 ? k + n : k;
}

// Deposit for a simplex swept in order o (L already relabelled by o); the
// grid type follows the problem, whatever precision the simplex is clipped
// in (TL).
template <typename TL>
__device__ inline DepF32 make_dep(const ProbDev<float> &p, const Local<TL> &L, const SweepOrder &o)
{
    DepF32 d;
    d.hi = p.out;
    d.lo = p.lo;
    d.cmax = p.cmax;
    const size_t s1 = (size_t)p.g.dims[0], s2 = (size_t)p.g.dims[0] * (size_t)p.g.dims[1];
    for (int k = 0; k < 3; ++k) {
        d.dims[k] = sel3(p.g.dims[0], p.g.dims[1], p.g.dims[2], o.ax[k]);
        d.periodic[k] = sel3(p.g.periodic[0], p.g.periodic[1], p.g.periodic[2], o.ax[k]);
        d.anchor[k] = d.periodic[k] ? wrap_index(L.anchor[k], d.dims[k]) : L.anchor[k];
        d.stride[k] = sel3((size_t)1, s1, s2, o.ax[k]);
    }
    d.scale = (float)p.g.out_scale;
    d.suppress_ix = -1;
    d.suppress_iy = 0;
    d.suppress_iz = 0;
    d.count = 0;
    d.tkey = nullptr;
    d.thi = nullptr;
    d.tlo = nullptr;
    return d;
}
template <typename TL>
__device__ inline DepF64 make_dep(const ProbDev<double> &p, const Local<TL> &L, const SweepOrder &o)
{
    DepF64 d;
    d.out = p.out;
    const size_t s1 = (size_t)p.g.dims[0], s2 = (size_t)p.g.dims[0] * (size_t)p.g.dims[1];
    for (int k = 0; k < 3; ++k) {
        d.dims[k] = sel3(p.g.dims[0], p.g.dims[1], p.g.dims[2], o.ax[k]);
        d.periodic[k] = sel3(p.g.periodic[0], p.g.periodic[1], p.g.periodic[2], o.ax[k]);
        d.anchor[k] = d.periodic[k] ? wrap_index(L.anchor[k], d.dims[k]) : L.anchor[k];
        d.stride[k] = sel3((size_t)1, s1, s2, o.ax[k]);
    }
    d.scale = p.g.out_scale;
    d.suppress_ix = -1;
    d.suppress_iy = 0;
    d.suppress_iz = 0;
    d.count = 0;
    return d;
}

// Expected number of pieces of a simplex with this local geometry: the
// volume of its Minkowski sum with a unit cell (volume + projected areas +
// widths + 1 in 3D; area + widths + 1 in 2D), a cost proxy for binning.
template <typename T, int D>
__device__ inline float piece_estimate(const Local<T> &L)
{
    float w[3];
    for (int d = 0; d < 3; ++d) {
        float mn = 1e30f, mx = -1e30f;
        for (int a = 0; a <= D; ++a) {
            float c = (float)(d == 0 ? L.v[a].x : (d == 1 ? L.v[a].y : L.v[a].z));
            mn = fminf(mn, c);
            mx = fmaxf(mx, c);
        }
        w[d] = mx - mn;
    }
    if (D == 2) return (float)L.det * 0.5f + w[0] + w[1] + 1.0f;
    float area[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < 4; ++k) {
        int i0 = (k + 1) & 3, i1 = (k + 2) & 3, i2 = (k + 3) & 3;
        float ax = (float)(L.v[i1].x - L.v[i0].x), ay = (float)(L.v[i1].y - L.v[i0].y), az = (float)(L.v[i1].z - L.v[i0].z);
        float bx = (float)(L.v[i2].x - L.v[i0].x), by = (float)(L.v[i2].y - L.v[i0].y), bz = (float)(L.v[i2].z - L.v[i0].z);
        area[0] += fabsf(ay * bz - az * by);
        area[1] += fabsf(az * bx - ax * bz);
        area[2] += fabsf(ax * by - ay * bx);
    }
    return (float)L.det / 6.0f + 0.25f * (area[0] + area[1] + area[2]) + w[0] + w[1] + w[2] + 1.0f;
}

// ---------------------------------------------------------------------------
// kernels

template <typename T>
__global__ void k_fill(T *p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = T(0);
}

__global__ void k_clear_state(CallState *cs, double *total)
{
    unsigned *w = reinterpret_cast<unsigned *>(cs);
    for (int i = threadIdx.x; i < (int)(sizeof(CallState) / 4); i += blockDim.x) w[i] = 0u;
    if (threadIdx.x == 0 && total) *total = 0.0;
}

// Single-cell simplices of one block are merged per cell before they reach
// the grid: an open-addressing table in LDS (twice as many slots as
// threads, so it never fills) of global cell indices and FP64 partial sums;
// each cell then costs one grid deposit per block instead of one per
// simplex, which matters where many small simplices share a cell.
constexpr int SETUP_TABLE = 512;
constexpr unsigned long long SETUP_EMPTY = ~0ull;

template <int D, typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_setup(ProbDev<T> p0, Batch b)
{
    static_assert(SETUP_TABLE >= 2 * 256, "the merge table needs room for every thread of a block");
    __shared__ unsigned s_hist[NCLS];
    __shared__ unsigned s_extra, s_extra_base;
    __shared__ unsigned long long s_key[SETUP_TABLE];
    __shared__ double s_sum[SETUP_TABLE];
    if (threadIdx.x < NCLS) s_hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) s_extra = 0u;
    for (int e = threadIdx.x; e < SETUP_TABLE; e += blockDim.x) {
        s_key[e] = SETUP_EMPTY;
        s_sum[e] = 0.0;
    }
    __syncthreads();
    ProbDev<T> p = p0;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (BATCH) {
        int64_t s0;
        int pi;
        block_problem(b, p, s0, pi);
        s = s0 + threadIdx.x;
    }
    int nit = 0, sx = 0;  // nit > 0: work items wanted for the clip kernel
    bool wide = false;    // FP32C simplex routed to FP64
    float est_all = 0.0f;
    if (s < p.n) {
        Local<T> L;
        int st = setup_any<D>(p, s, p.validate != 0, L);
        if (st == SETUP_OK) {
            if (L.span[0] == 1 && L.span[1] == 1 && L.span[2] == 1) {
                // the whole simplex lies in one cell: deposit its mass
                T rs = L.v[0].r + L.v[1].r + L.v[2].r + (D == 3 ? L.v[3].r : T(0));
                T val = D == 3 ? L.det * rs / T(24) : L.det * rs / T(6);
                const auto dep = make_dep<T>(p, L, kIdentity);
                size_t idx;
                if (dep.cell(0, 0, 0, idx)) {
                    const unsigned long long key = (unsigned long long)idx;
                    unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 55) & (SETUP_TABLE - 1);
                    for (int probe = 0; probe < SETUP_TABLE; ++probe) {
                        const unsigned long long k = atomicCAS(&s_key[h], SETUP_EMPTY, key);
                        if (k == SETUP_EMPTY || k == key) {
                            atomicAdd(&s_sum[h], (double)val);
                            break;
                        }
                        h = (h + 1) & (SETUP_TABLE - 1);
                    }
                }
                if (p.count_pieces) atomicAdd(&p.cs->pieces, 1ull);
            } else {
                const SweepOrder ord = sweep_order(L);
                wide = sizeof(T) == 4 && max(L.span[0], max(L.span[1], L.span[2])) >= WIDE_SPAN;
                sx = D == 3 ? sel3(L.span[0], L.span[1], L.span[2], ord.ax[0]) : L.span[0];
                if constexpr (D == 3) {
                    if (!wide) {
                        const Local<T> M = permuted(L, ord);
                        SimplexRec<T> r;
                        for (int k = 0; k < 4; ++k) r.v[k] = M.v[k];
                        for (int d = 0; d < 3; ++d) {
                            r.anchor[d] = M.anchor[d];
                            r.span[d] = M.span[d];
                        }
                        r.det = M.det;
                        r.order = pack_order(ord);
                        density_gradient(M.v, r.gd);
                        p.rec[s] = r;
                    }
                }
                if constexpr (sizeof(T) == 4) {
                    if (wide) {
                        // the items of a simplex routed to FP64 count the slabs
                        // of the FP64 set-up, which the clip will repeat
                        Local<double> Lw;
                        if (setup_any<D>(p, s, false, Lw) == SETUP_OK) {
                            const int aw = sweep_order(Lw, true).ax[0];
                            sx = D == 3 ? sel3(Lw.span[0], Lw.span[1], Lw.span[2], aw) : Lw.span[0];
                        } else {
                            sx = 0;  // the FP64 set-up drops it (zero volume, span): no items
                        }
                    }
                }
                // work items of about item_pieces expected pieces and at
                // most slab_group slabs: small simplices stay whole, big
                // ones are spread over many lanes
                est_all = piece_estimate<T, D>(L);
                if (sx > 0) {
                    const float per_slab = est_all / (float)sx;
                    // the few simplices routed to FP64 go one slab per item:
                    // whole, each would hold one lane for its hundreds of
                    // pieces while the rest of the launch waits for it
                    const int G = wide ? 1
                                       : (int)fminf((float)p.slab_group,
                                                    fmaxf(1.0f, floorf(p.item_pieces / per_slab)));
                    nit = (sx + G - 1) / G;
                    if (nit > MAX_ITEMS) nit = MAX_ITEMS;  // 12-bit field of the item count
                }
            }
        } else if (p.validate && st == SETUP_BAD_INDEX) {
            record_error(p.es, SP_E_OUT_OF_RANGE);
            atomicAdd(&p.es->n_bad_index, 1);
        } else if (p.validate && st == SETUP_NONFINITE) {
            record_error(p.es, SP_E_NONFINITE);
            atomicAdd(&p.es->n_nonfinite, 1);
        } else if (p.validate && st == SETUP_BAD_SPAN) {
            record_error(p.es, SP_E_PERIODIC_SPAN);
            atomicAdd(&p.es->n_bad_span, 1);
        }
    }
    // the block's extra items (beyond one per simplex) are reserved with one
    // global atomic; a simplex whose share does not fit stays one item
    unsigned my_extra = 0u;
    if (nit > 1) my_extra = atomicAdd(&s_extra, (unsigned)(nit - 1));
    __syncthreads();
    if (threadIdx.x == 0) s_extra_base = s_extra ? atomicAdd(&p0.cs->extra, s_extra) : 0u;
    __syncthreads();
    if (s < p.n) {
        uint32_t info = 0u;
        if (nit > 0) {
            if (nit > 1 && s_extra_base + my_extra + (unsigned)(nit - 1) > p.extra_cap) nit = 1;
            const float est = est_all / (float)nit;
            int cls = 1;
            while (cls < CLS_WIDE - 1 && (float)(1u << cls) < est) ++cls;
            if (wide) cls = CLS_WIDE;
            info = pack_setup(cls, nit, sx);
            atomicAdd(&s_hist[cls], (unsigned)nit);
        }
        p.tinfo[s] = info;
    }
    __syncthreads();
    if (threadIdx.x < NCLS && s_hist[threadIdx.x]) atomicAdd(&p0.cs->hist[threadIdx.x], s_hist[threadIdx.x]);
    // the merged single-cell deposits (every simplex of a block belongs to
    // one problem, so p's grid is the block's grid; only the grid pointers
    // and scale of the deposit are used here)
    Local<T> origin_cell;
    for (int d = 0; d < 3; ++d) origin_cell.anchor[d] = 0;
    const auto grid = make_dep<T>(p, origin_cell, kIdentity);
    for (int e = threadIdx.x; e < SETUP_TABLE; e += blockDim.x)
        if (s_key[e] != SETUP_EMPTY) grid.add((size_t)s_key[e], s_sum[e]);
}

__global__ void k_scan(CallState *cs)
{
    if (threadIdx.x == 0) {
        unsigned off = 0;
        for (int c = NCLS - 1; c >= 0; --c) {
            cs->cursor[c] = off;
            off += cs->hist[c];
        }
        cs->total = off;
        // the wide class comes first; the FP32 clip kernel starts after it
        cs->head = cs->hist[CLS_WIDE];
    }
}

// Simplices per thread of k_scatter: a single problem takes 8, so that each
// block claims its class ranges with 8x fewer global atomics on the 16
// cursors (their contention set the kernel's time); a batch keeps one, as
// its blocks follow the per-problem block table of k_setup.
template <bool BATCH>
constexpr int scatter_per_thread() { return BATCH ? 1 : 8; }

template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_scatter(ProbDev<T> p0, Batch b)
{
    constexpr int IPT = scatter_per_thread<BATCH>();
    __shared__ unsigned s_cnt[NCLS];
    __shared__ unsigned s_base[NCLS];
    if (threadIdx.x < NCLS) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    ProbDev<T> p = p0;
    int64_t s0 = (int64_t)blockIdx.x * blockDim.x * IPT;
    int pi = 0;
    if constexpr (BATCH) block_problem(b, p, s0, pi);
    uint32_t info[IPT];
    unsigned local[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t s = s0 + (int64_t)j * blockDim.x + threadIdx.x;
        info[j] = s < p.n ? p.tinfo[s] : 0u;
        local[j] = 0u;
        if (info[j]) local[j] = atomicAdd(&s_cnt[setup_class(info[j])], (unsigned)setup_items(info[j]));
    }
    __syncthreads();
    if (threadIdx.x < NCLS && s_cnt[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(&p0.cs->cursor[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (!info[j]) continue;
        const int64_t s = s0 + (int64_t)j * blockDim.x + threadIdx.x;
        const int cls = setup_class(info[j]), nit = setup_items(info[j]), sx = setup_span(info[j]);
        const unsigned pos = s_base[cls] + local[j];
        for (int k = 0; k < nit; ++k) {
            int sb, sc;
            item_range(sx, nit, k, sb, sc);
            p0.items[pos + k] = pack_item((uint32_t)s, sb, sc);
            if (BATCH) p0.item_prob[pos + k] = (uint16_t)pi;
        }
    }
}

// The clip kernel.  Persistent one-wave blocks; each wave takes 64 items at
// a time from the class-ordered list (most expensive first), and every lane
// takes its next item the moment it finishes the previous one, so lanes do
// not wait for the slowest item of a chunk.  The block is a single wave, so
// the queue state is wave-uniform (ballots, no LDS and no barriers) and the
// only LDS is each lane's own polytope.  Per loop iteration a busy lane
// performs one sweep step (a column build if due, then one piece).
//
// Waves per SIMD the compiler must leave room for: 3 (at most 168 VGPRs) for
// the 14-slot FP32 polytopes, whose LDS admits 12 waves per CU; the other
// forms are bound by their LDS to 2 or fewer anyway.
template <int D, typename T, int MAXV>
constexpr int clip_waves_per_simd() { return D == 3 && sizeof(T) == 4 && MAXV <= 17 ? 3 : 1; }

// T is the arithmetic of the clip, TI that of the problem (inputs and
// grids).  TI = float with T = double is the FP64 route of an FP32C problem:
// it takes the CLS_WIDE items at the head of the list (one slab each, swept
// with the simplex's longest axis outermost), and a polytope that outgrows
// its slots there is an internal error (it runs with 32 slots).
//
// TILED (FP32 3D, one problem, the grid's cells numbered below 2^32 - 1, no
// per-cell maximum recorded): pieces go through the wave's deposit tile
// (DepF32::tile_add), 64 cells of 12 bytes after the polytopes (13,312
// bytes a wave, which still lets 12 waves share a CU); each wave flushes
// its tile when its work is done.
template <int D, typename T, int MAXV, bool SINGLE, typename TI = T, bool TILED = false>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(clip_waves_per_simd<D, T, MAXV>()))) void k_clip(
    ProbDev<TI> p0, Batch b, int overflow_pass)
{
    static_assert(WG == 64, "the queue logic assumes one wave per block");
    static_assert(!TILED || (D == 3 && sizeof(T) == 4 && sizeof(TI) == 4 && SINGLE && DEP_TILE == WG),
                  "the deposit tile is for one FP32 3D problem, one entry per lane");
    constexpr bool WIDE = sizeof(T) == 8 && sizeof(TI) == 4;
    const ProbDev<TI> &p = p0;  // fields shared by every problem of the launch
    constexpr int SLOTS = D == 3 ? MAXV : 2 * MAXP2;
    // 3D: polytope positions, then neighbour words (then the deposit tile);
    // 2D: polygon buffers
    constexpr size_t POLY_BYTES = (size_t)MAXV * WG * (sizeof(P3T<T>) + sizeof(typename NbStore<T>::type));
    constexpr size_t LDS_BYTES = D == 3 ? POLY_BYTES + (TILED ? (size_t)DEP_TILE * 12 : 0)
                                        : (size_t)SLOTS * WG * sizeof(V4<T>);
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[LDS_BYTES];
    V4<T>(*s_p)[WG] = reinterpret_cast<V4<T>(*)[WG]>(s_raw);
    const int lane = threadIdx.x;
    const unsigned total = overflow_pass ? min(p.cs->ovf_count, (unsigned)OVF_CAP)
                                         : (WIDE ? p.cs->hist[CLS_WIDE] : p.cs->total);
    unsigned *head = overflow_pass ? &p.cs->ovf_head : (WIDE ? &p.cs->head_wide : &p.cs->head);
    // the few resumed items of the overflow pass are spread over many waves
    const unsigned chunk = overflow_pass ? 8u : (unsigned)WG;
    unsigned q_base = 0u, q_n = 0u, q_h = 0u;  // current chunk [q_base, q_base + q_n), next unclaimed q_h
    bool q_done = false;
    Poly3<T, MAXV, WG> P3;
    if constexpr (D == 3) {
        P3.pp = reinterpret_cast<P3T<T> *>(s_raw) + lane;
        P3.pn = reinterpret_cast<typename NbStore<T>::type *>(s_raw + (size_t)MAXV * WG * sizeof(P3T<T>)) + lane;
    }
    P3.live = 0u;
    uint32_t *t_key = nullptr;
    float *t_hi = nullptr, *t_lo = nullptr;
    if constexpr (TILED) {
        t_key = reinterpret_cast<uint32_t *>(s_raw + POLY_BYTES);
        t_hi = reinterpret_cast<float *>(s_raw + POLY_BYTES + DEP_TILE * 4);
        t_lo = reinterpret_cast<float *>(s_raw + POLY_BYTES + DEP_TILE * 8);
        t_key[lane] = DepF32::TILE_EMPTY;
        t_hi[lane] = 0.0f;
        t_lo[lane] = 0.0f;
        __builtin_amdgcn_wave_barrier();
    }
    Poly2<T, MAXP2, WG> P2;
    P2.a = &s_p[0][lane];
    P2.b = &s_p[D == 3 ? 0 : MAXP2][lane];
    P2.n = 0;
    bool busy = false;
    Local<T> L;
    typename DepFor<TI>::type dep;
    Sweep3 S;
    int64_t sid = 0;
    int sb = 0, sc = 0, pid = 0;
    for (;;) {
        const uint64_t idle = __ballot(!busy);
        if (idle != 0ull && q_h >= q_n && !q_done) {
            unsigned base = 0u;
            if (lane == 0) base = atomicAdd(head, chunk);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= total) {
                q_done = true;
            } else {
                q_base = base;
                q_n = min(chunk, total - base);
                q_h = 0u;
            }
        }
        if (!busy && q_h < q_n) {
            // idle lanes take consecutive entries in lane order
            const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(idle >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
            const unsigned k = q_h + rank;
            if (k < q_n) {
                const unsigned it = q_base + k;
                int ry = 0, rz = 0;
                if (overflow_pass) {
                    Ovf o = p.ovf[it];
                    sid = o.s;
                    sb = o.ix;
                    sc = o.end - o.ix;
                    ry = o.iy;
                    rz = o.iz;
                    pid = o.pid;
                } else {
                    uint64_t item = p.items[it];
                    sid = (int64_t)item_simplex(item);
                    sb = item_first(item);
                    sc = item_count(item);
                    pid = !SINGLE && b.nprob ? (int)p.item_prob[it] : 0;
                }
                const ProbDev<TI> q = !SINGLE && b.nprob ? static_cast<const ProbDev<TI> *>(b.probs)[pid] : p0;
                bool ok;
                SweepOrder ord = kIdentity;
                if constexpr (D == 3 && !WIDE) {
                    // the set-up k_setup left for this simplex
                    const SimplexRec<T> r = q.rec[sid];
                    for (int k = 0; k < 4; ++k) L.v[k] = r.v[k];
                    for (int d = 0; d < 3; ++d) {
                        L.anchor[d] = r.anchor[d];
                        L.span[d] = r.span[d];
                    }
                    L.det = r.det;
                    ord = unpack_order(r.order);
                    P3.set_density(L.v, r.gd);
                    ok = true;
                } else {
                    Local<T> L0;
                    ok = setup_any<D>(q, sid, false, L0) == SETUP_OK;
                    if (ok && D == 3) {
                        ord = sweep_order(L0, WIDE);
                        L = permuted(L0, ord);
                        P3.set_density(L.v);
                    } else if (ok) {
                        L = L0;
                    }
                }
                if (ok) {
                    dep = make_dep<T>(q, L, ord);
                    if constexpr (TILED) {
                        dep.tkey = t_key;
                        dep.thi = t_hi;
                        dep.tlo = t_lo;
                    }
                    if (overflow_pass) {
                        dep.suppress_ix = sb;
                        dep.suppress_iy = ry;
                        dep.suppress_iz = rz;
                    }
                    S.start(sb, sc, ry);
                    busy = true;
                }
            }
        }
        if (q_h < q_n) q_h = min(q_n, q_h + (unsigned)__popcll(idle));
        if (__ballot(busy) == 0ull) {
            if (q_done) break;
            continue;
        }
        if (!busy) continue;
        if constexpr (D == 3) {
            // A column build (a tetrahedron and up to four cuts) costs the
            // wave the same whether one lane or all of them need it, so a
            // lane whose column is done waits while other lanes still have
            // pieces, until BUILD_MIN lanes build together.
            const bool nb = S.needs_build();
            const uint64_t bn = __ballot(nb), br = __ballot(!nb);
            if (nb && br != 0ull && __popcll(bn) < BUILD_MIN) continue;
        }
        int r;
        if constexpr (D == 3) {
            r = S.step(P3, L, dep);
        } else {
            int fail2[3];
            r = sweep2(P2, L, sb, sc, dep, fail2) ? 0 : -1;
            S.fail[0] = fail2[0];
            S.fail[1] = fail2[1];
            S.fail[2] = fail2[2];
        }
        if (r > 0) continue;
        busy = false;
        if (p.count_pieces && dep.count) atomicAdd(&p.cs->pieces, (unsigned long long)dep.count);  // counting runs only
        if (r < 0) {
            if (!overflow_pass && !WIDE) {
                unsigned k = atomicAdd(&p.cs->ovf_count, 1u);
                if (k < OVF_CAP) {
                    Ovf o;
                    o.s = (int)sid;
                    o.ix = S.fail[0];
                    o.iy = S.fail[1];
                    o.iz = S.fail[2];
                    o.end = sb + sc;
                    o.pid = pid;
                    p.ovf[k] = o;
                    atomicAdd(&p.es->n_overflow, 1);
                } else {
                    record_error(p.es, SP_E_INTERNAL);
                    atomicAdd(&p.es->n_internal, 1);
                }
            } else {
                record_error(p.es, SP_E_INTERNAL);
                atomicAdd(&p.es->n_internal, 1);
            }
        }
    }
    if constexpr (TILED) {
        // the wave's work is done: each lane flushes one tile entry
        __builtin_amdgcn_wave_barrier();
        const uint32_t k = t_key[lane];
        if (k != DepF32::TILE_EMPTY) DepF32::flush(p0.out, p0.lo, (size_t)k, t_hi[lane], t_lo[lane]);
    }
}

// The FP32 3D clip kernel with one polytope per group of 16 lanes
// (sp_wave.h): persistent one-wave blocks of four groups; the wave claims
// chunks of items from the class-ordered list, and every group takes the
// next item of the chunk as soon as its sweep ends, so a group never waits
// for the others' items.  Per loop iteration every busy group performs one
// step of its sweep (one split, at most one piece).  An item that outgrows
// the 16 slots is handed, from its first undeposited piece, to the overflow
// pass of the one-polytope-per-lane kernel.
struct GroupDep {
    DepF32 d;
    __device__ void operator()(int ix, int iy, int iz, float v)
    {
        if ((threadIdx.x & (wv::G - 1)) == 0) d(ix, iy, iz, v);
    }
};

template <bool SINGLE>
__global__ __launch_bounds__(WG) void k_clipw(ProbDev<float> p0, Batch b)
{
    static_assert(WG == 4 * wv::G, "four groups per wave");
    const ProbDev<float> &p = p0;  // fields shared by every problem of the launch
    __shared__ wv::GroupLDS s_g[4];
    const int grp = (int)(threadIdx.x >> 4);
    wv::GroupLDS *sh = &s_g[grp];
    const unsigned total = p.cs->total;
    unsigned *head = &p.cs->head;
    constexpr unsigned chunk = 16u;
    unsigned q_base = 0u, q_n = 0u, q_h = 0u;  // wave-uniform chunk state
    bool q_done = false;
    bool busy = false;                         // group-uniform
    wv::Sweep S;
    S.phase = wv::PH_IDLE;
    GroupDep dep;
    int64_t sid = 0;
    int send = 0, pid = 0;
    for (;;) {
        const uint64_t bb = __ballot(busy);
        // one bit per group (its lanes agree)
        const unsigned idle = (~(unsigned)((bb & 1ull) | ((bb >> 15) & 2ull) | ((bb >> 30) & 4ull) | ((bb >> 45) & 8ull))) & 15u;
        if (idle != 0u && q_h >= q_n && !q_done) {
            unsigned base = 0u;
            if (threadIdx.x == 0) base = atomicAdd(head, chunk);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= total) {
                q_done = true;
            } else {
                q_base = base;
                q_n = min(chunk, total - base);
                q_h = 0u;
            }
        }
        if (!busy && q_h < q_n) {
            // idle groups take consecutive entries in group order
            const unsigned k = q_h + (unsigned)__builtin_popcount(idle & ((1u << grp) - 1u));
            if (k < q_n) {
                const unsigned it = q_base + k;
                const uint64_t item = p.items[it];
                sid = (int64_t)item_simplex(item);
                const int sb = item_first(item);
                const int sc = item_count(item);
                send = sb + sc;
                pid = !SINGLE && b.nprob ? (int)p.item_prob[it] : 0;
                const ProbDev<float> q = !SINGLE && b.nprob ? static_cast<const ProbDev<float> *>(b.probs)[pid] : p0;
                Local<float> L0;
                double ex0[4][3];
                if (setup_f32<3>(q.xyz, q.n_vert, q.simp, sid, q.rho, q.per_corner != 0, q.g, false, L0, ex0) ==
                    SETUP_OK) {
                    const SweepOrder ord = sweep_order(L0);
                    const Local<float> L = permuted(L0, ord);
                    double ex[4][3];
                    permuted_exact(ex0, ord, ex);
                    dep.d = make_dep<float>(q, L, ord);
                    wv::sweep_start(sh, S, L, ex, sb, sc);
                    busy = true;
                }
            }
        }
        if (q_h < q_n) q_h = min(q_n, q_h + (unsigned)__builtin_popcount(idle));
        if (__ballot(busy) == 0ull) {
            if (q_done) break;
            continue;
        }
        if (!busy) continue;
        if (!wv::sweep_step(sh, S, dep)) {
            // out of slots: the rest goes to the overflow pass
            if ((threadIdx.x & (wv::G - 1)) == 0) {
                const unsigned k = atomicAdd(&p.cs->ovf_count, 1u);
                if (k < OVF_CAP) {
                    Ovf o;
                    o.s = (int)sid;
                    o.ix = S.fail[0];
                    o.iy = S.fail[1];
                    o.iz = S.fail[2];
                    o.end = send;
                    o.pid = pid;
                    p.ovf[k] = o;
                    atomicAdd(&p.es->n_overflow, 1);
                } else {
                    record_error(p.es, SP_E_INTERNAL);
                    atomicAdd(&p.es->n_internal, 1);
                }
            }
            S.phase = wv::PH_IDLE;
        }
        if (S.phase == wv::PH_IDLE) {
            busy = false;
            if (p.count_pieces && dep.d.count && (threadIdx.x & (wv::G - 1)) == 0)
                atomicAdd(&p.cs->pieces, (unsigned long long)dep.d.count);  // counting runs only
            dep.d.count = 0;
        }
    }
}

// Projection by first-order corner sums (Section 3.1, Appendix D), FP64:
// one thread per simplex enumerates the vertices of all its cell pieces
// (simplex corners, edge-face and facet-edge crossings, grid points inside)
// and adds each vertex's terms to its cell(s).  Grid-stride over simplices.
// The kernel waits on memory far more than it computes; held to 2 waves
// per SIMD (128 VGPRs, the rest spilled) it ran 1.7x faster than at 1 wave
// with 256 VGPRs, and 3 or 4 waves ran slower again.  One-wave blocks
// measured 7 % faster than 256-thread ones.
// Fused facet contributions of the corner sums (App. D, eq.
// eq_contribFused): the facets of the summed simplices are matched by their
// vertex ids in an open-addressing table (linear probing, insert or find),
// so that each facet shared by two of them knows the other.  Facet ids are
// s * 4 + k, k the input corner opposite the facet; tables hold id + 1, 0
// meaning empty (hence fewer than 2^30 simplices).
struct FuseDev {
    uint32_t *tab;   // mask + 1 entries
    uint32_t mask;
    uint32_t *mate;  // [4n] the facet id + 1 across each facet, 0 if none
    int8_t *side;    // [4n] facet_side of each facet, 0 if its simplex is not summed
    double *grad;    // [3n] density gradient of each summed simplex
};

// input corner of local corner a (set-up exchanges corners 1 and 2 of a
// negatively oriented simplex)
__device__ inline int corner_input(int a, bool swapped) { return swapped && (a == 1 || a == 2) ? 3 - a : a; }

// sorted vertex ids of the facet opposite input corner k of simplex s
__device__ inline void facet_key(const int32_t *simp, int64_t s, int k, int32_t key[3])
{
    int n = 0;
    for (int a = 0; a < 4; ++a)
        if (a != k) key[n++] = simp[s * 4 + a];
    if (key[1] < key[0]) { const int32_t t = key[0]; key[0] = key[1]; key[1] = t; }
    if (key[2] < key[1]) { const int32_t t = key[1]; key[1] = key[2]; key[2] = t; }
    if (key[1] < key[0]) { const int32_t t = key[0]; key[0] = key[1]; key[1] = t; }
}

__device__ inline uint32_t facet_hash(const int32_t key[3])
{
    uint64_t h = (uint64_t)(uint32_t)key[0] * 0x9E3779B97F4A7C15ull;
    h = (h ^ (h >> 29)) + (uint64_t)(uint32_t)key[1] * 0xC2B2AE3D27D4EB4Full;
    h = (h ^ (h >> 31)) + (uint64_t)(uint32_t)key[2] * 0x165667B19E3779F9ull;
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    return (uint32_t)h;
}

// Insert facet fid, or pair it with the facet of the same vertices already
// there (a third facet on the same vertices stays unpaired).
__device__ inline void facet_insert(const FuseDev &f, const int32_t *simp, uint32_t fid)
{
    int32_t key[3];
    facet_key(simp, fid >> 2, (int)(fid & 3u), key);
    uint32_t h = facet_hash(key) & f.mask;
    for (uint32_t probe = 0; probe <= f.mask; ++probe, h = (h + 1u) & f.mask) {
        const uint32_t cur = atomicCAS(&f.tab[h], 0u, fid + 1u);
        if (cur == 0u) return;
        int32_t kc[3];
        facet_key(simp, (cur - 1u) >> 2, (int)((cur - 1u) & 3u), kc);
        if (kc[0] == key[0] && kc[1] == key[1] && kc[2] == key[2]) {
            if (atomicCAS(&f.mate[cur - 1u], 0u, fid + 1u) == 0u) f.mate[fid] = cur;
            return;
        }
    }
}

// Per simplex: whether the corner sums will sum it with fused terms, its
// density gradient, the side of each facet, and its facets into the table.
__global__ __launch_bounds__(256) void k_corner_prep(ProbDev<double> p, FuseDev f)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    Local<double> L;
    bool sw = false;
    int sd[4] = {0, 0, 0, 0};
    if (setup_f64<3>(p.xyz, p.n_vert, p.simp, s, p.rho, p.per_corner != 0, p.g, false, L, &sw) == SETUP_OK &&
        corner_box_ok(L)) {
        int64_t vid[4];
        for (int a = 0; a < 4; ++a) vid[a] = p.simp[s * 4 + corner_input(a, sw)];
        const D3 g = corner_gradient(L);
        f.grad[s * 3 + 0] = g.x;
        f.grad[s * 3 + 1] = g.y;
        f.grad[s * 3 + 2] = g.z;
        if (corner_fusable(L, g))
            for (int m = 0; m < 4; ++m) sd[corner_input(m, sw)] = facet_side(L, vid, m);
    }
    for (int k = 0; k < 4; ++k) f.side[s * 4 + k] = (int8_t)sd[k];
    for (int k = 0; k < 4; ++k)
        if (sd[k] != 0) facet_insert(f, p.simp, (uint32_t)(s * 4 + k));
}

// The fused-term data of simplex s (local corners L, corners 1 and 2
// exchanged at set-up if swapped): for each facet, plain, left to the
// neighbour of lower index, or summed here with the neighbour's density.
__device__ inline void corner_fuse(const ProbDev<double> &p, const FuseDev &f, int64_t s, const Local<double> &L,
                                   bool sw, FacetFuse &fz)
{
    fz.cell_origin = false;
    const D3 g = d3(f.grad[s * 3 + 0], f.grad[s * 3 + 1], f.grad[s * 3 + 2]);
    for (int m = 0; m < 4; ++m) {
        fz.mode[m] = FACET_PLAIN;
        const int k = corner_input(m, sw);
        const uint32_t mt = f.mate[s * 4 + k];
        if (mt == 0u) continue;
        fz.cell_origin = true;
        const uint32_t fid = mt - 1u;
        const int64_t j = (int64_t)(fid >> 2);
        if (j < s) {
            fz.mode[m] = FACET_SKIP;
            continue;
        }
        const int a = m == 0 ? 1 : 0;  // a corner of the facet
        const int32_t va = p.simp[s * 4 + corner_input(a, sw)];
        double rj = L.v[a].r;  // per-vertex densities agree on shared corners
        if (p.per_corner)
            for (int kk = 0; kk < 4; ++kk)
                if (p.simp[j * 4 + kk] == va) rj = p.rho[j * 4 + kk];
        const D3 gj = d3(f.grad[j * 3 + 0], f.grad[j * 3 + 1], f.grad[j * 3 + 2]);
        fuse_facet(fz, m, L, g, a, gj, rj, (int)f.side[s * 4 + k] * (int)f.side[fid]);
    }
}

template <bool FUSED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_corner(ProbDev<double> p, FuseDev f)
{
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < p.n; s += st) {
        Local<double> L;
        bool sw = false;
        const int r = setup_f64<3>(p.xyz, p.n_vert, p.simp, s, p.rho, p.per_corner != 0, p.g, p.validate != 0, L, &sw);
        if (r == SETUP_OK) {
            auto dep = make_dep<double>(p, L, kIdentity);
            FacetFuse fz;
            if constexpr (FUSED) corner_fuse(p, f, s, L, sw, fz);
            const int big = corner_project(L, dep, FUSED ? &fz : nullptr);
            // counting runs only: grid deposits (one per vertex and cell with terms)
            if (p.count_pieces && dep.count) atomicAdd(&p.cs->pieces, (unsigned long long)dep.count);
            if (big > 0) {
                record_error(p.es, SP_E_UNSUPPORTED);
                atomicAdd(&p.es->n_degenerate, 1);
            }
        } else if (p.validate && r == SETUP_BAD_INDEX) {
            record_error(p.es, SP_E_OUT_OF_RANGE);
            atomicAdd(&p.es->n_bad_index, 1);
        } else if (p.validate && r == SETUP_NONFINITE) {
            record_error(p.es, SP_E_NONFINITE);
            atomicAdd(&p.es->n_nonfinite, 1);
        } else if (p.validate && r == SETUP_BAD_SPAN) {
            record_error(p.es, SP_E_PERIODIC_SPAN);
            atomicAdd(&p.es->n_bad_span, 1);
        }
    }
}

// Per-vertex density estimate (Section 4, "Calculation of the acceleration"):
// rho_j = (sum of the masses of the simplices incident to j) / (sum of their
// unsigned volumes).  One thread per simplex adds its mass and volume to its
// D+1 vertices (FP64 atomics, both precisions); a second pass divides.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_vd_accum(const T *xyz, int64_t n_vert, const int32_t *simp, int64_t n,
                                                  const T *mass, double m0, double3 ext, int3 per, double *acc,
                                                  ErrState *es)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t vi[D + 1];
    double x[D + 1][3];
    for (int a = 0; a <= D; ++a) {
        vi[a] = simp[s * (D + 1) + a];
        if (vi[a] < 0 || vi[a] >= n_vert) {
            record_error(es, SP_E_OUT_OF_RANGE);
            atomicAdd(&es->n_bad_index, 1);
            return;
        }
        for (int d = 0; d < D; ++d) x[a][d] = (double)xyz[(int64_t)vi[a] * D + d];
    }
    const double m = mass ? (double)mass[s] : m0;
    bool finite = isfinite(m);
    const double L[3] = {ext.x, ext.y, ext.z};
    const int P[3] = {per.x, per.y, per.z};
    double e[D][3];
    for (int a = 1; a <= D; ++a) {
        for (int d = 0; d < D; ++d) {
            double dx = x[a][d] - x[0][d];
            if (P[d]) dx -= L[d] * rint(dx / L[d]);  // minimum image
            e[a - 1][d] = dx;
            finite = finite && isfinite(dx);
        }
    }
    if (!finite) {
        record_error(es, SP_E_NONFINITE);
        atomicAdd(&es->n_nonfinite, 1);
        return;
    }
    double vol;
    if (D == 3) {
        vol = fabs(e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                   e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0])) /
              6.0;
    } else {
        vol = fabs(e[0][0] * e[1][1] - e[0][1] * e[1][0]) / 2.0;
    }
    for (int a = 0; a <= D; ++a) {
        unsafeAtomicAdd(acc + 2 * (int64_t)vi[a], m);
        unsafeAtomicAdd(acc + 2 * (int64_t)vi[a] + 1, vol);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_vd_finish(const double *acc, int64_t n_vert, T *rho)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_vert) return;
    const double num = acc[2 * j], den = acc[2 * j + 1];
    rho[j] = den > 0.0 ? (T)(num / den) : T(0);
}

// Per-voxel accuracy control (Section 3.4, eq. eq_accuracy and
// eq_accuracy2): a cell whose sum P has a binary exponent below
// e_max - S + W + A (e_max: the largest contribution's exponent; S the
// significand bits of the arithmetic, W the bits a contribution may have
// wrong, A the bits wanted) is flagged, the simplices touching flagged cells
// are re-projected at higher precision, and their values replace the
// flagged cells'.  Here the test is |P| < max|C| * 2^(W + A - S), S = 23.
__global__ __launch_bounds__(256) void k_flag(const float *hi, const float *lo, const uint32_t *cmax, size_t ncell,
                                              float factor, uint8_t *flags, unsigned long long *nflag)
{
    unsigned long long nf = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
        const float cm = __uint_as_float(cmax[i]);
        const double P = (double)hi[i] + (double)lo[i];
        const bool f = cm > 0.0f && fabs(P) < (double)cm * (double)factor;
        flags[i] = f ? 1 : 0;
        nf += f ? 1ull : 0ull;
    }
    if (nf) atomicAdd(nflag, nf);
}

// Simplices whose bounding box holds a flagged cell (boxes of more than
// 4096 cells are taken without looking).
__global__ __launch_bounds__(256) void k_tag(ProbDev<float> p, const uint8_t *flags, int32_t *list,
                                             unsigned long long *ntag)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    Local<float> L;
    if (setup_any<3>(p, s, false, L) != SETUP_OK) return;
    const int sx = L.span[0], sy = L.span[1], sz = L.span[2];
    bool hit = (int64_t)sx * sy * sz > 4096;
    for (int k = 0; k < sz && !hit; ++k) {
        int cz = L.anchor[2] + k;
        if (p.g.periodic[2]) cz = wrap_index(cz, p.g.dims[2]);
        else if (cz < 0 || cz >= p.g.dims[2]) continue;
        for (int j = 0; j < sy && !hit; ++j) {
            int cy = L.anchor[1] + j;
            if (p.g.periodic[1]) cy = wrap_index(cy, p.g.dims[1]);
            else if (cy < 0 || cy >= p.g.dims[1]) continue;
            for (int i = 0; i < sx && !hit; ++i) {
                int cx = L.anchor[0] + i;
                if (p.g.periodic[0]) cx = wrap_index(cx, p.g.dims[0]);
                else if (cx < 0 || cx >= p.g.dims[0]) continue;
                const size_t idx = ((size_t)cz * p.g.dims[1] + cy) * p.g.dims[0] + cx;
                hit = flags[idx] != 0;
            }
        }
    }
    if (hit) list[atomicAdd(ntag, 1ull)] = (int32_t)s;
}

// The tagged simplices as an FP64 problem: all vertices widened to double,
// the tagged simplices' connectivity and per-corner densities compacted.
__global__ __launch_bounds__(256) void k_widen(const float *x, size_t n, double *y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

__global__ __launch_bounds__(256) void k_gather_tagged(ProbDev<float> p, const int32_t *list, int64_t ntag,
                                                       int32_t *simp, double *rho)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntag) return;
    const int64_t s = list[t];
    for (int a = 0; a < 4; ++a) {
        const int32_t v = p.simp[s * 4 + a];
        simp[t * 4 + a] = v;
        rho[t * 4 + a] = (double)(p.per_corner ? p.rho[s * 4 + a] : p.rho[v]);
    }
}

// Flagged cells take the FP64 value, split into hi + lo.
__global__ __launch_bounds__(256) void k_patch(float *hi, float *lo, const uint8_t *flags, const double *val,
                                               size_t ncell)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
        if (!flags[i]) continue;
        const double v = val[i];
        const float h = (float)v;
        hi[i] = h;
        lo[i] = (float)(v - (double)h);
    }
}

// Adaptive-grid projection (Section 4, "Calculation of the acceleration"):
// an octree over the grid is refined region by region while its cells are
// larger than the smallest height of any simplex intersecting them (or down
// to the grid's own cells), the density is projected exactly onto it, and
// each leaf's mass is spread evenly over the grid cells it holds (donor
// cell).  Kernels, in order:
//   k_amr_level    the level l_i = floor(log2 h_i) of every tetrahedron
//                  (clamped to [0, max_level]; h_i its smallest height,
//                  3 V / largest face area, in cells, FP64)
//   k_amr_mark     every block of side 2^(l_i + 1) a tetrahedron intersects
//                  is marked (separating axis test in FP64)
//   k_amr_refine   a block is refined if it or a block inside it is marked
//   k_amr_plevel   the level each tetrahedron is projected at: the largest
//                  level <= l_i at which no block of its bounding box is
//                  refined, so that every leaf it meets is a union of its
//                  cells there
//   (compaction by level, one batched exact projection, in mass units)
//   k_amr_restrict the leaf sums, level by level: a block's mass is its own
//                  level's projection plus the sums of its 8 children
//   k_amr_gather   each grid cell takes its leaf's mass / 8^level

// Unwrapped corner positions in cells of the grid, FP64: on periodic axes the
// minimum image of the first corner, then (x - origin) * scale.
template <typename T>
__device__ inline bool amr_corners(const ProbDev<T> &p, int64_t s, double P[4][3])
{
    int32_t vi[4];
    for (int a = 0; a < 4; ++a) {
        vi[a] = p.simp[s * 4 + a];
        if (vi[a] < 0 || vi[a] >= p.n_vert) return false;
    }
    for (int d = 0; d < 3; ++d) {
        const double x0 = (double)p.xyz[(int64_t)vi[0] * 3 + d];
        for (int a = 0; a < 4; ++a) {
            double x = (double)p.xyz[(int64_t)vi[a] * 3 + d];
            if (!isfinite(x)) return false;
            if (p.g.periodic[d]) x = x - p.g.extent[d] * rint((x - x0) / p.g.extent[d]);
            P[a][d] = (x - p.g.origin[d]) * p.g.scale[d];
        }
    }
    return true;
}

// Interiors of the tetrahedron P and the box lo + [0, size]^3 intersect:
// separating axis test over the 3 axes, the 4 face normals (corners
// {1,2,3}, {0,2,3}, {0,1,3}, {0,1,2}: (c1 - c0) x (c2 - c0)) and the 18
// products of the 6 edges (c1 - c0 for {0,1}, {0,2}, {0,3}, {1,2}, {1,3},
// {2,3}) with the axes, strict on every non-zero axis.  Evaluated without
// fused multiply-adds, each normal and projection in the order written (the
// same FP64 steps decide the same way on any implementation that takes
// them); the normals are formed as they are tested, which keeps the kernel
// in few registers.
__device__ inline bool amr_meets(const double P[4][3], const double lo[3], double size)
{
#pragma clang fp contract(off)
    double rel[4][3];
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) rel[a][d] = P[a][d] - lo[d];
    // separated along (nx, ny, nz)?
    auto sep = [&](double nx, double ny, double nz) {
        if (nx == 0.0 && ny == 0.0 && nz == 0.0) return false;
        double tmin = 0.0, tmax = 0.0;
        for (int a = 0; a < 4; ++a) {
            const double t = (nx * rel[a][0] + ny * rel[a][1]) + nz * rel[a][2];
            tmin = a == 0 || t < tmin ? t : tmin;
            tmax = a == 0 || t > tmax ? t : tmax;
        }
        const double sx = nx * size, sy = ny * size, sz = nz * size;
        const double bmin = (fmin(0.0, sx) + fmin(0.0, sy)) + fmin(0.0, sz);
        const double bmax = (fmax(0.0, sx) + fmax(0.0, sy)) + fmax(0.0, sz);
        return !(tmin < bmax && bmin < tmax);
    };
    if (sep(1.0, 0.0, 0.0) || sep(0.0, 1.0, 0.0) || sep(0.0, 0.0, 1.0)) return false;
    const int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = P[F[f][1]][d] - P[F[f][0]][d];
            e2[d] = P[F[f][2]][d] - P[F[f][0]][d];
        }
        if (sep(e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]))
            return false;
    }
    const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll 1
    for (int k = 0; k < 6; ++k) {
        double e[3];
        for (int d = 0; d < 3; ++d) e[d] = P[E[k][1]][d] - P[E[k][0]][d];
        if (sep(0.0, e[2], -e[1]) || sep(-e[2], 0.0, e[0]) || sep(e[1], -e[0], 0.0)) return false;
    }
    return true;
}

// A corner of P lies inside the box lo + [0, size]^3 by a margin of
// size / 2^20 on every axis: no axis then separates them, whatever the
// rounding of the test above, so the test can be skipped.
__device__ inline bool amr_corner_inside(const double P[4][3], const double lo[3], double size)
{
    const double m = size * 0x1p-20;
    for (int a = 0; a < 4; ++a) {
        bool in = true;
        for (int d = 0; d < 3; ++d) in = in && P[a][d] > lo[d] + m && P[a][d] < lo[d] + size - m;
        if (in) return true;
    }
    return false;
}

// One slot per lane in counter ctr[key], claimed with one atomic per key
// present in the wave (the lanes of a key take consecutive slots).  Every
// active lane of the wave must call it.
__device__ inline unsigned wave_claim(unsigned *ctr, int key)
{
    const int lane = (int)__lane_id();
    uint64_t todo = __ballot(1);
    unsigned slot = 0u;
    while (todo) {
        const int first = __builtin_ctzll(todo);
        const int k = __shfl(key, first);
        const uint64_t m = __ballot(key == k) & todo;
        unsigned base = 0u;
        if (lane == first) base = atomicAdd(&ctr[k], (unsigned)__popcll(m));
        base = __shfl(base, first);
        if ((m >> lane) & 1ull) slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
        todo &= ~m;
    }
    return slot;
}

// Blocks of side 2^l of a grid with dims: their counts per axis and the
// offset of level l's byte grid in a buffer holding levels 1..max_level.
struct AmrLevels {
    int nb[11][3];
    size_t off[11];
};

template <typename T>
__global__ __launch_bounds__(256) void k_amr_level(ProbDev<T> p, int max_level, uint8_t *level)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    int lv = 0;
    int32_t vi[4];
    bool ok = true;
    for (int a = 0; a < 4; ++a) {
        vi[a] = p.simp[s * 4 + a];
        ok = ok && vi[a] >= 0 && vi[a] < p.n_vert;
    }
    if (ok) {
        double e[3][3];
        for (int a = 1; a < 4; ++a) {
            for (int d = 0; d < 3; ++d) {
                double dx = (double)p.xyz[(int64_t)vi[a] * 3 + d] - (double)p.xyz[(int64_t)vi[0] * 3 + d];
                if (p.g.periodic[d]) dx -= p.g.extent[d] * rint(dx / p.g.extent[d]);
                e[a - 1][d] = dx * p.g.scale[d];
            }
        }
        auto cross = [](const double *x, const double *y, double *z) {
            z[0] = x[1] * y[2] - x[2] * y[1];
            z[1] = x[2] * y[0] - x[0] * y[2];
            z[2] = x[0] * y[1] - x[1] * y[0];
        };
        auto norm = [](const double *z) { return sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]); };
        double c01[3], c02[3], c12[3], f[3], g[3], c3[3];
        cross(e[0], e[1], c01);
        cross(e[0], e[2], c02);
        cross(e[1], e[2], c12);
        for (int d = 0; d < 3; ++d) {
            f[d] = e[1][d] - e[0][d];
            g[d] = e[2][d] - e[0][d];
        }
        cross(f, g, c3);
        const double V = fabs(e[0][0] * c12[0] + e[0][1] * c12[1] + e[0][2] * c12[2]) / 6.0;
        const double amax = fmax(fmax(norm(c01), norm(c02)), fmax(norm(c12), norm(c3))) / 2.0;
        const double h = amax > 0.0 ? 3.0 * V / amax : 0.0;
        if (h >= 1.0 && isfinite(h)) {
            lv = (int)floor(log2(h));
            lv = lv > max_level ? max_level : lv;
        }
    }
    level[s] = (uint8_t)lv;
}

// Blocks of side 2^(l_i + 1) the tetrahedron intersects are marked (byte
// stores of 1; concurrent ones agree).  Tetrahedra at max_level mark nothing.
template <typename T>
__global__ __launch_bounds__(64) void k_amr_mark(ProbDev<T> p, int max_level, const uint8_t *level, uint8_t *marks,
                                                 AmrLevels L)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    const int l = (int)level[s] + 1;
    if (l > max_level) return;
    double P[4][3];
    if (!amr_corners(p, s, P)) return;
    const double size = (double)(1 << l);
    int blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
        double mn = P[0][d], mx = P[0][d];
        for (int a = 1; a < 4; ++a) {
            mn = fmin(mn, P[a][d]);
            mx = fmax(mx, P[a][d]);
        }
        blo[d] = (int)floor(mn / size);
        bhi[d] = (int)floor(mx / size);
    }
    const int *nb = L.nb[l];
    uint8_t *m = marks + L.off[l];
    // a bounding box of more than 2^22 blocks is marked whole without the
    // test (a finer grid there than the rule asks for; it keeps one thread's
    // loop bounded)
    const bool all = (double)(bhi[0] - blo[0] + 1) * (bhi[1] - blo[1] + 1) * (bhi[2] - blo[2] + 1) > 4194304.0;
    for (int bz = blo[2]; bz <= bhi[2]; ++bz) {
        int wz = bz;
        if (p.g.periodic[2]) wz = wrap_index(bz, nb[2]);
        else if (bz < 0 || bz >= nb[2]) continue;
        for (int by = blo[1]; by <= bhi[1]; ++by) {
            int wy = by;
            if (p.g.periodic[1]) wy = wrap_index(by, nb[1]);
            else if (by < 0 || by >= nb[1]) continue;
            for (int bx = blo[0]; bx <= bhi[0]; ++bx) {
                int wx = bx;
                if (p.g.periodic[0]) wx = wrap_index(bx, nb[0]);
                else if (bx < 0 || bx >= nb[0]) continue;
                uint8_t *mk = m + ((size_t)wz * nb[1] + wy) * nb[0] + wx;
                if (*mk) continue;  // marked already (by another simplex)
                const double lo[3] = {bx * size, by * size, bz * size};
                if (all || amr_corner_inside(P, lo, size) || amr_meets(P, lo, size)) *mk = 1;
            }
        }
    }
}

// Level l's marks become "refined": marked, or a child (level l - 1) refined.
__global__ __launch_bounds__(256) void k_amr_refine(uint8_t *marks, AmrLevels L, int l)
{
    const int *nb = L.nb[l], *nc = L.nb[l - 1];
    const size_t nblk = (size_t)nb[0] * nb[1] * nb[2];
    uint8_t *m = marks + L.off[l];
    const uint8_t *c = marks + L.off[l - 1];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nblk; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nb[0]), y = (int)((i / nb[0]) % nb[1]), z = (int)(i / ((size_t)nb[0] * nb[1]));
        uint8_t r = m[i];
        for (int k = 0; k < 8 && !r; ++k) {
            const int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
            r = c[((size_t)cz * nc[1] + cy) * nc[0] + cx];
        }
        m[i] = r;
    }
}

// The projection level of each tetrahedron (and the count per level).
template <typename T>
__global__ __launch_bounds__(64) void k_amr_plevel(ProbDev<T> p, uint8_t *level, const uint8_t *refined, AmrLevels L,
                                                   unsigned *counts)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    int l = level[s];
    double P[4][3];
    if (l > 0 && amr_corners(p, s, P)) {
        double mn[3], mx[3];
        for (int d = 0; d < 3; ++d) {
            mn[d] = mx[d] = P[0][d];
            for (int a = 1; a < 4; ++a) {
                mn[d] = fmin(mn[d], P[a][d]);
                mx[d] = fmax(mx[d], P[a][d]);
            }
        }
        for (; l > 0; --l) {
            const double size = (double)(1 << l);
            const int *nb = L.nb[l];
            const uint8_t *r = refined + L.off[l];
            // (a box of more than 2^22 blocks counts as refined: one level down)
            bool any = (floor(mx[0] / size) - floor(mn[0] / size) + 1) * (floor(mx[1] / size) - floor(mn[1] / size) + 1) *
                           (floor(mx[2] / size) - floor(mn[2] / size) + 1) > 4194304.0;
            for (int bz = (int)floor(mn[2] / size); bz <= (int)floor(mx[2] / size) && !any; ++bz) {
                int wz = bz;
                if (p.g.periodic[2]) wz = wrap_index(bz, nb[2]);
                else if (bz < 0 || bz >= nb[2]) continue;
                for (int by = (int)floor(mn[1] / size); by <= (int)floor(mx[1] / size) && !any; ++by) {
                    int wy = by;
                    if (p.g.periodic[1]) wy = wrap_index(by, nb[1]);
                    else if (by < 0 || by >= nb[1]) continue;
                    for (int bx = (int)floor(mn[0] / size); bx <= (int)floor(mx[0] / size) && !any; ++bx) {
                        int wx = bx;
                        if (p.g.periodic[0]) wx = wrap_index(bx, nb[0]);
                        else if (bx < 0 || bx >= nb[0]) continue;
                        any = r[((size_t)wz * nb[1] + wy) * nb[0] + wx] != 0;
                    }
                }
            }
            if (!any) break;
        }
    } else {
        l = 0;
    }
    level[s] = (uint8_t)l;
    (void)wave_claim(counts, l);
}

struct AmrBases {
    unsigned b[16];  // first compacted slot of each level
};

template <typename T>
__global__ __launch_bounds__(256) void k_amr_scatter(ProbDev<T> p, const uint8_t *level, unsigned *cursor,
                                                     AmrBases base, int32_t *simp, T *rho)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n) return;
    const int lv = level[s];
    const int64_t t = (int64_t)base.b[lv] + wave_claim(cursor, lv);
    for (int a = 0; a < 4; ++a) {
        simp[t * 4 + a] = p.simp[s * 4 + a];
        if (rho) rho[t * 4 + a] = p.rho[s * 4 + a];
    }
}

// Level l's grid (masses of its own simplices) plus the sums of the 8
// children of each of its cells in level l - 1's summed grid.
template <typename T>
__global__ __launch_bounds__(256) void k_amr_restrict(T *up, const T *down, AmrLevels L, int l)
{
    const int *nb = L.nb[l], *nc = L.nb[l - 1];
    const size_t nblk = (size_t)nb[0] * nb[1] * nb[2];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nblk; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nb[0]), y = (int)((i / nb[0]) % nb[1]), z = (int)(i / ((size_t)nb[0] * nb[1]));
        T acc = up[i];
        for (int k = 0; k < 8; ++k) {
            const int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
            acc += down[((size_t)cz * nc[1] + cy) * nc[0] + cx];
        }
        up[i] = acc;
    }
}

// Each grid cell: descend from the largest blocks while refined; the leaf's
// summed mass / 8^level, divided by the cell volume for density output.
// sums[l] points at level l's summed grid (sums[0] is out itself).
struct AmrSums {
    void *p[11];
};

template <typename T>
__global__ __launch_bounds__(256) void k_amr_gather(T *out, AmrSums sums, const uint8_t *refined, AmrLevels L,
                                                    int max_level, double to_out)
{
    const int *n0 = L.nb[0];
    const size_t ncell = (size_t)n0[0] * n0[1] * n0[2];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n0[0]), y = (int)((i / n0[0]) % n0[1]), z = (int)(i / ((size_t)n0[0] * n0[1]));
        int l = max_level;
        for (; l > 0; --l) {
            const int *nb = L.nb[l];
            if (!refined[L.off[l] + ((size_t)(z >> l) * nb[1] + (y >> l)) * nb[0] + (x >> l)]) break;
        }
        const int *nb = L.nb[l];
        const T *a = static_cast<const T *>(sums.p[l]);
        const T m = a[((size_t)(z >> l) * nb[1] + (y >> l)) * nb[0] + (x >> l)];
        out[i] = (T)((double)m * (to_out / (double)(1ull << (3 * l))));
    }
}

// hi + lo -> out (unless the caller keeps lo), FP64 total of the grid in mass
// units.
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(T *out, float *lo, int keep_lo, size_t ncell, double to_mass,
                                                  double *total)
{
    __shared__ double s_sum[256];
    double acc = 0.0;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < ncell; i += st) {
        if constexpr (sizeof(T) == 4) {
            float h = out[i], l = lo[i];
            acc += (double)h + (double)l;
            if (!keep_lo) out[i] = h + l;
        } else {
            acc += (double)out[i];
        }
    }
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) unsafeAtomicAdd(total, s_sum[0] * to_mass);
}

} // namespace

// ---------------------------------------------------------------------------
// host runtime

enum Stage { ST_FILL, ST_SETUP, ST_BIN, ST_CLIP, ST_RETRY, ST_FINAL, ST_N };

// Scratch of sp_project_tets_noalloc: a fixed array in device memory, one
// copy per GPU the library runs on, held until the process ends.  In host
// code `scratch` only names the symbol; its device address (per device) comes
// from hipGetSymbolAddress, taken once per device by sp_create with that
// device current, and only that address is ever handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_noalloc_mu;

// SP_SCRATCH_CAP: bytes, with an optional K, M or G suffix (powers of 1024).
static size_t parse_bytes(const char *e)
{
    char *end = nullptr;
    const double v = strtod(e, &end);
    if (!(v > 0.0)) return 0;
    double m = 1.0;
    if (end && (*end == 'K' || *end == 'k')) m = 1024.0;
    else if (end && (*end == 'M' || *end == 'm')) m = 1024.0 * 1024.0;
    else if (end && (*end == 'G' || *end == 'g')) m = 1024.0 * 1024.0 * 1024.0;
    return (size_t)(v * m);
}

struct sp_ctx {
    int device;
    void *noalloc;   // this device's copy of `scratch` (NULL if its address could not be taken)
    int num_cu;
    void *scratch;
    size_t scratch_cap;
    size_t held;           // device memory held in scratch and aux buffers
    size_t scratch_limit;  // SP_SCRATCH_CAP (0: none)
    CallState *cs;
    ErrState *es;
    double *dummy_total;
    Tuning tune;
    int profiling;
    int group_clip;  // 1: the FP32 3D clip runs one polytope per 16 lanes (k_clipw) instead of one per lane
    int tiled_deposit;  // 1: single FP32 3D problems clip with the per-wave deposit tile
    int prof_calls;
    int last_clip_blocks;
    // (start, end) events per recorded stage and per whole call
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ST_N];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_call;
    // captured batched launches, by problem signature
    hipStream_t cap_stream;
    std::vector<struct GraphEntry> graphs;
    // buffers of the accuracy-controlled projection (grown on demand)
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    } aux[2];
};

struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
    void *dev;  // problem descriptors and simplex offsets of this signature
};

static void drop_graphs(sp_ctx *ctx)
{
    for (GraphEntry &g : ctx->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.dev) (void)hipFree(g.dev);
    }
    ctx->graphs.clear();
}

// Event pair around one stage of a call (no-op unless profiling).
struct StageTimer {
    sp_ctx *ctx;  // NULL: no timing
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *dst;
    StageTimer(sp_ctx *c, hipStream_t st, std::vector<std::pair<hipEvent_t, hipEvent_t>> *d) : ctx(c), s(st), dst(d)
    {
        if (ctx && ctx->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
    }
    StageTimer(StageTimer &&o) noexcept : ctx(o.ctx), s(o.s), a(o.a), b(o.b), dst(o.dst)
    {
        o.a = o.b = nullptr;
    }
    StageTimer(const StageTimer &) = delete;
    ~StageTimer()
    {
        if (a && b) {
            (void)hipEventRecord(b, s);
            dst->push_back({a, b});
        }
    }
};

static thread_local std::string g_err;
static void drop_events(sp_ctx *ctx);

static sp_status fail(sp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHECK(call)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail(SP_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

extern "C" sp_status sp_create(int hip_device, sp_ctx **ctx)
{
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(SP_E_DEVICE, "no HIP device");
    if (hip_device < 0 || hip_device >= n) return fail(SP_E_DEVICE, "device %d out of range (%d devices)", hip_device, n);
    hipDeviceProp_t prop;
    HIPCHECK(hipGetDeviceProperties(&prop, hip_device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SP_E_DEVICE, "device %d is %s, this library is built for gfx950", hip_device, prop.gcnArchName);
    HIPCHECK(hipSetDevice(hip_device));
    sp_ctx *c = new sp_ctx();
    c->device = hip_device;
    c->num_cu = prop.multiProcessorCount;
    c->scratch = nullptr;
    c->scratch_cap = 0;
    c->held = 0;
    c->scratch_limit = 0;
    if (const char *e = getenv("SP_SCRATCH_CAP")) c->scratch_limit = parse_bytes(e);
    void *st = nullptr;
    if (hipMalloc(&st, 4096) != hipSuccess) {
        delete c;
        return fail(SP_E_NO_MEMORY, "hipMalloc of the context state failed");
    }
    c->cs = reinterpret_cast<CallState *>(st);
    c->es = reinterpret_cast<ErrState *>(reinterpret_cast<char *>(st) + 1024);
    c->dummy_total = reinterpret_cast<double *>(reinterpret_cast<char *>(st) + 2048);
    (void)hipMemset(st, 0, 4096);
    (void)hipDeviceSynchronize();
    c->tune.slab_group = 16;
    c->tune.chunks_per_cu = 0;
    c->tune.item_pieces = 0;
    // launch-shape overrides for tuning experiments
    if (const char *e = getenv("SIMPROJ_SLAB_GROUP")) c->tune.slab_group = atoi(e) > 0 ? atoi(e) : 16;
    if (const char *e = getenv("SIMPROJ_CLIP_BLOCKS_PER_CU")) c->tune.chunks_per_cu = atoi(e) > 0 ? atoi(e) : 0;
    if (const char *e = getenv("SIMPROJ_ITEM_PIECES")) c->tune.item_pieces = atoi(e) > 0 ? atoi(e) : 0;
    c->profiling = 0;
    c->group_clip = 0;
    if (const char *e = getenv("SIMPROJ_GROUP_CLIP")) c->group_clip = atoi(e) != 0;
    c->tiled_deposit = 0;
    if (const char *e = getenv("SIMPROJ_TILED_DEPOSIT")) c->tiled_deposit = atoi(e) != 0;
    c->prof_calls = 0;
    c->last_clip_blocks = 0;
    c->noalloc = nullptr;
    if (hip_device < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[hip_device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_noalloc_ptr[hip_device] = ptr;
            else (void)hipGetLastError();
        }
        c->noalloc = g_noalloc_ptr[hip_device];
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(st);
        delete c;
        return fail(SP_E_DEVICE, "stream creation failed");
    }
    *ctx = c;
    return SP_OK;
}

extern "C" void sp_destroy(sp_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    drop_events(ctx);
    drop_graphs(ctx);
    (void)hipStreamDestroy(ctx->cap_stream);
    // (the stream-ordered blocks are returned on the null stream, which the
    // device-wide synchronisation above has drained, and waited for)
    for (auto &b : ctx->aux)
        if (b.p) (void)hipFreeAsync(b.p, nullptr);
    if (ctx->scratch) (void)hipFreeAsync(ctx->scratch, nullptr);
    (void)hipStreamSynchronize(nullptr);
    (void)hipFree(ctx->cs);
    delete ctx;
}

extern "C" const char *sp_last_error(const sp_ctx *)
{
    return g_err.c_str();
}

// Device memory the context owns grows in stream order on the call's
// stream: the old block is freed and the new one allocated behind the work
// already enqueued there (calls on one context are ordered, so nothing else
// still uses it), without waiting for the device.  SP_SCRATCH_CAP bounds the
// total the context may hold; a call that needs more fails with
// SP_E_NO_MEMORY before it enqueues anything.
static sp_status grow(sp_ctx *ctx, void *&p, size_t &cap, size_t bytes, hipStream_t stream, const char *what)
{
    const size_t others = ctx->held - cap;
    if (ctx->scratch_limit && others + bytes > ctx->scratch_limit)
        return fail(SP_E_NO_MEMORY, "the call needs %zu bytes of %s (%zu held elsewhere); SP_SCRATCH_CAP allows %zu",
                    bytes, what, others, ctx->scratch_limit);
    size_t want = bytes + bytes / 4;
    if (ctx->scratch_limit && others + want > ctx->scratch_limit) want = ctx->scratch_limit - others;
    if (p) (void)hipFreeAsync(p, stream);
    p = nullptr;
    ctx->held -= cap;
    cap = 0;
    if (hipMallocAsync(&p, want, stream) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return fail(SP_E_NO_MEMORY, "allocation of %zu bytes of %s failed", want, what);
    }
    cap = want;
    ctx->held += cap;
    return SP_OK;
}

static sp_status ensure_buf(sp_ctx *ctx, sp_ctx::Buf &b, size_t bytes, hipStream_t stream)
{
    if (bytes <= b.cap) return SP_OK;
    return grow(ctx, b.p, b.cap, bytes, stream, "buffer");
}

static sp_status ensure_scratch(sp_ctx *ctx, size_t bytes, hipStream_t stream)
{
    if (bytes <= ctx->scratch_cap) return SP_OK;
    if (!ctx->graphs.empty()) {
        // captured launches refer to the old scratch: let them finish, drop them
        HIPCHECK(hipDeviceSynchronize());
        drop_graphs(ctx);
    }
    return grow(ctx, ctx->scratch, ctx->scratch_cap, bytes, stream, "scratch");
}


static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static sp_status check_problem(const sp_problem *p, int dim, sp_precision prec)
{
    if (!p) return fail(SP_E_INVALID_ARG, "problem is NULL");
    if (prec != SP_PREC_FP64 && prec != SP_PREC_FP32C) return fail(SP_E_INVALID_ARG, "unknown precision %d", (int)prec);
    const uint32_t known = SP_PERIODIC_X | SP_PERIODIC_Y | SP_PERIODIC_Z | SP_RHO_PER_CORNER | SP_OUT_MASS |
                           SP_ACCUMULATE | SP_VALIDATE;
    if (p->grid.flags & ~known) return fail(SP_E_INVALID_ARG, "unknown flag bits 0x%x", p->grid.flags & ~known);
    if (p->n_vert < 0 || p->n_vert >= (int64_t)1 << 31) return fail(SP_E_INVALID_ARG, "n_vert %lld out of range", (long long)p->n_vert);
    if (p->n_simplex < 0 || p->n_simplex >= (int64_t)1 << 31)
        return fail(SP_E_INVALID_ARG, "n_simplex %lld out of range", (long long)p->n_simplex);
    for (int d = 0; d < dim; ++d) {
        if (p->grid.dims[d] <= 0 || p->grid.dims[d] > (1 << 20)) return fail(SP_E_INVALID_ARG, "dims[%d] = %d out of range", d, p->grid.dims[d]);
        if (!(p->grid.extent[d] > 0.0) || !isfinite(p->grid.extent[d])) return fail(SP_E_INVALID_ARG, "extent[%d] must be > 0", d);
        if (!isfinite(p->grid.origin[d])) return fail(SP_E_INVALID_ARG, "origin[%d] must be finite", d);
    }
    double nc = 1.0;
    for (int d = 0; d < dim; ++d) nc *= p->grid.dims[d];
    if (nc > 34359738368.0) return fail(SP_E_INVALID_ARG, "grid of %.0f cells is too large (limit 2^35)", nc);
    if (!p->out) return fail(SP_E_INVALID_ARG, "out is NULL");
    if (p->n_simplex > 0 && (!p->xyz || !p->simplices || !p->rho)) return fail(SP_E_INVALID_ARG, "xyz, simplices and rho must not be NULL");
    if (p->out_lo && prec != SP_PREC_FP32C) return fail(SP_E_INVALID_ARG, "out_lo is only used with SP_PREC_FP32C");
    return SP_OK;
}

template <typename T>
static void fill_grid(GridDev &g, const sp_problem *p, int dim)
{
    memset(&g, 0, sizeof g);
    double cellvol = 1.0;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            g.dims[d] = p->grid.dims[d];
            g.periodic[d] = (p->grid.flags >> d) & 1u;
            g.origin[d] = p->grid.origin[d];
            g.extent[d] = p->grid.extent[d];
            g.scale[d] = (double)p->grid.dims[d] / p->grid.extent[d];
            cellvol *= p->grid.extent[d] / (double)p->grid.dims[d];
        } else {
            g.dims[d] = 1;
            g.periodic[d] = 1;
            g.origin[d] = 0;
            g.extent[d] = 1;
            g.scale[d] = 1;
        }
        g.o_hi[d] = (float)g.origin[d];
        g.o_lo[d] = (float)(g.origin[d] - (double)g.o_hi[d]);
        g.s_hi[d] = (float)g.scale[d];
        g.s_lo[d] = (float)(g.scale[d] - (double)g.s_hi[d]);
    }
    g.out_scale = (p->grid.flags & SP_OUT_MASS) ? cellvol : 1.0;
}

static int grid_blocks(size_t n, int per)
{
    size_t b = (n + per - 1) / per;
    if (b > 65536 * 8) b = 65536 * 8;
    if (b < 1) b = 1;
    return (int)b;
}

// One problem of a launch: its device descriptor and the host-side facts
// its fill and finalize steps need.
template <typename T>
struct Prepared {
    ProbDev<T> p;
    size_t ncell;
    bool keep_lo, accumulate;
    double to_mass;
    double *total;
};

// Scratch layout and descriptors for a launch over n problems.
template <int D, typename T>
// work_lists = false (the corner-sum path) leaves out the set-up, item and
// overflow lists that only the clipping kernels use.
// fixed != NULL (the no-allocation entry point): lay the scratch out in
// that buffer of fixed_cap bytes instead of the context's, with room for
// fewer split items, and fail when it does not fit.
static sp_status prepare(sp_ctx *ctx, const sp_problem *probs, int n, Prepared<T> *out, int64_t &ntotal,
                         hipStream_t stream, bool batched = false, bool work_lists = true, void *fixed = nullptr,
                         size_t fixed_cap = 0)
{
    const bool fp32 = sizeof(T) == 4;
    ntotal = 0;
    size_t lo_cells = 0;
    for (int i = 0; i < n; ++i) {
        ntotal += probs[i].n_simplex;
        size_t nc = 1;
        for (int d = 0; d < D; ++d) nc *= (size_t)probs[i].grid.dims[d];
        if (fp32 && !probs[i].out_lo) lo_cells += nc;
    }
    if (ntotal >= ((int64_t)1 << 31)) return fail(SP_E_INVALID_ARG, "%lld simplices in one launch (limit 2^31)", (long long)ntotal);
    // room for the split items: as many again as the simplices plus 2M
    // (16 MB); the no-allocation scratch holds half the simplices plus 256K.
    // A block whose split items do not fit keeps its simplices whole.
    const unsigned extra_cap = (unsigned)(fixed ? ntotal / 2 + (1 << 18) : ntotal + (1 << 21));
    const size_t nitems = work_lists ? (size_t)ntotal + extra_cap : 0;
    size_t off = 0;
    const size_t o_tinfo = off;
    if (work_lists) off = align_up(off + sizeof(uint32_t) * (size_t)(ntotal > 0 ? ntotal : 1));
    const size_t o_rec = off;
    if (work_lists && D == 3) off = align_up(off + sizeof(SimplexRec<T>) * (size_t)(ntotal > 0 ? ntotal : 1));
    const size_t o_items = off;
    off = align_up(off + sizeof(uint64_t) * nitems);
    const size_t o_iprob = off;
    if (batched) off = align_up(off + sizeof(uint16_t) * nitems);  // problem id per item
    const size_t o_ovf = off;
    if (work_lists) off = align_up(off + sizeof(Ovf) * OVF_CAP);
    const size_t o_lo = off;
    off = align_up(off + sizeof(float) * lo_cells);
    char *base;
    if (fixed) {
        if (off > fixed_cap)
            return fail(SP_E_NO_MEMORY, "the problem needs %zu bytes of scratch; the static scratch of the no-allocation "
                                        "entry point holds %zu", off, fixed_cap);
        base = reinterpret_cast<char *>(fixed);
    } else {
        sp_status st = ensure_scratch(ctx, off, stream);
        if (st != SP_OK) return st;
        base = reinterpret_cast<char *>(ctx->scratch);
    }
    int64_t toff = 0;
    size_t loff = 0;
    for (int i = 0; i < n; ++i) {
        const sp_problem *prob = &probs[i];
        Prepared<T> &q = out[i];
        ProbDev<T> &p = q.p;
        q.ncell = 1;
        for (int d = 0; d < D; ++d) q.ncell *= (size_t)prob->grid.dims[d];
        q.keep_lo = fp32 && prob->out_lo != nullptr;
        q.accumulate = (prob->grid.flags & SP_ACCUMULATE) != 0;
        q.total = prob->total_mass;
        q.to_mass = 1.0;
        if (!(prob->grid.flags & SP_OUT_MASS))
            for (int d = 0; d < D; ++d) q.to_mass *= prob->grid.extent[d] / (double)prob->grid.dims[d];
        p.xyz = reinterpret_cast<const T *>(prob->xyz);
        p.n_vert = prob->n_vert;
        p.simp = prob->simplices;
        p.n = prob->n_simplex;
        p.rho = reinterpret_cast<const T *>(prob->rho);
        p.per_corner = (prob->grid.flags & SP_RHO_PER_CORNER) != 0;
        p.validate = (prob->grid.flags & SP_VALIDATE) != 0;
        fill_grid<T>(p.g, prob, D);
        p.out = reinterpret_cast<T *>(prob->out);
        p.lo = nullptr;
        if (fp32) {
            if (q.keep_lo) {
                p.lo = prob->out_lo;
            } else {
                p.lo = reinterpret_cast<float *>(base + o_lo) + loff;
                loff += q.ncell;
            }
        }
        p.tinfo = work_lists ? reinterpret_cast<uint32_t *>(base + o_tinfo) + toff : nullptr;
        p.rec = work_lists && D == 3 ? reinterpret_cast<SimplexRec<T> *>(base + o_rec) + toff : nullptr;
        toff += prob->n_simplex;
        p.items = work_lists ? reinterpret_cast<uint64_t *>(base + o_items) : nullptr;
        p.item_prob = batched && work_lists ? reinterpret_cast<uint16_t *>(base + o_iprob) : nullptr;
        p.extra_cap = extra_cap;
        p.ovf = work_lists ? reinterpret_cast<Ovf *>(base + o_ovf) : nullptr;
        p.cs = ctx->cs;
        p.es = ctx->es;
        p.slab_group = ctx->tune.slab_group;
        p.item_pieces = (float)(ctx->tune.item_pieces > 0 ? ctx->tune.item_pieces : auto_item_pieces(ntotal, ctx->num_cu));
        p.count_pieces = ctx->profiling >= 2;
        p.cmax = nullptr;
    }
    return SP_OK;
}

// The kernels of one launch, in stream order.  With timers, each stage is
// bracketed by HIP events (profiling of direct calls; captured graphs are
// timed as a whole).
template <int D, typename T>
static void enqueue(sp_ctx *ctx, const Prepared<T> *v, int nv, const Batch &b, int64_t nblocks, hipStream_t stream,
                    bool timers)
{
    const bool fp32 = sizeof(T) == 4;
    const bool single = b.nprob == 0;
    const ProbDev<T> &p0 = v[0].p;
    auto timer = [&](int stage) { return StageTimer(timers ? ctx : nullptr, stream, &ctx->ev[stage]); };
    {
        StageTimer t = timer(ST_FILL);
        hipLaunchKernelGGL(k_clear_state, dim3(1), dim3(64), 0, stream, ctx->cs, single ? v[0].total : nullptr);
        for (int qi = 0; qi < nv; ++qi) {
            const Prepared<T> &q = v[qi];
            if (!single && q.total) hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, stream, q.total, (size_t)1);
            if (!q.accumulate)
                hipLaunchKernelGGL(k_fill<T>, dim3(grid_blocks(q.ncell, 256)), dim3(256), 0, stream, q.p.out, q.ncell);
            if (fp32 && (!q.accumulate || !q.keep_lo))
                hipLaunchKernelGGL(k_fill<float>, dim3(grid_blocks(q.ncell, 256)), dim3(256), 0, stream, q.p.lo, q.ncell);
        }
    }
    if (nblocks > 0) {
        const int nb = (int)nblocks;
        {
            StageTimer t = timer(ST_SETUP);
            if (single) hipLaunchKernelGGL((k_setup<D, T, false>), dim3(nb), dim3(256), 0, stream, p0, b);
            else hipLaunchKernelGGL((k_setup<D, T, true>), dim3(nb), dim3(256), 0, stream, p0, b);
        }
        {
            StageTimer t = timer(ST_BIN);
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, stream, ctx->cs);
            constexpr int ipt = scatter_per_thread<false>();
            if (single) hipLaunchKernelGGL((k_scatter<T, false>), dim3((nb + ipt - 1) / ipt), dim3(256), 0, stream, p0, b);
            else hipLaunchKernelGGL((k_scatter<T, true>), dim3(nb), dim3(256), 0, stream, p0, b);
        }
        constexpr int MAXV3 = maxv3<T>();
        // a single FP32 problem takes the instance whose problem fields are
        // kernel arguments (uniform registers); the FP64 kernel measured
        // faster with the run-time choice for both forms
        const bool one = fp32 && single;
        auto kclip = one ? k_clip<D, T, MAXV3, true> : k_clip<D, T, MAXV3, false>;
        if constexpr (D == 3 && sizeof(T) == 4) {
            // the deposit tile when asked for and the grid's cells fit its keys
            // (it measured 7-8 % slower than direct deposits on the soup, the
            // lattice and the refined mesh)
            if (one && ctx->tiled_deposit && p0.cmax == nullptr && v[0].ncell < (size_t)DepF32::TILE_EMPTY)
                kclip = k_clip<D, T, MAXV3, true, T, true>;
        }
        auto kretry = D == 3 ? (one ? k_clip<D, T, MAXV3_BIG, true> : k_clip<D, T, MAXV3_BIG, false>) : kclip;
        // 3D FP32: the group kernel when asked for (it measured slower than
        // one polytope per lane on every workload tried)
        const bool grouped = D == 3 && fp32 && ctx->group_clip;
        int occ = 0;
        if constexpr (D == 3 && sizeof(T) == 4) {
            if (grouped)
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, one ? k_clipw<true> : k_clipw<false>, WG, 0);
        }
        if (!grouped) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kclip, WG, 0);
        if (occ < 1) occ = 1;
        const int cpc = ctx->tune.chunks_per_cu > 0 ? ctx->tune.chunks_per_cu : occ;
        const int blocks = ctx->num_cu * cpc;
        ctx->last_clip_blocks = blocks;
        {
            StageTimer t = timer(ST_CLIP);
            if constexpr (D == 3 && sizeof(T) == 4) {
                if (grouped) {
                    if (one) hipLaunchKernelGGL(k_clipw<true>, dim3(blocks), dim3(WG), 0, stream, p0, b);
                    else hipLaunchKernelGGL(k_clipw<false>, dim3(blocks), dim3(WG), 0, stream, p0, b);
                }
            }
            if (!grouped) hipLaunchKernelGGL(kclip, dim3(blocks), dim3(WG), 0, stream, p0, b, 0);
        }
        {
            StageTimer t = timer(ST_RETRY);
            int rocc = 0;
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&rocc, kretry, WG, 0);
            hipLaunchKernelGGL(kretry, dim3(ctx->num_cu * (rocc < 1 ? 1 : rocc)), dim3(WG), 0, stream, p0, b, 1);
            if constexpr (sizeof(T) == 4) {
                // the simplices routed to FP64 (none in most launches: then
                // every wave stops at its first claim)
                auto kwide = k_clip<D, double, MAXV3_BIG, false, float>;
                int wocc = 0;
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&wocc, kwide, WG, 0);
                hipLaunchKernelGGL(kwide, dim3(ctx->num_cu * (wocc < 1 ? 1 : wocc)), dim3(WG), 0, stream, p0, b, 0);
            }
        }
    }
    {
        StageTimer t = timer(ST_FINAL);
        for (int qi = 0; qi < nv; ++qi) {
            const Prepared<T> &q = v[qi];
            if (fp32 || q.total)
                hipLaunchKernelGGL(k_finalize<T>, dim3(grid_blocks(q.ncell, 256 * 8)), dim3(256), 0, stream, q.p.out,
                                   q.p.lo, q.keep_lo ? 1 : 0, q.ncell, q.to_mass, q.total);
        }
    }
}

template <int D, typename T>
static sp_status project_impl(sp_ctx *ctx, const sp_problem *prob, hipStream_t stream)
{
    HIPCHECK(hipSetDevice(ctx->device));
    std::vector<Prepared<T>> v;
    int64_t ntotal = 0;
    v.resize(1);
    sp_status st = prepare<D, T>(ctx, prob, 1, v.data(), ntotal, stream);
    if (st != SP_OK) return st;
    Batch b = {nullptr, nullptr, 0};
    if (ctx->profiling) ctx->prof_calls++;
    {
        StageTimer whole(ctx->profiling ? ctx : nullptr, stream, &ctx->ev_call);
        enqueue<D, T>(ctx, v.data(), (int)v.size(), b, (ntotal + 255) / 256, stream, ctx->profiling != 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return SP_OK;
}

extern "C" sp_status sp_project_tets(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream)
{
    sp_status st = check_problem(prob, 3, prec);
    if (st != SP_OK) return st;
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return prec == SP_PREC_FP32C ? project_impl<3, float>(ctx, prob, s) : project_impl<3, double>(ctx, prob, s);
}

// sp_project_tets without allocating: the work lists live in this device's
// copy of the static scratch; stage timing is off (no events are created).
extern "C" sp_status sp_project_tets_noalloc(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream)
{
    sp_status st = check_problem(prob, 3, prec);
    if (st != SP_OK) return st;
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    if (!ctx->noalloc) return fail(SP_E_DEVICE, "the static scratch of device %d has no device address", ctx->device);
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Batch b = {nullptr, nullptr, 0};
    int64_t ntotal = 0;
    if (prec == SP_PREC_FP32C) {
        Prepared<float> one;
        st = prepare<3, float>(ctx, prob, 1, &one, ntotal, s, false, true, ctx->noalloc, NOALLOC_SCRATCH_BYTES);
        if (st != SP_OK) return st;
        enqueue<3, float>(ctx, &one, 1, b, (ntotal + 255) / 256, s, false);
    } else {
        Prepared<double> one;
        st = prepare<3, double>(ctx, prob, 1, &one, ntotal, s, false, true, ctx->noalloc, NOALLOC_SCRATCH_BYTES);
        if (st != SP_OK) return st;
        enqueue<3, double>(ctx, &one, 1, b, (ntotal + 255) / 256, s, false);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return SP_OK;
}

// Projection by corner sums (FP64): the same result as sp_project_tets in
// FP64 mode, by the paper's own formulation, for comparison; with `fused`
// the terms on facets shared by two simplices are summed once.
static sp_status corners_impl(sp_ctx *ctx, const sp_problem *prob, void *stream, bool fused)
{
    sp_status st = check_problem(prob, 3, SP_PREC_FP64);
    if (st != SP_OK) return st;
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    if (fused && prob->n_simplex >= ((int64_t)1 << 30))
        return fail(SP_E_INVALID_ARG, "n_simplex %lld: the fused corner sums take fewer than 2^30 simplices",
                    (long long)prob->n_simplex);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHECK(hipSetDevice(ctx->device));
    std::vector<Prepared<double>> v;
    int64_t ntotal = 0;
    v.resize(1);
    st = prepare<3, double>(ctx, prob, 1, v.data(), ntotal, s, false, false);
    if (st != SP_OK) return st;
    const Prepared<double> &q = v[0];
    FuseDev f = {nullptr, 0u, nullptr, nullptr, nullptr};
    if (fused && ntotal > 0) {
        // a table of at least twice as many slots as facets
        size_t slots = 1024;
        while (slots < 8 * (size_t)ntotal) slots *= 2;
        const size_t o_tab = 0, o_mate = align_up(o_tab + 4 * slots), o_grad = align_up(o_mate + 16 * (size_t)ntotal),
                     o_side = align_up(o_grad + 24 * (size_t)ntotal), end = align_up(o_side + 4 * (size_t)ntotal);
        st = ensure_buf(ctx, ctx->aux[0], end, s);
        if (st != SP_OK) return st;
        char *base = static_cast<char *>(ctx->aux[0].p);
        f.tab = reinterpret_cast<uint32_t *>(base + o_tab);
        f.mask = (uint32_t)(slots - 1);
        f.mate = reinterpret_cast<uint32_t *>(base + o_mate);
        f.grad = reinterpret_cast<double *>(base + o_grad);
        f.side = reinterpret_cast<int8_t *>(base + o_side);
        // the table and the mates start empty (zero); tab and mate are contiguous
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_blocks(o_grad / 4, 256)), dim3(256), 0, s, f.tab, o_grad / 4);
    }
    hipLaunchKernelGGL(k_clear_state, dim3(1), dim3(64), 0, s, ctx->cs, q.total);
    if (!q.accumulate)
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_blocks(q.ncell, 256)), dim3(256), 0, s, q.p.out, q.ncell);
    if (f.mate)
        hipLaunchKernelGGL(k_corner_prep, dim3(grid_blocks((size_t)ntotal, 256)), dim3(256), 0, s, q.p, f);
    if (ntotal > 0) {
        if (f.mate)
            hipLaunchKernelGGL(k_corner<true>, dim3(grid_blocks((size_t)ntotal, 64)), dim3(64), 0, s, q.p, f);
        else
            hipLaunchKernelGGL(k_corner<false>, dim3(grid_blocks((size_t)ntotal, 64)), dim3(64), 0, s, q.p, f);
    }
    if (q.total)
        hipLaunchKernelGGL(k_finalize<double>, dim3(grid_blocks(q.ncell, 256 * 8)), dim3(256), 0, s, q.p.out, nullptr,
                           0, q.ncell, q.to_mass, q.total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return SP_OK;
}

extern "C" sp_status sp_project_tets_corners(sp_ctx *ctx, const sp_problem *prob, void *stream)
{
    return corners_impl(ctx, prob, stream, false);
}

extern "C" sp_status sp_project_tets_corners_fused(sp_ctx *ctx, const sp_problem *prob, void *stream)
{
    return corners_impl(ctx, prob, stream, true);
}

extern "C" sp_status sp_project_tris(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream)
{
    sp_status st = check_problem(prob, 2, prec);
    if (st != SP_OK) return st;
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return prec == SP_PREC_FP32C ? project_impl<2, float>(ctx, prob, s) : project_impl<2, double>(ctx, prob, s);
}

// Accuracy-controlled projection (Section 3.4): FP32C projection with the
// largest contribution of every cell recorded, flag the cells whose sum may
// have fewer than `accurate_bits` correct bits, re-project in FP64 the
// simplices that touch them, and replace the flagged cells.
extern "C" sp_status sp_project_tets_accurate(sp_ctx *ctx, const sp_problem *prob, int accurate_bits,
                                              int wrong_bits, int64_t *counts, void *stream)
{
    sp_status st = check_problem(prob, 3, SP_PREC_FP32C);
    if (st != SP_OK) return st;
    if (prob->grid.flags & SP_ACCUMULATE) return fail(SP_E_INVALID_ARG, "SP_ACCUMULATE is not supported here");
    if (accurate_bits < 1 || accurate_bits > 40) return fail(SP_E_INVALID_ARG, "accurate_bits %d not in 1..40", accurate_bits);
    if (wrong_bits < 0 || wrong_bits > 23) return fail(SP_E_INVALID_ARG, "wrong_bits %d not in 0..23", wrong_bits);
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    size_t ncell = 1;
    for (int d = 0; d < 3; ++d) ncell *= (size_t)prob->grid.dims[d];
    const int64_t n = prob->n_simplex;
    const bool own_lo = prob->out_lo == nullptr;
    // phase-1 buffers: low grid (unless the caller's), largest contribution,
    // flags, two counters, tag list, FP64 patch grid
    size_t off = 0;
    const size_t o_lo = off;
    off = align_up(off + (own_lo ? sizeof(float) * ncell : 0));
    const size_t o_cmax = off;
    off = align_up(off + sizeof(uint32_t) * ncell);
    const size_t o_flag = off;
    off = align_up(off + ncell);
    const size_t o_cnt = off;
    off = align_up(off + 2 * sizeof(unsigned long long));
    const size_t o_list = off;
    off = align_up(off + sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_patch = off;
    off = align_up(off + sizeof(double) * ncell);
    st = ensure_buf(ctx, ctx->aux[0], off, s);
    if (st != SP_OK) return st;
    char *base = static_cast<char *>(ctx->aux[0].p);
    float *lo = own_lo ? reinterpret_cast<float *>(base + o_lo) : prob->out_lo;
    uint32_t *cmax = reinterpret_cast<uint32_t *>(base + o_cmax);
    uint8_t *flags = reinterpret_cast<uint8_t *>(base + o_flag);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(base + o_cnt);
    int32_t *list = reinterpret_cast<int32_t *>(base + o_list);
    double *patch = reinterpret_cast<double *>(base + o_patch);

    // 1. FP32C projection into out + lo (both kept), largest contribution per cell
    sp_problem p1 = *prob;
    p1.out_lo = lo;
    p1.total_mass = nullptr;
    std::vector<Prepared<float>> v;
    int64_t ntotal = 0;
    v.resize(1);
    st = prepare<3, float>(ctx, &p1, 1, v.data(), ntotal, s);
    if (st != SP_OK) return st;
    v[0].p.cmax = cmax;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_blocks(ncell, 256)), dim3(256), 0, s, cmax, ncell);
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, cnt, (size_t)2);
    Batch nb = {nullptr, nullptr, 0};
    enqueue<3, float>(ctx, v.data(), (int)v.size(), nb, (ntotal + 255) / 256, s, false);
    // 2. flags and tags
    const float factor = ldexpf(1.0f, wrong_bits + accurate_bits - 23);
    hipLaunchKernelGGL(k_flag, dim3(grid_blocks(ncell, 256)), dim3(256), 0, s, (const float *)prob->out,
                       (const float *)lo, (const uint32_t *)cmax, ncell, factor, flags, cnt);
    if (n > 0)
        hipLaunchKernelGGL(k_tag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v[0].p, (const uint8_t *)flags,
                           list, cnt + 1);
    unsigned long long hc[2] = {0, 0};
    HIPCHECK(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const int64_t ntag = (int64_t)hc[1];
    // 3. FP64 re-projection of the tagged simplices, patched into the flagged cells
    if (ntag > 0) {
        const size_t nx = 3 * (size_t)prob->n_vert;
        const size_t q_x = 0;
        const size_t q_s = align_up(q_x + sizeof(double) * nx);
        const size_t q_r = align_up(q_s + sizeof(int32_t) * 4 * (size_t)ntag);
        const size_t q_end = align_up(q_r + sizeof(double) * 4 * (size_t)ntag);
        st = ensure_buf(ctx, ctx->aux[1], q_end, s);
        if (st != SP_OK) return st;
        char *b2 = static_cast<char *>(ctx->aux[1].p);
        double *x64 = reinterpret_cast<double *>(b2 + q_x);
        int32_t *simp = reinterpret_cast<int32_t *>(b2 + q_s);
        double *rho = reinterpret_cast<double *>(b2 + q_r);
        hipLaunchKernelGGL(k_widen, dim3(grid_blocks(nx, 256)), dim3(256), 0, s, (const float *)prob->xyz, nx, x64);
        hipLaunchKernelGGL(k_gather_tagged, dim3((unsigned)((ntag + 255) / 256)), dim3(256), 0, s, v[0].p,
                           (const int32_t *)list, ntag, simp, rho);
        sp_problem p2;
        memset(&p2, 0, sizeof p2);
        p2.xyz = x64;
        p2.n_vert = prob->n_vert;
        p2.simplices = simp;
        p2.n_simplex = ntag;
        p2.rho = rho;
        p2.grid = prob->grid;
        p2.grid.flags = (prob->grid.flags & (SP_PERIODIC_X | SP_PERIODIC_Y | SP_PERIODIC_Z | SP_OUT_MASS)) |
                        SP_RHO_PER_CORNER;
        p2.out = patch;
        st = project_impl<3, double>(ctx, &p2, s);
        if (st != SP_OK) return st;
        hipLaunchKernelGGL(k_patch, dim3(grid_blocks(ncell, 256)), dim3(256), 0, s, (float *)prob->out, lo,
                           (const uint8_t *)flags, (const double *)patch, ncell);
    }
    // 4. merge (unless the caller keeps the low grid) and the FP64 total
    if (prob->total_mass) hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, s, prob->total_mass, (size_t)1);
    hipLaunchKernelGGL(k_finalize<float>, dim3(grid_blocks(ncell, 256 * 8)), dim3(256), 0, s, (float *)prob->out, lo,
                       own_lo ? 0 : 1, ncell, v[0].to_mass, prob->total_mass);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    if (counts) {
        counts[0] = (int64_t)hc[0];
        counts[1] = ntag;
    }
    return SP_OK;
}

template <int D, typename T>
static sp_status batch_impl(sp_ctx *ctx, const sp_problem *probs, int n, sp_precision prec, hipStream_t stream);

template <typename T>
static sp_status amr_impl(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, int max_level, int64_t *level_counts,
                          hipStream_t s)
{
    HIPCHECK(hipSetDevice(ctx->device));
    const int64_t n = prob->n_simplex;
    const bool per_corner = (prob->grid.flags & SP_RHO_PER_CORNER) != 0;
    // block counts per level; byte grids of marks (later: refined) for
    // levels 1..max_level, packed in one buffer
    AmrLevels L;
    memset(&L, 0, sizeof L);
    size_t mark_bytes = 0;
    size_t nblk[11];
    for (int l = 0; l <= max_level; ++l) {
        nblk[l] = 1;
        for (int d = 0; d < 3; ++d) {
            L.nb[l][d] = prob->grid.dims[d] >> l;
            nblk[l] *= (size_t)L.nb[l][d];
        }
        if (l >= 1) {
            L.off[l] = mark_bytes;
            mark_bytes = align_up(mark_bytes + nblk[l]);
        }
    }
    // buffers: levels, counters, cursors, compacted simplices (and corner
    // densities), marks, one summed grid per level >= 1
    size_t off = 0;
    const size_t o_lv = off;
    off = align_up(off + (size_t)(n > 0 ? n : 1));
    const size_t o_cnt = off;
    off = align_up(off + 3 * 16 * sizeof(unsigned));
    const size_t o_simp = off;
    off = align_up(off + sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
    const size_t o_rho = off;
    off = align_up(off + (per_corner ? sizeof(T) * 4 * (size_t)n : 0));
    const size_t o_marks = off;
    off = align_up(off + (mark_bytes > 0 ? mark_bytes : 1));
    size_t o_sum[11] = {0};
    for (int l = 1; l <= max_level; ++l) {
        o_sum[l] = off;
        off = align_up(off + sizeof(T) * nblk[l]);
    }
    sp_status st = ensure_buf(ctx, ctx->aux[1], off, s);
    if (st != SP_OK) return st;
    char *base = static_cast<char *>(ctx->aux[1].p);
    uint8_t *lv = reinterpret_cast<uint8_t *>(base + o_lv);
    unsigned *counts = reinterpret_cast<unsigned *>(base + o_cnt);
    unsigned *cursor = counts + 16;
    int32_t *simp = reinterpret_cast<int32_t *>(base + o_simp);
    T *rho = per_corner ? reinterpret_cast<T *>(base + o_rho) : nullptr;
    uint8_t *marks = reinterpret_cast<uint8_t *>(base + o_marks);
    std::vector<Prepared<T>> v;
    int64_t ntot = 0;
    // a descriptor of the input, for the per-simplex kernels
    v.resize(1);
    st = prepare<3, T>(ctx, prob, 1, v.data(), ntot, s);
    if (st != SP_OK) return st;
    const ProbDev<T> pin = v[0].p;
    unsigned hc[16] = {0}, hb[16] = {0};
    hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, counts, (size_t)48);
    if (mark_bytes > 0)
        hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_blocks(mark_bytes, 256)), dim3(256), 0, s, marks, mark_bytes);
    if (n > 0) {
        const unsigned nb64 = (unsigned)((n + 63) / 64), nb256 = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_amr_level<T>, dim3(nb256), dim3(256), 0, s, pin, max_level, lv);
        if (max_level >= 1) {
            hipLaunchKernelGGL(k_amr_mark<T>, dim3(nb64), dim3(64), 0, s, pin, max_level, (const uint8_t *)lv, marks, L);
            for (int l = 2; l <= max_level; ++l)
                hipLaunchKernelGGL(k_amr_refine, dim3(grid_blocks(nblk[l], 256)), dim3(256), 0, s, marks, L, l);
        }
        hipLaunchKernelGGL(k_amr_plevel<T>, dim3(nb64), dim3(64), 0, s, pin, lv, (const uint8_t *)marks, L, counts);
        HIPCHECK(hipMemcpyAsync(hc, counts, sizeof hc, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        AmrBases ab;
        for (int l = 0; l < 16; ++l) ab.b[l] = 0u;
        for (int l = 1; l <= max_level; ++l) hb[l] = hb[l - 1] + hc[l - 1];
        for (int l = 0; l <= max_level; ++l) ab.b[l] = hb[l];
        hipLaunchKernelGGL(k_amr_scatter<T>, dim3(nb256), dim3(256), 0, s, pin, (const uint8_t *)lv, cursor, ab, simp,
                           rho);
    }
    // one problem per projection level, in mass units (level 0 writes the
    // caller's grid), projected in one batched launch; all levels add to the
    // caller's total; an unused level's grid is zeroed
    std::vector<sp_problem> probs;
    AmrSums sums;
    memset(&sums, 0, sizeof sums);
    sums.p[0] = prob->out;
    for (int l = 0; l <= max_level; ++l) {
        if (l > 0) sums.p[l] = base + o_sum[l];
        if (l > 0 && hc[l] == 0) {
            hipLaunchKernelGGL(k_fill<T>, dim3(grid_blocks(nblk[l], 256)), dim3(256), 0, s, (T *)sums.p[l], nblk[l]);
            continue;
        }
        sp_problem q = *prob;
        q.simplices = simp + 4 * (size_t)hb[l];
        q.n_simplex = hc[l];
        if (per_corner) q.rho = rho + 4 * (size_t)hb[l];
        for (int d = 0; d < 3; ++d) q.grid.dims[d] = prob->grid.dims[d] >> l;
        q.grid.flags |= SP_OUT_MASS;
        q.out = sums.p[l];
        q.out_lo = nullptr;
        probs.push_back(q);
    }
    st = batch_impl<3, T>(ctx, probs.data(), (int)probs.size(), prec, s);
    if (st != SP_OK) return st;
    for (int l = 1; l <= max_level; ++l)
        hipLaunchKernelGGL(k_amr_restrict<T>, dim3(grid_blocks(nblk[l], 256)), dim3(256), 0, s, (T *)sums.p[l],
                           (const T *)sums.p[l - 1], L, l);
    double cellvol = 1.0;
    for (int d = 0; d < 3; ++d) cellvol *= prob->grid.extent[d] / (double)prob->grid.dims[d];
    const double to_out = (prob->grid.flags & SP_OUT_MASS) ? 1.0 : 1.0 / cellvol;
    hipLaunchKernelGGL(k_amr_gather<T>, dim3(grid_blocks(nblk[0], 256)), dim3(256), 0, s, (T *)prob->out, sums,
                       (const uint8_t *)marks, L, max_level, to_out);
    if (prob->out_lo)  // the whole result is in out
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_blocks(nblk[0], 256)), dim3(256), 0, s, prob->out_lo, nblk[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    if (level_counts)
        for (int l = 0; l <= max_level; ++l) level_counts[l] = hc[l];
    return SP_OK;
}

extern "C" sp_status sp_project_tets_amr(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, int max_level,
                                         int64_t *level_counts, void *stream)
{
    sp_status st = check_problem(prob, 3, prec);
    if (st != SP_OK) return st;
    if (prob->grid.flags & SP_ACCUMULATE) return fail(SP_E_INVALID_ARG, "SP_ACCUMULATE is not supported here");
    if (max_level < 0 || max_level > 10) return fail(SP_E_INVALID_ARG, "max_level %d not in 0..10", max_level);
    for (int d = 0; d < 3; ++d)
        if (prob->grid.dims[d] % (1 << max_level) != 0)
            return fail(SP_E_INVALID_ARG, "dims[%d] = %d is not a multiple of 2^max_level", d, prob->grid.dims[d]);
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return prec == SP_PREC_FP32C ? amr_impl<float>(ctx, prob, prec, max_level, level_counts, s)
                                 : amr_impl<double>(ctx, prob, prec, max_level, level_counts, s);
}

// FNV-1a over the bytes that determine a batched launch.
static uint64_t fnv(uint64_t h, const void *data, size_t n)
{
    const unsigned char *c = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <int D, typename T>
static sp_status batch_impl(sp_ctx *ctx, const sp_problem *probs, int n, sp_precision prec, hipStream_t stream)
{
    HIPCHECK(hipSetDevice(ctx->device));
    std::vector<Prepared<T>> v;
    int64_t ntotal = 0;
    v.resize(n);
    sp_status st = prepare<D, T>(ctx, probs, n, v.data(), ntotal, stream, true);
    if (st != SP_OK) return st;
    uint64_t key = 1469598103934665603ull;
    const int dim = D;
    key = fnv(key, &dim, sizeof dim);
    key = fnv(key, &prec, sizeof prec);
    key = fnv(key, &n, sizeof n);
    key = fnv(key, probs, sizeof(sp_problem) * (size_t)n);
    key = fnv(key, &ctx->tune, sizeof ctx->tune);
    const int pmode = ctx->profiling >= 2 ? 2 : 0;
    key = fnv(key, &pmode, sizeof pmode);
    key = fnv(key, &ctx->scratch, sizeof ctx->scratch);
    GraphEntry *ge = nullptr;
    for (GraphEntry &g : ctx->graphs)
        if (g.key == key) ge = &g;
    if (!ge) {
        if (ctx->graphs.size() >= 16) drop_graphs(ctx);
        GraphEntry g;
        g.key = key;
        g.exec = nullptr;
        g.dev = nullptr;
        // descriptors and first set-up blocks, uploaded once for this signature
        const size_t bytes = sizeof(ProbDev<T>) * (size_t)n + sizeof(int32_t) * (size_t)(n + 1);
        HIPCHECK(hipMalloc(&g.dev, bytes));
        std::vector<unsigned char> host(bytes);
        std::vector<int32_t> boffs(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            memcpy(host.data() + sizeof(ProbDev<T>) * i, &v[i].p, sizeof(ProbDev<T>));
            boffs[i + 1] = boffs[i] + (int32_t)((probs[i].n_simplex + 255) / 256);
        }
        memcpy(host.data() + sizeof(ProbDev<T>) * n, boffs.data(), sizeof(int32_t) * (n + 1));
        HIPCHECK(hipMemcpy(g.dev, host.data(), bytes, hipMemcpyHostToDevice));
        Batch b;
        b.probs = g.dev;
        b.boffs = reinterpret_cast<const int32_t *>(static_cast<char *>(g.dev) + sizeof(ProbDev<T>) * n);
        b.nprob = n;
        // capture the whole launch sequence once; replays cost one launch
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue<D, T>(ctx, v.data(), (int)v.size(), b, boffs[n], ctx->cap_stream, false);
        hipError_t e1 = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (e1 != hipSuccess) {
            (void)hipFree(g.dev);
            return fail(SP_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e1));
        }
        hipError_t e2 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            (void)hipFree(g.dev);
            return fail(SP_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e2));
        }
        ctx->graphs.push_back(g);
        ge = &ctx->graphs.back();
    }
    if (ctx->profiling) ctx->prof_calls++;
    {
        StageTimer whole(ctx->profiling ? ctx : nullptr, stream, &ctx->ev_call);
        HIPCHECK(hipGraphLaunch(ge->exec, stream));
    }
    return SP_OK;
}

extern "C" sp_status sp_project_batch(sp_ctx *ctx, int dim, const sp_problem *probs, int n, sp_precision prec, void *stream)
{
    if (dim != 2 && dim != 3) return fail(SP_E_INVALID_ARG, "dim must be 2 or 3");
    if (n < 0 || (n > 0 && !probs)) return fail(SP_E_INVALID_ARG, "bad problem array");
    if (n > 65535) return fail(SP_E_INVALID_ARG, "at most 65535 problems per batch");
    for (int i = 0; i < n; ++i) {
        sp_status st = check_problem(&probs[i], dim, prec);
        if (st != SP_OK) return st;
    }
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    if (n == 0) return SP_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dim == 2)
        return prec == SP_PREC_FP32C ? batch_impl<2, float>(ctx, probs, n, prec, s)
                                     : batch_impl<2, double>(ctx, probs, n, prec, s);
    return prec == SP_PREC_FP32C ? batch_impl<3, float>(ctx, probs, n, prec, s)
                                 : batch_impl<3, double>(ctx, probs, n, prec, s);
}

template <int D, typename T>
static sp_status vertex_density_impl(sp_ctx *ctx, const void *xyz, int64_t n_vert, const int32_t *simp, int64_t n,
                                     const void *mass, double m0, const sp_grid *box, void *rho, hipStream_t stream)
{
    HIPCHECK(hipSetDevice(ctx->device));
    if (n_vert == 0) return SP_OK;
    sp_status st = ensure_scratch(ctx, sizeof(double) * 2 * (size_t)n_vert, stream);
    if (st != SP_OK) return st;
    double *acc = reinterpret_cast<double *>(ctx->scratch);
    const size_t nacc = 2 * (size_t)n_vert;
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_blocks(nacc, 256)), dim3(256), 0, stream, acc, nacc);
    if (n > 0) {
        const double3 ext = make_double3(box->extent[0], box->extent[1], box->extent[2]);
        const int3 per = make_int3((box->flags & SP_PERIODIC_X) ? 1 : 0, (box->flags & SP_PERIODIC_Y) ? 1 : 0,
                                   (box->flags & SP_PERIODIC_Z) ? 1 : 0);
        hipLaunchKernelGGL((k_vd_accum<D, T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                           reinterpret_cast<const T *>(xyz), n_vert, simp, n, reinterpret_cast<const T *>(mass), m0,
                           ext, per, acc, ctx->es);
    }
    hipLaunchKernelGGL(k_vd_finish<T>, dim3((unsigned)((n_vert + 255) / 256)), dim3(256), 0, stream, acc, n_vert,
                       reinterpret_cast<T *>(rho));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SP_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return SP_OK;
}

extern "C" sp_status sp_vertex_density(sp_ctx *ctx, int dim, const void *xyz, int64_t n_vert, const int32_t *simplices,
                                       int64_t n_simplex, const void *mass, double mass_uniform, const sp_grid *box,
                                       void *rho_out, sp_precision prec, void *stream)
{
    if (dim != 2 && dim != 3) return fail(SP_E_INVALID_ARG, "dim must be 2 or 3");
    if (prec != SP_PREC_FP64 && prec != SP_PREC_FP32C) return fail(SP_E_INVALID_ARG, "unknown precision %d", (int)prec);
    if (n_vert < 0 || n_vert >= ((int64_t)1 << 31)) return fail(SP_E_INVALID_ARG, "n_vert %lld out of range", (long long)n_vert);
    if (n_simplex < 0 || n_simplex >= ((int64_t)1 << 31))
        return fail(SP_E_INVALID_ARG, "n_simplex %lld out of range", (long long)n_simplex);
    if (!box) return fail(SP_E_INVALID_ARG, "box is NULL");
    if (box->flags & ~(uint32_t)(SP_PERIODIC_X | SP_PERIODIC_Y | SP_PERIODIC_Z))
        return fail(SP_E_INVALID_ARG, "only the SP_PERIODIC_* flags apply to sp_vertex_density");
    for (int d = 0; d < dim; ++d) {
        if (((box->flags >> d) & 1u) && !(box->extent[d] > 0.0 && box->extent[d] < 1e300))
            return fail(SP_E_INVALID_ARG, "extent[%d] must be positive and finite on a periodic axis", d);
    }
    if (n_vert > 0 && (!xyz || !rho_out)) return fail(SP_E_INVALID_ARG, "xyz and rho_out must not be NULL");
    if (n_simplex > 0 && !simplices) return fail(SP_E_INVALID_ARG, "simplices must not be NULL");
    if (n_simplex > 0 && n_vert == 0) return fail(SP_E_INVALID_ARG, "simplices given without vertices");
    if (!mass && !(mass_uniform == mass_uniform && fabs(mass_uniform) < 1e300))
        return fail(SP_E_INVALID_ARG, "mass_uniform must be finite");
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dim == 3)
        return prec == SP_PREC_FP32C
                   ? vertex_density_impl<3, float>(ctx, xyz, n_vert, simplices, n_simplex, mass, mass_uniform, box, rho_out, s)
                   : vertex_density_impl<3, double>(ctx, xyz, n_vert, simplices, n_simplex, mass, mass_uniform, box, rho_out, s);
    return prec == SP_PREC_FP32C
               ? vertex_density_impl<2, float>(ctx, xyz, n_vert, simplices, n_simplex, mass, mass_uniform, box, rho_out, s)
               : vertex_density_impl<2, double>(ctx, xyz, n_vert, simplices, n_simplex, mass, mass_uniform, box, rho_out, s);
}

extern "C" sp_status sp_sync_status(sp_ctx *ctx, void *stream)
{
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
    ErrState e;
    HIPCHECK(hipMemcpy(&e, ctx->es, sizeof e, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemset(ctx->es, 0, sizeof e));
    if (e.first != 0) {
        return fail((sp_status)e.first,
                    "device errors: %d bad index, %d non-finite, %d periodic span, %d internal (%d overflow retries), "
                    "%d simplices too large for the corner sums",
                    e.n_bad_index, e.n_nonfinite, e.n_bad_span, e.n_internal, e.n_overflow, e.n_degenerate);
    }
    return SP_OK;
}

static void drop_events(sp_ctx *ctx)
{
    for (int k = 0; k <= ST_N; ++k) {
        auto &v = k < ST_N ? ctx->ev[k] : ctx->ev_call;
        for (auto &e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        v.clear();
    }
    ctx->prof_calls = 0;
}

extern "C" sp_status sp_profile_enable(sp_ctx *ctx, int on)
{
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
    if (on) {
        HIPCHECK(hipDeviceSynchronize());
        drop_events(ctx);
    }
    ctx->profiling = on < 0 ? 0 : (on > 2 ? 2 : on);
    return SP_OK;
}

extern "C" sp_status sp_profile_read(sp_ctx *ctx, sp_profile *out)
{
    if (!ctx || !out) return fail(SP_E_INVALID_ARG, "ctx or out is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipDeviceSynchronize());
    memset(out, 0, sizeof *out);
    double *dst[ST_N] = {&out->ms_fill, &out->ms_setup, &out->ms_bin, &out->ms_clip, &out->ms_clip_retry,
                         &out->ms_finalize};
    for (int k = 0; k <= ST_N; ++k) {
        auto &v = k < ST_N ? ctx->ev[k] : ctx->ev_call;
        double acc = 0.0;
        for (auto &e : v) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) acc += ms;
        }
        if (k < ST_N) *dst[k] = acc;
        else out->ms_call = acc;
    }
    out->calls = ctx->prof_calls;
    CallState cs;
    HIPCHECK(hipMemcpy(&cs, ctx->cs, sizeof cs, hipMemcpyDeviceToHost));
    out->pieces = (long long)cs.pieces;
    out->items = (long long)cs.total;
    out->clip_blocks = ctx->last_clip_blocks;
    drop_events(ctx);
    return SP_OK;
}

// Launch parameters the autotuner searches: the slab group (at most how
// many x-slabs one work item covers), the expected pieces a big simplex's
// work items are cut down to (0: from the launch size) and the clip blocks
// per CU (0: as many as fit).
static const int kTuneSlab[] = {1, 2, 4, 8, 16, 32, 64};
static const int kTuneItem[] = {0, 32, 128, 512, 2048};
static const int kTuneBlocks[] = {0, 4, 8};

// Signature of a tuning sample: what determines the best parameters, not
// where the buffers live.
static uint64_t sample_signature(int dim, const sp_problem *sample, int n, sp_precision prec, int num_cu)
{
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &dim, sizeof dim);
    h = fnv(h, &prec, sizeof prec);
    h = fnv(h, &num_cu, sizeof num_cu);
    for (int i = 0; i < n; ++i) {
        h = fnv(h, &sample[i].n_vert, sizeof sample[i].n_vert);
        h = fnv(h, &sample[i].n_simplex, sizeof sample[i].n_simplex);
        h = fnv(h, &sample[i].grid, sizeof sample[i].grid);
    }
    return h;
}

// The cache: one line per tuned sample, the last matching line wins.
// Version 1 lines (no item size) are read with the automatic item size.
static bool cache_lookup(const char *path, uint64_t sig, Tuning &t)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        unsigned long long k = 0;
        int g = 0, c = 0, ip = 0;
        const bool v2 = sscanf(line, "simproj-tune 2 sig=%llx slab_group=%d blocks_per_cu=%d item_pieces=%d", &k, &g,
                               &c, &ip) == 4;
        const bool v1 = !v2 && sscanf(line, "simproj-tune 1 sig=%llx slab_group=%d blocks_per_cu=%d", &k, &g, &c) == 3;
        if ((v1 || v2) && k == sig && g > 0 && g <= 4095 && c >= 0 && c <= 64 && ip >= 0 && ip <= 65536) {
            t.slab_group = g;
            t.chunks_per_cu = c;
            t.item_pieces = v2 ? ip : 0;
            found = true;
        }
    }
    fclose(f);
    return found;
}

extern "C" sp_status sp_autotune(sp_ctx *ctx, int dim, const sp_problem *sample, int n, sp_precision prec,
                                 const char *cache_path)
{
    if (dim != 2 && dim != 3) return fail(SP_E_INVALID_ARG, "dim must be 2 or 3");
    if (n <= 0 || !sample) return fail(SP_E_INVALID_ARG, "an autotuning sample needs at least one problem");
    for (int i = 0; i < n; ++i) {
        sp_status st = check_problem(&sample[i], dim, prec);
        if (st != SP_OK) return st;
    }
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
    const uint64_t sig = sample_signature(dim, sample, n, prec, ctx->num_cu);
    Tuning best = ctx->tune;
    if (cache_path && cache_lookup(cache_path, sig, best)) {
        ctx->tune = best;
        return SP_OK;
    }
    const int saved_prof = ctx->profiling;
    ctx->profiling = 0;
    hipStream_t s = ctx->cap_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    sp_status st = SP_OK;
    // one sample run: a single problem by itself, several as one batched
    // launch (the form they are tuned for)
    auto run = [&]() -> sp_status {
        if (n > 1) {
            if (dim == 3)
                return prec == SP_PREC_FP32C ? batch_impl<3, float>(ctx, sample, n, prec, s)
                                             : batch_impl<3, double>(ctx, sample, n, prec, s);
            return prec == SP_PREC_FP32C ? batch_impl<2, float>(ctx, sample, n, prec, s)
                                         : batch_impl<2, double>(ctx, sample, n, prec, s);
        }
        if (dim == 3)
            return prec == SP_PREC_FP32C ? project_impl<3, float>(ctx, sample, s) : project_impl<3, double>(ctx, sample, s);
        return prec == SP_PREC_FP32C ? project_impl<2, float>(ctx, sample, s) : project_impl<2, double>(ctx, sample, s);
    };
    // time of the current parameters: one warm-up run (it also captures a
    // batched launch), then the best of two
    auto timed = [&](float &ms) -> sp_status {
        ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, s);
            sp_status r = run();
            if (r != SP_OK) return r;
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(SP_E_DEVICE, "autotune run failed");
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep > 0 && t < ms) ms = t;
        }
        return SP_OK;
    };
    // coordinate descent from the current parameters: each parameter in turn
    // over its candidates with the others held, twice round
    float best_ms = 0.f;
    st = timed(best_ms);
    for (int pass = 0; pass < 2 && st == SP_OK; ++pass) {
        for (int which = 0; which < 3 && st == SP_OK; ++which) {
            const int *cand = which == 0 ? kTuneSlab : (which == 1 ? kTuneItem : kTuneBlocks);
            const int nc = which == 0 ? (int)(sizeof kTuneSlab / sizeof(int))
                                      : (which == 1 ? (int)(sizeof kTuneItem / sizeof(int))
                                                    : (int)(sizeof kTuneBlocks / sizeof(int)));
            for (int k = 0; k < nc && st == SP_OK; ++k) {
                Tuning t = best;
                int &field = which == 0 ? t.slab_group : (which == 1 ? t.item_pieces : t.chunks_per_cu);
                if (field == cand[k]) continue;
                field = cand[k];
                ctx->tune = t;
                float ms = 0.f;
                st = timed(ms);
                if (st == SP_OK && ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profiling = saved_prof;
    ctx->tune = best;
    if (st != SP_OK) return st;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (!f) return fail(SP_E_INVALID_ARG, "cannot write the tuning cache %s", cache_path);
        fprintf(f, "simproj-tune 2 sig=%llx slab_group=%d blocks_per_cu=%d item_pieces=%d ms=%.4f\n",
                (unsigned long long)sig, best.slab_group, best.chunks_per_cu, best.item_pieces, best_ms);
        fclose(f);
    }
    return SP_OK;
}

extern "C" sp_status sp_tuning_set(sp_ctx *ctx, int slab_group, int blocks_per_cu, int item_pieces)
{
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    if (slab_group < 1 || slab_group > 4095) return fail(SP_E_INVALID_ARG, "slab_group %d not in 1..4095", slab_group);
    if (blocks_per_cu < 0 || blocks_per_cu > 64)
        return fail(SP_E_INVALID_ARG, "blocks_per_cu %d not in 0..64", blocks_per_cu);
    if (item_pieces < 0 || item_pieces > 65536)
        return fail(SP_E_INVALID_ARG, "item_pieces %d not in 0..65536", item_pieces);
    ctx->tune.slab_group = slab_group;
    ctx->tune.chunks_per_cu = blocks_per_cu;
    ctx->tune.item_pieces = item_pieces;
    return SP_OK;
}

extern "C" sp_status sp_tuning_read(sp_ctx *ctx, int *slab_group, int *blocks_per_cu, int *item_pieces)
{
    if (!ctx) return fail(SP_E_INVALID_ARG, "ctx is NULL");
    if (slab_group) *slab_group = ctx->tune.slab_group;
    if (blocks_per_cu) *blocks_per_cu = ctx->tune.chunks_per_cu;
    if (item_pieces) *item_pieces = ctx->tune.item_pieces;
    return SP_OK;
}
