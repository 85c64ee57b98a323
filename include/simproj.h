/*
 * simproj.h -- exact projection of a piecewise-linear density defined on a
 * simplicial mesh onto a regular grid, on AMD Instinct MI355X (gfx950).
 *
 * Operation (Sousbie & Colombi, "ColDICE", Section 3.1, eq. eq_firstOrder and
 * the input/output statement of the exact-projection algorithm, Appendix D):
 * for every grid cell G_j
 *
 *     P_j = sum over simplices S_i of  integral over (S_i intersect G_j) of rho_i(x) dx,
 *
 * where rho_i is the linear interpolant of simplex i's D+1 vertex densities
 * (per vertex, or per corner with SP_RHO_PER_CORNER).  The output is the
 * density P_j / |G_j| (default) or the mass P_j (SP_OUT_MASS).  Simplices of
 * either orientation are accepted: each contributes rho integrated over the
 * region it covers.  Overlapping simplices (a multi-stream sheet) add up.
 *
 * Conventions.
 *   - Cell j = (i, j, k) covers [origin + i h, origin + (i+1) h) per axis,
 *     h = extent / dims; the output grid is C order [dims2][dims1][dims0]
 *     (x fastest), 2D [dims1][dims0].
 *   - Periodic axes: each simplex is unwrapped to the minimum image of its
 *     first vertex; its extent must be < extent/2 along that axis.
 *     Contributions on non-periodic axes outside [0, dims) are dropped.
 *   - A point exactly on a cell face belongs to the upper cell.  This only
 *     decides measure-zero sets; integrals do not depend on it.
 *   - Zero-volume simplices deposit nothing and are not errors.
 *
 * Precision.
 *   SP_PREC_FP64   positions, densities and output in double; clipping,
 *                  integration and accumulation in double.
 *   SP_PREC_FP32C  positions, densities and output in float; clipping and
 *                  integration in float on error-free cell-local
 *                  coordinates, per-cell compensated (hi, lo) accumulation;
 *                  double only for the orientation of near-degenerate
 *                  simplices, each simplex's density gradient (once per
 *                  work item) and its value at one point per piece, and the
 *                  total-mass reduction.
 *
 * Memory and streams.  Every data pointer in sp_problem is a DEVICE pointer
 * owned by the caller; the buffers must stay valid until the work enqueued
 * on `stream` (a hipStream_t, NULL for the default stream) has completed.
 * All projection calls are asynchronous: they validate their arguments on
 * the host, enqueue kernels and return.  On the device every simplex is
 * checked before it is cut: one with a vertex index outside [0, n_vert), a
 * non-finite position or density, an extent of half the box or more on a
 * periodic axis, or an extent of 32768 cells or more on any axis is skipped
 * (SP_E_PERIODIC_SPAN for both extent limits); with SP_VALIDATE the first
 * such error is reported by sp_sync_status.  The context owns its
 * scratch memory; a context must not be used by two host threads at once,
 * and calls on one context must be ordered (one stream, or synchronised).
 * Scratch grows in stream order on the call's stream (freed and allocated
 * behind the work already enqueued there, with no device-wide wait; only a
 * context holding captured batch launches waits for the device before it
 * drops them).  The environment variable SP_SCRATCH_CAP (bytes, with an
 * optional K, M or G suffix), read by sp_create, bounds the device memory a
 * context holds; a call that would need more returns SP_E_NO_MEMORY before
 * it enqueues anything, and the context stays usable.  Also read by
 * sp_create, each choosing a context's kernels or initial launch
 * parameters without changing results beyond rounding: SIMPROJ_SLAB_GROUP,
 * SIMPROJ_ITEM_PIECES, SIMPROJ_CLIP_BLOCKS_PER_CU (launch parameters, as
 * sp_tuning_set sets them), SIMPROJ_GROUP_CLIP=1 (FP32 3D clipping with one
 * polytope per 16 lanes) and SIMPROJ_TILED_DEPOSIT=1 (single FP32 3D
 * problems deposit through a per-wave cell tile in LDS, the per-thread
 * contribution buffers of Section 3.5; both measured slower than the
 * defaults).
 */
#ifndef SIMPROJ_H
#define SIMPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sp_ctx sp_ctx;

typedef enum {
    SP_OK = 0,
    SP_E_INVALID_ARG = 1,   /* null pointer, bad dims/sizes, unsupported flag */
    SP_E_OUT_OF_RANGE = 2,  /* (SP_VALIDATE) a vertex index outside [0, n_vert) */
    SP_E_NONFINITE = 3,     /* (SP_VALIDATE) a NaN/Inf position or density */
    SP_E_PERIODIC_SPAN = 4, /* (SP_VALIDATE) a simplex spans >= extent/2 on a periodic axis,
                               or 32768 cells or more on any axis */
    SP_E_NO_MEMORY = 5,     /* scratch allocation failed, or SP_SCRATCH_CAP exceeded */
    SP_E_DEVICE = 6,        /* no usable HIP device, or a HIP call failed */
    SP_E_UNSUPPORTED = 7,   /* valid request this build does not handle */
    SP_E_INTERNAL = 8       /* a polytope exceeded every capacity (should not happen) */
} sp_status;

typedef enum { SP_PREC_FP64 = 0, SP_PREC_FP32C = 1 } sp_precision;

enum {
    SP_PERIODIC_X = 1u,
    SP_PERIODIC_Y = 2u,
    SP_PERIODIC_Z = 4u,
    SP_RHO_PER_CORNER = 8u, /* rho is [n_simplex][D+1] instead of [n_vert]          */
    SP_OUT_MASS = 16u,      /* write mass per cell instead of density                 */
    SP_ACCUMULATE = 32u,    /* add into out (and out_lo) instead of overwriting them  */
    SP_VALIDATE = 64u       /* report skipped (invalid) simplices via sp_sync_status  */
};

/* Grid: cell (i,j,k) covers origin + [i,i+1)*h ... with h = extent/dims.
 * 2D problems use entries [0] and [1] only.  1 <= dims[d] <= 2^20, at most
 * 2^35 cells in all (cell indices are 64-bit); extent[d] > 0 and finite. */
typedef struct {
    double origin[3];
    double extent[3];
    int32_t dims[3];
    uint32_t flags;
} sp_grid;

typedef struct {
    const void *xyz;           /* [n_vert][D], double (FP64) or float (FP32C)              */
    int64_t n_vert;            /* 0 <= n_vert < 2^31                                        */
    const int32_t *simplices;  /* [n_simplex][D+1] vertex indices                           */
    int64_t n_simplex;         /* 0 <= n_simplex < 2^31                                     */
    const void *rho;           /* [n_vert], or [n_simplex][D+1] with SP_RHO_PER_CORNER      */
    sp_grid grid;
    void *out;                 /* grid, double (FP64) or float (FP32C)                      */
    float *out_lo;             /* FP32C only, optional: low part of the compensated sum;
                                  when given, out holds the high part and out + out_lo is
                                  the result; when NULL, out receives the rounded sum      */
    double *total_mass;        /* optional device double, overwritten with the FP64 sum
                                  over all cells of the output grid, in mass units        */
} sp_problem;

/* Create a context on HIP device `hip_device`.  SP_E_DEVICE when the device
 * does not exist or is not gfx950.  *ctx is NULL on failure. */
sp_status sp_create(int hip_device, sp_ctx **ctx);

/* Release the context and its scratch memory (waits for its device to be
 * idle first).  NULL is accepted. */
void sp_destroy(sp_ctx *ctx);

/* Project tetrahedra (D = 3).  Section 3, eq. eq_firstOrder; the hot path of
 * Appendix D's algorithm (the per-simplex single-voxel shortcut of its first
 * step included).  Host-detectable argument errors return synchronously and
 * enqueue nothing. */
sp_status sp_project_tets(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream);

/* sp_project_tets for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation, arguments, results and errors, but the
 * call allocates nothing -- no hipMalloc, hipFree or allocating library
 * routine, and no HIP events (stage profiling does not record it).  Its work
 * lists live in a static scratch array of 128 MiB in device memory, one copy
 * per GPU the library runs on, held from the first sp_create on that device
 * until the process ends.  A problem whose work lists do not fit returns
 * SP_E_NO_MEMORY synchronously and enqueues nothing; roughly, 136 bytes per
 * simplex (work lists and its set-up record) plus, when out_lo is NULL in
 * FP32C mode, 4 bytes per cell, on top of 26 MiB of fixed lists (about 780K
 * tetrahedra with a caller-held out_lo).
 * Every call on one GPU shares that GPU's array, and a call leaves its
 * contents behind: each call writes everything it reads before reading it,
 * but calls whose work overlaps in time on one GPU (different streams or
 * contexts, unsynchronised) race on it and must not be issued. */
sp_status sp_project_tets_noalloc(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream);

/* Project triangles (D = 2): the same operation in two dimensions (the
 * paper's 2D, i.e. 4D phase-space, case; Section 3.1 eq. eq:E02D). */
sp_status sp_project_tris(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, void *stream);

/* Accuracy-controlled projection of tetrahedra (Section 3.4, eq. eq_accuracy
 * and eq_accuracy2, and the per-voxel control the paper describes after its
 * Table 1).  The problem is projected in FP32C while the largest |contribution|
 * C_max of every cell is recorded; a cell whose sum P satisfies
 *     |P| < C_max * 2^(wrong_bits + accurate_bits - 23)
 * may have fewer than `accurate_bits` correct bits when each FP32
 * contribution has up to `wrong_bits` wrong trailing bits of its 23.  Those
 * cells are flagged, every simplex whose bounding box holds a flagged cell is
 * projected again in FP64, and the FP64 sums replace the flagged cells (as
 * out + out_lo when the caller keeps out_lo).  With non-negative densities
 * P >= C_max and nothing is flagged; the control matters where signed
 * densities cancel.
 *   prob           as for sp_project_tets with SP_PREC_FP32C; SP_ACCUMULATE is
 *                  rejected (SP_E_INVALID_ARG)
 *   accurate_bits  1..40;  wrong_bits  0..23 (the paper's W)
 *   counts         optional HOST int64[2]: flagged cells, re-projected simplices
 * Synchronises with `stream` once (after flagging, to size the FP64 pass);
 * uses context-owned buffers of about 19 bytes per cell plus, when cells are
 * flagged, 24 bytes per vertex and 48 per re-projected simplex. */
sp_status sp_project_tets_accurate(sp_ctx *ctx, const sp_problem *prob, int accurate_bits, int wrong_bits,
                                   int64_t *counts, void *stream);

/* Projection of tetrahedra onto an adaptive grid, gathered onto the uniform
 * grid by donor cell (Section 4, "Calculation of the acceleration").  The
 * adaptive grid is an octree over the caller's grid, refined region by
 * region as long as its cells are larger than the smallest height of any
 * tetrahedron intersecting them, down to the caller's cells at most: a block
 * of side 2^l cells stays whole only if every tetrahedron meeting its
 * interior has smallest height h >= 2^l (h = 3 V / largest face area, in
 * cells, after the minimum-image unwrap, FP64; "meeting" decided by a
 * separating axis test in FP64).  The density is projected exactly onto the
 * leaves, and each leaf's mass is spread evenly over the cells it holds.
 * The result is the exact projection wherever the leaves are single cells
 * (around thin simplices) and a block average elsewhere (inside large ones).
 * Each tetrahedron is projected at the coarsest level at which no block of
 * its bounding box is refined, so large simplices away from thin ones cost
 * pieces at their own resolution.
 *   prob          as for sp_project_tets (SP_ACCUMULATE rejected; a given
 *                 out_lo is zeroed, out holds the whole result)
 *   max_level     0..10; every dims[d] must be a multiple of 2^max_level
 *                 (max_level 0 is sp_project_tets)
 *   level_counts  optional HOST int64[max_level + 1]: simplices projected at
 *                 each level
 * A tetrahedron whose bounding box holds more than 2^22 blocks of the size
 * it is tested against marks them all without the test (a finer grid there).
 * Synchronises with `stream` once (to size the levels); the levels are
 * projected in one batched launch (sp_project_batch). */
sp_status sp_project_tets_amr(sp_ctx *ctx, const sp_problem *prob, sp_precision prec, int max_level,
                              int64_t *level_counts, void *stream);

/* Projection of tetrahedra by first-order corner sums, FP64 (Section 3.1,
 * eq. eq_firstOrder with the corner terms of eq. eq:E03D and eq:E13D;
 * Appendix D's four kinds of vertex of a simplex-cell intersection: simplex
 * corners, edge-face crossings, facet-edge crossings, grid points inside the
 * simplex).  Every vertex of every piece adds its terms to its cell; no
 * piece is built.  The same result as sp_project_tets in FP64 mode, by the
 * paper's own formulation, for comparison of speed and accuracy; the terms
 * are signed and cancel within a cell (tested to 1e-12 of the cell's
 * coverage scale and of the total, degenerate meshes included).
 *   prob   as for sp_project_tets, with xyz, rho and out in double
 * Degenerate positions with respect to the grid (corners on grid planes,
 * lines or points, edges or facets through grid lines or points, as on
 * lattice-aligned meshes and FP32 inputs) are resolved by simulation of
 * simplicity (Section 3.3, eq. eq_sos; App. E.1 and E.3): the grid is
 * perturbed symbolically and each predicate that is exactly zero takes the
 * sign of its first non-zero perturbation term.  Predicates are filtered:
 * FP64 decides unless its value is within its rounding bound, then a
 * double-double evaluation on the exact differences decides or declares
 * the tie (exact for inputs with up to about 26 significant bits in cell
 * units).  A simplex whose bounding box holds more than 2^24 cells is
 * skipped and reported by sp_sync_status as SP_E_UNSUPPORTED (one thread
 * enumerates its cells). */
sp_status sp_project_tets_corners(sp_ctx *ctx, const sp_problem *prob, void *stream);

/* sp_project_tets_corners with the fused facet contributions of Appendix D
 * (eq. eq_contribFused and eq_diffRho): where two summed simplices share a
 * facet (the same three vertex indices), each term one of them contributes
 * at a vertex of its piece in a cell, with an edge on that facet, has a
 * twin from the other simplex that differs only in the sign of the facet
 * normal (or not at all, when a fold puts both simplices on one side), so
 * the pair is summed once, by the simplex of lower index, with the
 * difference (or sum) of the two density functions.  The pieces of such
 * simplices take the cell centre as their common origin.  Facets are matched
 * on the device by their vertex indices (a hash table in the context's
 * scratch, 76 to 108 bytes per simplex); a facet met by more than two
 * simplices is paired once and its other simplices sum it alone.  The same
 * result as sp_project_tets_corners up to rounding (tested to 1e-12 of each
 * cell's coverage scale); n_simplex below 2^30 (else SP_E_INVALID_ARG).
 * Asynchronous on `stream`. */
sp_status sp_project_tets_corners_fused(sp_ctx *ctx, const sp_problem *prob, void *stream);

/* Project n independent problems of dimension `dim` (2 or 3; 1 <= n <=
 * 65535, n == 0 is a no-op) in one persistent, work-stealing
 * launch; `probs` is a HOST array of n problems whose buffers are device
 * pointers, each problem as in sp_project_tets / sp_project_tris (flags, out_lo and
 * total_mass per problem; their output grids must not overlap).  The work
 * items of all problems are ordered by estimated cost in one list, so the
 * load is balanced across problems (the cost-based balancing the paper
 * proposes for its future work, Section 7).  The launch sequence is captured
 * once per signature (the sp_problem bytes, precision, tuning and scratch
 * buffer) into a HIP graph and replayed on `stream` by later calls with the
 * same signature; the context keeps at most 16 such graphs.  The first call
 * of a signature synchronises with the device (graph capture, descriptor
 * upload); the others only enqueue.  Stage times of sp_profile are not
 * split for batches (ms_call only). */
sp_status sp_project_batch(sp_ctx *ctx, int dim, const sp_problem *probs, int n, sp_precision prec, void *stream);

/* Per-vertex density of a simplicial mesh from the simplex masses: for each
 * vertex j, rho_j = (sum of M_i) / (sum of |V_i|) over the simplices i
 * incident to j, |V_i| the unsigned volume (area in 2D) of simplex i in box
 * units after minimum-image unwrapping on the periodic axes (Section 4,
 * "Calculation of the acceleration": the estimate that turns simplex masses
 * into the vertex densities the projection interpolates).
 *   xyz        device [n_vert][dim], double (SP_PREC_FP64) or float (SP_PREC_FP32C)
 *   simplices  device [n_simplex][dim+1] int32 vertex indices
 *   mass       device [n_simplex] masses, same type as xyz; or NULL, then every
 *              simplex has mass `mass_uniform`
 *   box        host; only extent[] and the SP_PERIODIC_* flags are used (other
 *              flags: SP_E_INVALID_ARG)
 *   rho_out    device [n_vert], same type as xyz; vertices without a simplex of
 *              non-zero volume get 0
 * Sums and the division are in FP64 in both precisions (the FP32C result is
 * the correctly rounded FP64 value up to summation order).  Simplices with an
 * index out of range or a non-finite coordinate or mass are skipped and
 * reported by sp_sync_status.  Uses the context's scratch (16 bytes per
 * vertex); asynchronous on `stream`. */
sp_status sp_vertex_density(sp_ctx *ctx, int dim, const void *xyz, int64_t n_vert, const int32_t *simplices,
                            int64_t n_simplex, const void *mass, double mass_uniform, const sp_grid *box,
                            void *rho_out, sp_precision prec, void *stream);

/* Wait for `stream`, then report the first device-side error recorded since
 * the previous call (SP_VALIDATE checks, capacity failures) and clear it. */
sp_status sp_sync_status(sp_ctx *ctx, void *stream);

/* Time the tunable launch parameters (the x-slab group of a work item, the
 * expected pieces a big simplex's work items are cut down to, and the clip
 * blocks per CU) on the n sample problems of dimension `dim` and keep the
 * fastest for subsequent calls of this context (the cost-based balancing of
 * the work items, Section 7).  The sample is timed in the form it is tuned
 * for: one problem by itself, several as one sp_project_batch launch.
 * Search: coordinate descent from the parameters in use, each parameter in
 * turn over its candidates with the others held, twice round; every
 * candidate is run once to warm up and then timed twice with HIP events.
 * The sample's output grids are overwritten.  When cache_path is not NULL
 * the text file is searched first for a line with the sample's signature
 * (its sizes, grid descriptions, precision and CU count, not its pointers);
 * if found, its parameters are applied without timing, else the result is
 * appended to the file (SP_E_INVALID_ARG if it cannot be written; the
 * result is applied anyway).  Synchronous. */
sp_status sp_autotune(sp_ctx *ctx, int dim, const sp_problem *sample, int n, sp_precision prec,
                      const char *cache_path);

/* The launch parameters in use: the most x-slabs per work item, clip blocks
 * per CU (0: as many as fit on a CU) and the expected pieces per work item
 * of a big simplex (0: about one lane's share of the launch's pieces).  Any
 * pointer may be NULL.  (A big simplex is cut into work items of fewer
 * slabs, each of about that many expected pieces; the slab group caps it.) */
sp_status sp_tuning_read(sp_ctx *ctx, int *slab_group, int *blocks_per_cu, int *item_pieces);

/* Set the launch parameters by hand (slab_group in 1..4095, blocks_per_cu
 * in 0..64, item_pieces in 0..65536, else SP_E_INVALID_ARG); they hold for
 * later calls of this context until changed or retuned.  Results do not
 * depend on them. */
sp_status sp_tuning_set(sp_ctx *ctx, int slab_group, int blocks_per_cu, int item_pieces);

/* Per-stage device times of the projection calls made while profiling is
 * on, from HIP events recorded on each call's own stream around its kernels
 * (the tracing hook of this library; it adds no synchronisation to the
 * calls themselves). */
typedef struct {
    int calls;               /* projection calls recorded                          */
    double ms_call;          /* first kernel start to last kernel end, summed       */
    double ms_fill;          /* zeroing of the output and state                     */
    double ms_setup;         /* set-up, single-cell deposits, class histogram       */
    double ms_bin;           /* class offsets and scatter of the work items         */
    double ms_clip;          /* clip-integrate-deposit over all work items          */
    double ms_clip_retry;    /* items resumed with larger polytopes                 */
    double ms_finalize;      /* hi+lo merge and total-mass reduction                */
    long long pieces;        /* pieces deposited by the last call (mode 2 only);    */
                             /* for the corner sums, the grid deposits (one per    */
                             /* piece vertex and cell)                             */
    long long items;         /* work items of the last call                         */
    int clip_blocks;         /* persistent blocks of the last call's clip launch    */
} sp_profile;

/* on = 0: off; 1: record stage times; 2: also count the pieces deposited
 * (one extra atomic per work item, so keep it out of timed runs).  Turning
 * recording on clears what was recorded before.  Applies to the calls that
 * follow. */
sp_status sp_profile_enable(sp_ctx *ctx, int on);

/* Wait for the device, then return the times accumulated since profiling
 * was enabled and clear them. */
sp_status sp_profile_read(sp_ctx *ctx, sp_profile *out);

/* Message describing the last error returned on this thread. */
const char *sp_last_error(const sp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SIMPROJ_H */
