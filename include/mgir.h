/*
 * mgir.h - C ABI of the MI355X (gfx950) mixed-precision geometric-multigrid /
 * iterative-refinement Poisson solver.
 *
 * Method: Oo & Vogel, "Accelerating Geometric Multigrid Preconditioning with
 * Half-Precision Arithmetic on GPUs" (arXiv 2007.07539).  The outer solver is
 * iterative refinement with residuum scaling (Algorithm 2, Section 4.3) in
 * FP64; its correction equation is approximated by one multigrid V-cycle
 * (Algorithm 1 applied recursively, Section 4.2) whose levels store vectors in
 * FP64, FP32, FP16 or BF16 (the per-level precision variants of Table 2 and
 * Section 6).
 *
 * Problem: -Laplace(u) = f on the unit square (dim = 2) or cube (dim = 3) with
 * u = 0 on the boundary (Section 5), discretised by the 5-/7-point finite-
 * difference stencil on n^dim interior points, n = 2^m - 1, h = 1/(n+1):
 *     (A u)_i = (2 dim u_i - sum of face neighbours) / h^2.
 * The hierarchy coarsens by two per dimension down to one interior point,
 * where the base-level solve is exact.
 *
 * Conventions for every function below:
 *   - Every function returns an mg_status_t; no C++ exception crosses the ABI.
 *     On error, mg_last_error() returns a thread-local message.
 *   - Validation errors (MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_PREC,
 *     MG_ERR_WORKSPACE, MG_ERR_STATE) leave the handle unchanged.
 *   - "device" pointers are HIP device memory of the GPU that was current at
 *     mg_setup; the caller owns them and all workspace memory.  The library
 *     owns only the handle and what hangs off it (plan, HIP graph, a small
 *     pinned host buffer for the residual norms).
 *   - Dense arrays at the ABI are n^dim values, x fastest:
 *     index (z*n + y)*n + x in 3-D, y*n + x in 2-D.
 *   - stream is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued on that stream; see each function for synchronisation.
 */
#ifndef MGIR_H
#define MGIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_ERR_ARG = -1,            /* null pointer, out-of-range option or index */
    MG_ERR_SHAPE = -2,          /* n not of an accepted form, dim not 2 or 3, base level too large */
    MG_ERR_PREC = -3,           /* unknown precision code in a level map */
    MG_ERR_WORKSPACE = -4,      /* no workspace bound, or bound one too small / misaligned */
    MG_ERR_HIP = -5,            /* a HIP runtime call failed (message in mg_last_error) */
    MG_ERR_NOT_CONVERGED = -6,  /* max_iter reached; u holds the last iterate, stats filled */
    MG_ERR_NONFINITE = -7,      /* a residual norm became NaN or Inf */
    MG_ERR_STATE = -8           /* call not valid in the handle's current state */
} mg_status_t;

/* Storage format of one level's vectors.  FP16/BF16/FP32 levels accumulate in
 * FP32 registers, FP64 levels in FP64; every store rounds to nearest even. */
typedef enum { MG_F64 = 0, MG_F32 = 1, MG_F16 = 2, MG_BF16 = 3 } mg_prec_t;

/* Discretisation of -Laplace(u) = f with zero boundary values (Section 5).
 * MG_DISC_FD: the (2D+1)-point finite-difference stencil, A = L / h^2 with
 *   L = [2D centre, -1 face neighbours]; b holds f at the interior nodes.
 * MG_DISC_Q1: bilinear (2-D) / trilinear (3-D) finite elements, the
 *   discretisation of the paper's measurements: A_ij = integral of
 *   grad(phi_i) . grad(phi_j), the 9-point stencil [8, -1 (8x)] / 3 in 2-D
 *   and h [32, 0 (faces), -2 (edges), -1 (corners)] / 12 in 3-D; b is the
 *   load vector (integral of f phi_i; h^dim f_i when the mass is lumped).
 *   Restriction is P^T and the coarse operators are the Q1 matrices of the
 *   coarser meshes (= the Galerkin products P^T A P). */
typedef enum { MG_DISC_FD = 0, MG_DISC_Q1 = 1 } mg_disc_t;

typedef struct {
    int nu1;                 /* pre-smoothing sweeps (Algorithm 1), default 2 */
    int nu2;                 /* post-smoothing sweeps (Algorithm 1), default 2 */
    double omega;            /* damped-Jacobi weight, default 0.8 */
    int residual_scaling;    /* 1: alpha = 2^j ||r||_inf before the cast (Algorithm 2; the
                                scaled residual has max-norm 2^-j).  j = 0 unless an FP16
                                level's correction could leave FP16's range: in grid-
                                scaled units the correction of a right-hand side of
                                max-norm one on a level of n points per dimension is
                                below K (n+1)^2 (K = 0.074 in 2-D, 0.058 in 3-D, above
                                the torsion-function maximum), and j is the least power that
                                brings that bound under 2^14 on every FP16 level (see
                                mg_alpha_shift; 2-D n >= 511, 3-D n = 1023).
                                0: alpha = 1 (the FP64 baseline omits scaling, Section 6) */
    int max_iter;            /* refinement steps at most, default 100 */
    double rtol;             /* stop when ||r||_2 <= rtol * ||b||_2 (FP64), default 1e-10 */
    int use_initial_guess;   /* 0: ir_solve starts from u = 0 (default); 1: from the given u */
    int use_graph;           /* 1: replay one captured HIP graph per refinement step (default) */
    int autotune;            /* 1: time launch shapes at mg_bind_workspace (synchronises).
                                When the environment variable MGIR_TUNE_CACHE names a
                                file, the chosen shapes are appended to it under a key
                                of device architecture, CU count, grid, level formats
                                and the kernel-changing options, and a later handle of
                                the same key reads them back instead of timing. */
    int rescale_half;        /* 1: every restriction into an FP16 or BF16 level keeps the
                                restricted residual t in the finer level's accumulator
                                format, takes s = max|t| and stores round(t / s); the
                                coarse correction is multiplied by s before it is
                                prolongated (the DSH_MG residuum scaling, Section 6).
                                Default 0.  Single-grid handles only: mg_setup_batched
                                and mg_setup_multi reject it with MG_ERR_ARG. */
    int cycles_per_step;     /* V-cycles per refinement step, 1..16 (default 1, Algorithm 2).
                                Each further cycle continues from the correction so far
                                (nu1 sweeps from it, then the usual cycle) on the same
                                scaled residual, before u and r are updated once (the
                                inner iteration the paper's conclusion points to).
                                ir_solve then counts steps in max_iter and iterations.
                                Single-grid handles only, as rescale_half. */
    double base_tol;         /* base level of more than one point (nlevels < m): CG until
                                ||b - L x||_2 <= base_tol ||b||_2 (default 1e-4, the
                                paper's bound for residuals scaled to norm one,
                                Section 4.2) */
    int base_max_iter;       /* ... at most this many CG steps; 0: min(10000, base points) */
    int discretization;      /* an mg_disc_t, default MG_DISC_FD.  MG_DISC_Q1 runs its own
                                kernels (no fused forms; the launch shapes are those of
                                the LDS-staged 3-D kernels, see "Q1 handles" under
                                mg_set_shape); single-grid handles only, as rescale_half. */
    int defer_update;        /* 0 (default): ir_solve adds alpha c to u in every step, as
                                Algorithm 2 writes it.  k in 1..64: the step's update
                                kernel (3-D finite differences with the fused last
                                sweep + update, MG_SHAPE_FUSE in use; or the Q1 update,
                                2-D and 3-D) stores c in the finest level's
                                format in a ring of k slots instead of reading and
                                writing the FP64 u; when the ring is full, and before
                                u is read (the recomputed residual, the return), one
                                pass adds the stored alpha_j c_j to u in step order.
                                u is bit for bit the same, since the same roundings
                                happen in the same sequence; the refinement loop itself
                                only needs r.  The workspace grows by k finest-level
                                vectors of that format.  Pays where the format is
                                narrower than FP64 (FP16: 2 instead of 16 bytes per
                                point and step).  Single-grid handles only. */
} mg_options_t;

typedef struct {
    int iterations;          /* refinement steps applied (V-cycles when cycles_per_step = 1) */
    double rel_residual;     /* ||b - A u||_2 / ||b||_2 of the returned u, recomputed in FP64 */
    double seconds;          /* host wall time of the call, to the final synchronisation */
    double *history;         /* optional caller-owned host array: ||r_k||_2/||b||_2, k = 0.. */
    int history_cap;         /* its capacity; entries beyond it are dropped */
} mg_stats_t;

typedef struct mg_ctx *mg_handle;

/* Fill *opt with the defaults listed above. */
void mg_default_options(mg_options_t *opt);

/* Create a solver for one grid.
 *   dim        2 or 3.
 *   n          interior points per dimension, n <= 1023 in 3-D.
 *              MG_DISC_FD: n = 2^m - 1 with m >= 2 (n <= 4095 in 2-D).
 *              MG_DISC_Q1: any odd n >= 3 (n <= 8191 in 2-D), in particular
 *              the paper's c 2^k - 1 with odd c
 *              (meshes of 193^3 .. 289^3 and 4097^2 .. 6145^2 vertices,
 *              Section 6).
 *   nlevels    0 for the full hierarchy n, (n-1)/2, ... while the size is odd
 *              and above 1: m levels, ending on one point (solved exactly)
 *              for n = 2^m - 1, otherwise on c - 1 points per dimension
 *              (solved by CG); 2..m for the first nlevels of it, whose last
 *              level is solved by CG (Section 4.2; opt.base_tol,
 *              opt.base_max_iter).  A CG base level runs in one workgroup and
 *              may hold at most 262144 points (MG_ERR_SHAPE beyond).
 *   level_prec one entry per level used, FINEST FIRST: level_prec[0] is the
 *              finest grid (the paper's level L), the last entry the base
 *              level (the paper's level 0).  NULL means all MG_F64.
 *   opt        NULL for defaults.
 * No device memory is allocated: query mg_workspace_size, allocate, then
 * mg_bind_workspace.  Errors: MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_PREC. */
mg_status_t mg_setup(mg_handle *out, int dim, int n, int nlevels, const mg_prec_t *level_prec,
                     const mg_options_t *opt);

/* Bytes of device workspace the handle needs (all levels' right-hand side and
 * correction vectors in their storage formats, the FP64 solution and residual
 * of the finest level, reduction partials). */
mg_status_t mg_workspace_size(mg_handle h, size_t *bytes);

/* Bind caller-owned device memory (at least mg_workspace_size bytes, 256-byte
 * aligned).  Zero-fills it on stream and waits for that; with opt.autotune it
 * also times launch shapes.  May be called again with another buffer; the
 * previous one is no longer referenced afterwards. */
mg_status_t mg_bind_workspace(mg_handle h, void *dev_ptr, size_t bytes, void *stream);

/* One V-cycle from a zero initial guess for A_L e = b (Algorithm 1, recursive).
 *   b  device, dense, n^dim values in level_prec[0]'s format (FP16/BF16 as
 *      IEEE binary16 / bfloat16 bit patterns).
 *   c  device, dense, n^dim values in the same format; receives the
 *      correction in grid-scaled units c = e / h^2 (so the physical
 *      correction is h^2 c; this keeps FP16 values away from underflow).
 * Asynchronous on stream.  Errors: MG_ERR_ARG, MG_ERR_WORKSPACE, MG_ERR_HIP. */
mg_status_t mg_vcycle(mg_handle h, const void *b, void *c, void *stream);

/* mg_vcycle for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same V-cycle, with the level vectors in a 128 MiB array the library holds on
 * each GPU (a file-scope device array, held until the process ends) instead of
 * the bound workspace, which this call neither needs nor touches.  128 MiB
 * holds the V-cycle of a 255^3 FP16 or a 127^3 FP64 hierarchy.  The handle
 * comes from mg_setup (which allocates no device memory); nothing is
 * allocated and nothing synchronises.  Every call on a GPU shares that GPU's
 * array and clears the part it uses first, so calls that overlap on one GPU
 * (other streams, other threads) race; serialise them.
 *   b, c  as for mg_vcycle; the result is bit for bit mg_vcycle's.
 * Errors: MG_ERR_ARG, MG_ERR_STATE (batched or many-right-hand-side handle),
 * MG_ERR_WORKSPACE (the handle's V-cycle needs more than 128 MiB), MG_ERR_HIP. */
mg_status_t mg_vcycle_noalloc(mg_handle h, const void *b, void *c, void *stream);

/* Solve A u = b by iterative refinement with residuum scaling (Algorithm 2):
 * r = b - A u;  while ||r||_2 > rtol ||b||_2:  alpha = ||r||_inf (or 1);
 * c = V-cycle(r / alpha) in the level formats;  u += alpha c;  r -= alpha A c.
 * Residual, update, norms and the stop test are FP64.  The recursively
 * updated residual of Algorithm 2 drives the loop; before returning,
 * b - A u is recomputed from scratch and iteration continues if it does not
 * meet the tolerance.
 *   b  device, dense FP64, n^dim.
 *   u  device, dense FP64, n^dim; input guess if opt.use_initial_guess,
 *      output solution (also on MG_ERR_NOT_CONVERGED: the last iterate).
 *   stats may be NULL.
 * b == 0 returns MG_OK with u = 0 and 0 iterations.  Synchronises stream once
 * per iteration (the 32-byte norm readback).  Errors: MG_ERR_ARG,
 * MG_ERR_WORKSPACE, MG_ERR_HIP, MG_ERR_NOT_CONVERGED, MG_ERR_NONFINITE. */
mg_status_t ir_solve(mg_handle h, const double *b, double *u, mg_stats_t *stats, void *stream);

/* ---- Batched instances ----------------------------------------------------
 * Many independent 3-D problems of different sizes solved together with the
 * method of Algorithms 1 and 2 (the paper solves one grid at a time; the
 * batch is an extension).  Stages are aligned from the finest level down:
 * stage d is ONE kernel launch over level d of every instance that has it,
 * so the small coarse grids of all instances share launches instead of each
 * costing a launch per level.
 *
 * Create a batched solver.
 *   ninst      1..4096 instances.
 *   n          ninst sizes, each 2^m - 1 with 2 <= m <= 10.
 *   level_prec Lmax entries (Lmax = the largest m), FINEST FIRST: instance i
 *              with m_i levels stores its level l < m_i - 1 in level_prec[l]
 *              and its one-point base level in level_prec[Lmax - 1] -- the
 *              same map a single-grid solver gets from level_prec[0..m_i-2]
 *              followed by level_prec[Lmax-1].  NULL means all MG_F64.
 *   opt        NULL for defaults; needs nu1 >= 2.  use_graph captures one
 *              refinement step of the whole batch; autotune times launch
 *              shapes per class of levels (pitch and format) at
 *              mg_bind_workspace, whole batched steps at a time (cached as
 *              for mg_setup under MGIR_TUNE_CACHE).
 * Each instance computes bit for bit what a single-grid solver with its size
 * and map computes.  Workspace as for mg_setup (mg_workspace_size,
 * mg_bind_workspace).  The single-grid calls (mg_vcycle, ir_solve, stage and
 * shape access) refuse a batched handle with MG_ERR_STATE.
 * Errors: MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_PREC. */
mg_status_t mg_setup_batched(mg_handle *out, int dim, int ninst, const int *n, const mg_prec_t *level_prec,
                             const mg_options_t *opt);

/* Algorithm 2 for every instance of a batched handle: the iteration of
 * ir_solve with per-instance alpha, norms, stop test and confirmation;
 * converged instances drop out of the following launches.
 *   b      host array of ninst device pointers, b[i] dense FP64 n_i^3.
 *   u      host array of ninst device pointers, u[i] dense FP64 n_i^3
 *          (input guess with opt.use_initial_guess; output as in ir_solve).
 *   stats  NULL or ninst entries; history of each entry as in ir_solve;
 *          seconds is the wall time of the whole batch.
 * Returns MG_OK when every instance converged, else the first failing
 * instance's status (every instance's u and stats are still written).
 * Synchronises stream once per refinement step. */
mg_status_t ir_solve_batched(mg_handle h, const double *const *b, double *const *u, mg_stats_t *stats,
                             void *stream);

/* Number of instances of a handle (1 for a single-grid handle). */
mg_status_t mg_instances(mg_handle h, int *ninst);

/* ---- Many right-hand sides -------------------------------------------------
 * nrhs Poisson problems on one 3-D grid (same operator, different b), stored
 * interleaved: value k of grid point (x, y, z) (0-based) at
 * ((z*n + y)*n + x)*nrhs + k.  One kernel launch per V-cycle stage serves all
 * right-hand sides; each one runs Algorithm 2 on its own (its own alpha_k,
 * norms, stop test and confirmation), and column k computes what a
 * single-grid solve of that right-hand side computes.  (The paper solves one
 * right-hand side at a time; the interleaved batch is an extension.)
 *
 * Create a solver.
 *   dim        3.
 *   n          2^m - 1 with 2 <= m <= 9.
 *   nrhs       4, 8, 16, 32 or 64, and at least 8 when any level is stored
 *              in FP32, FP16 or BF16 (a thread handles 8 such columns).
 *   level_prec m formats, finest first, as for mg_setup.
 *   opt        NULL for defaults; needs nu1 >= 2; autotune times the planes
 *              per thread of each level's stages at mg_bind_workspace, whole
 *              steps at a time (cached under MGIR_TUNE_CACHE).
 * Errors: MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_PREC.  Workspace as for mg_setup;
 * single-grid calls other than mg_levels / mg_level_n refuse the handle with
 * MG_ERR_STATE. */
mg_status_t mg_setup_multi(mg_handle *out, int dim, int n, int nrhs, const mg_prec_t *level_prec,
                           const mg_options_t *opt);

/* Algorithm 2 for every right-hand side of a handle from mg_setup_multi.
 *   b      device, FP64, n^3 * nrhs values, interleaved as above.
 *   u      device, same layout; the guess with opt.use_initial_guess, and the
 *          result on return.  A right-hand side that is zero gets u = 0; one
 *          with a non-finite value keeps its guess (0 without one).
 *   stats  NULL or nrhs entries, as for ir_solve (seconds: whole call).
 * Returns MG_OK when every column converged, else the first failing
 * column's status.  Synchronises stream once per refinement step. */
mg_status_t ir_solve_multi(mg_handle h, const double *b, double *u, mg_stats_t *stats, void *stream);

/* Number of right-hand sides of a handle (1 unless from mg_setup_multi). */
mg_status_t mg_rhs_count(mg_handle h, int *nrhs);

/* The exponent j of alpha = 2^j ||r||_inf (see residual_scaling) that instance
 * `instance` of the handle uses (0 for single-grid and many-right-hand-side
 * handles); *shift = -1 when residual scaling is off.  mg_setup fails with
 * MG_ERR_PREC when opt.rescale_half would enter an FP16 level whose bound
 * exceeds 2^14 (its right-hand side is rescaled to max-norm one on its own).
 * Errors: MG_ERR_ARG. */
mg_status_t mg_alpha_shift(mg_handle h, int instance, int *shift);

/* Release the handle (never frees caller memory).  NULL is accepted. */
mg_status_t mg_destroy(mg_handle h);

const char *mg_status_string(mg_status_t s);
const char *mg_last_error(void);

/* ---- Stage-level access, for per-kernel checks and custom cycles ----------
 * Level index `level` counts from the finest (0) to the base (levels-1), as in
 * level_prec.  Buffers: */
typedef enum {
    MG_BUF_RHS = 0,   /* b_l: right-hand side of level l's correction equation */
    MG_BUF_COR = 1,   /* c_l: level l's current correction, grid-scaled (e_l / h_l^2) */
    MG_BUF_RES = 2,   /* finest level only: FP64 residual r of the refinement loop */
    MG_BUF_SOL = 3    /* finest level only: FP64 iterate u of the refinement loop */
} mg_buffer_t;

typedef enum {
    MG_STAGE_SMOOTH_FIRST = 0,   /* c_l = nu1 damped-Jacobi sweeps on L c = b_l from c = 0 */
    MG_STAGE_SWEEP = 1,          /* c_l = one damped-Jacobi sweep of c_l */
    MG_STAGE_RESTRICT = 2,       /* b_{l+1} = round(FW(b_l - L c_l)), full weighting */
    MG_STAGE_PROLONG_SWEEP = 3,  /* c_l = round(c_l + 4 P c_{l+1}), then one sweep if nu2 >= 1 */
    MG_STAGE_COARSE = 4          /* base level: c = b / (2 dim), the exact one-point solve */
} mg_stage_t;

/* Copy a dense device array (n_l^dim values in format src_prec) into a level
 * buffer, rounding to nearest even into the level's format.  Async. */
mg_status_t mg_level_write(mg_handle h, int level, mg_buffer_t buf, const void *src,
                           mg_prec_t src_prec, void *stream);

/* Copy a level buffer out to a dense device array in format dst_prec
 * (rounding to nearest even if narrower).  Async. */
mg_status_t mg_level_read(mg_handle h, int level, mg_buffer_t buf, void *dst, mg_prec_t dst_prec,
                          void *stream);

/* Run one stage of the cycle on the bound workspace.  Async. */
mg_status_t mg_stage(mg_handle h, mg_stage_t stage, int level, void *stream);

/* Levels of the handle, and n of one level. */
mg_status_t mg_levels(mg_handle h, int *nlevels);
mg_status_t mg_level_n(mg_handle h, int level, int *n);

/* ---- Launch shapes --------------------------------------------------------
 * Each level except the base has two launch shapes; the autotuner and callers
 * may change them (results do not depend on the shape: every shape forms the
 * same roundings).  Changing a shape discards the captured graph. */
typedef enum {
    MG_SHAPE_STENCIL = 0,   /* smoothing, sweeps, prolongation, refinement update:
                               {V (4|8 values per thread along x), zc (planes per
                               thread), bs (threads per block, 64..256, register-queue
                               kernel), xcd (0|1: keep neighbouring tiles on one XCD),
                               ty (3-D: 0 = register-queue kernel, > 0 = LDS-plane
                               kernel with ty output rows per block)[, dp (LDS-plane
                               kernel: 1 or 2 planes loaded ahead; default 1)[, sg
                               (LDS-plane prolongation: 1 = stage the z-interpolated
                               coarse plane in LDS where it fits, default; 0 = each row
                               reads its coarse rows from memory)]]} */
    MG_SHAPE_RESTRICT = 1,  /* residual + restriction: {V (4|8), tyc (coarse rows per
                               block, 3-D), zcc (coarse planes per block), pipe (3-D:
                               1 = correction plane staged in LDS, next plane
                               prefetched; 2 = as 1 with the x weights applied in
                               the fine threads, needs P/V <= 64; 3, 4 = as 2 with
                               2 or 3 planes prefetched)} */
    MG_SHAPE_UPDATE = 2,    /* level 0 only: the FP64 refinement update, same five
                               values as MG_SHAPE_STENCIL */
    MG_SHAPE_SMOOTH = 3,    /* the first pre-smoothing kernel only (five values) */
    MG_SHAPE_SWEEP = 4,     /* the single sweeps only (five values); MG_SHAPE_STENCIL
                               sets SMOOTH, SWEEP and PROLONG together and reads SWEEP */
    MG_SHAPE_PROLONG = 5,   /* prolongation + correction + sweep only (five values) */
    MG_SHAPE_TAIL = 6,      /* 3-D, level argument 0: {on (0|1)}.  When on (the
                               default), the coarse end of the V-cycle -- from the
                               first level of pitch <= 16 (<= 8 for FP64 levels)
                               whose levels share one format, down to the base and
                               back -- runs as one single-workgroup kernel with the
                               levels in LDS; bitwise the same result.  The
                               workspace copies of those levels are then not
                               updated. */
    MG_SHAPE_FUSE = 7,      /* 3-D, level argument 0: {on (0|1)[, V (4), zc, xcd,
                               ty[, from_r (0|1)]]}.  When on (the default; the
                               autotuner keeps it only where it is faster), the last
                               post-smoothing sweep of the finest level and the
                               refinement update run as one kernel inside ir_solve
                               (same result).  from_r = 1 forms the sweep's
                               right-hand side round(r / alpha) from the FP64
                               residual r, as the first smoothing did, instead of
                               reading it back (the element size fewer bytes per
                               point; r is also read on the tile's halo rows); the
                               kernel then writes the new residual to a second array
                               of the workspace and the two swap roles every step.
                               An FP64 finest level without residual scaling, whose
                               right-hand side is r itself, takes only from_r = 1.
                               Default: 1 for FP32/FP64 finest levels, 0 for 2-byte
                               ones; the autotuner times both.  Not used when nu2 < 2.
                               Reading returns whether it is in use and its shape. */
    MG_SHAPE_FUSE_SR = 8    /* 3-D, level l below the base: {on (0|1)[, tyc, zcc[, lds16]]}.  When
                               on, the level's first pre-smoothing (two sweeps from zero)
                               and the residual + restriction of its result run as one
                               kernel (same result).  Level 0: the finest level inside
                               ir_solve, from the scaled residual (on by default).  Level
                               l >= 1: that level, from its stored right-hand side (off by
                               default).  The autotuner keeps it only where it is faster.
                               Needs nu1 = 2 and P/8 dividing 64 (an FP64 level: one
                               coarse row per tile at P = 512); level 0 reads the
                               scaled residual, or with an FP64 finest level and no
                               residual scaling the residual itself; not used into a
                               rescaled level.  lds16 = 1 (FP16/BF16 levels) keeps the
                               two sweeps' results in LDS in that 2-byte format instead of
                               FP32 (exact: they are values of it), so that two workgroups
                               fit a CU; three values set lds16 = 0.  Reading returns
                               whether it is in use and its shape (lds16 as a fourth value
                               when nparams >= 4). */
} mg_shape_kind_t;
/* Q1 handles: the levels stored in a 2-byte format on a 3-D grid of pitch a
 * multiple of 4 run their sweep, their residual (ahead of the restriction) and,
 * on level 0, the refinement update as LDS-staged kernels (every plane read
 * from memory once per block row).
 * MG_SHAPE_SWEEP, MG_SHAPE_RESTRICT and MG_SHAPE_UPDATE then take {ty (rows per
 * block), zc (planes per block)}, or {0, 0} for the built-in choice; a shape
 * must fit 1024 threads ((ty + 2) P / 4), 64 KB of LDS and the update's partial
 * budget (MG_ERR_ARG otherwise, and on other levels for any shape but {0, 0}).
 * The residual runs fused with its restriction (the fine residual kept in LDS,
 * bitwise the same coarse b): its shape takes even ty and zc and (ty + 3) P / 4
 * threads; {ty, zc, 1} runs residual and restriction as two kernels instead.
 * The other kinds return MG_ERR_STATE.  opt.autotune times these shapes per
 * level and kernel against the built-in one (cached as for finite differences).
 * Reading returns the {ty, zc} in use, {0, 0} on levels without such kernels. */
mg_status_t mg_set_shape(mg_handle h, int level, int kind, const int *params, int nparams);
/* Reading a shape: the values mg_set_shape takes (up to nparams).  On a
 * many-right-hand-side handle, the stencil kinds and MG_SHAPE_RESTRICT of
 * levels below the base (only zc, and zcc of the restriction, shape those
 * kernels).  A batched handle's shapes are read per instance with
 * mg_get_instance_shape. */
mg_status_t mg_get_shape(mg_handle h, int level, int kind, int *params, int nparams);

/* A batched handle: the launch shape of level `level` (below the base) of
 * instance `inst` -- the stencil kinds, MG_SHAPE_RESTRICT, and MG_SHAPE_UPDATE on
 * level 0 -- as mg_get_shape returns them.  MG_ERR_STATE on other handles,
 * MG_ERR_ARG for an instance, level or kind out of range. */
mg_status_t mg_get_instance_shape(mg_handle h, int inst, int level, int kind, int *params, int nparams);

/* ---- Measurement --------------------------------------------------------
 * Bandwidth probe: one kernel launch that copies (kind 0), reads (1) or
 * writes (2) `bytes` (a multiple of 16) of device memory with 16-byte lanes,
 * `blocks` blocks of 256 threads in a grid-stride loop.  Kind 3 streams the
 * access mix of the refinement update: dst holds two FP64 arrays of `bytes`
 * each (read and written), src two FP16 arrays of bytes/4 each (read), 36
 * bytes per element; bytes a multiple of 32.  Kinds 4, 5 are kinds 0, 1 with
 * non-temporal loads and stores; kind 6 is kind 3 with non-temporal loads and
 * stores, kind 7 with non-temporal stores only.  Used to measure the
 * achievable HBM bandwidth and to calibrate traffic counters.  For kinds 1 and
 * 5 the first 4 bytes of dst may be written.  Async. */
mg_status_t mg_bandwidth_probe(void *dst, const void *src, size_t bytes, int kind, int blocks, void *stream);

/* Run one refinement step eagerly with a HIP event pair around every kernel
 * launch, on stream, and return per-kernel durations.  The step uses the
 * workspace state left by the last ir_solve (it updates u and r like a real
 * step).  names/ms/bytes are caller arrays of capacity cap; *count receives the
 * number of kernels launched.  bytes[i] is the algorithmic HBM traffic of
 * launch i (each array read or written once).  Synchronises. */
mg_status_t mg_profile_step(mg_handle h, void *stream, int cap, int *count, const char **names,
                            double *ms, double *bytes, int *levels_out);

#ifdef __cplusplus
}
#endif
#endif /* MGIR_H */
