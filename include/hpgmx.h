/*
 * hpgmx.h -- C ABI of the MI355X (gfx950) HPG-MxP hot path: restarted,
 * right-preconditioned GMRES with iterative refinement (GMRES-IR, CGS2
 * orthogonalisation, Givens least squares) and a geometric-multigrid V-cycle
 * (multicolour Gauss-Seidel smoother, injection restriction fused with the
 * residual, prolongation P = R^T) on a nonsymmetric 27-point stencil.
 *
 * Paper: Kashi et al., "Scaling the memory wall using mixed-precision --
 * HPG-MxP on an exascale machine", SC'25, arXiv 2507.11512.  Section
 * references below are to that paper.
 *
 * Conventions shared by every entry point
 *  - All vector arguments are DEVICE pointers to contiguous arrays in the
 *    natural lexicographic order I = i + nx*(j + ny*k) of the level they
 *    belong to (0-based, i fastest).  The library's internal colour-blocked
 *    ordering is never visible through the ABI.
 *  - Vectors are float64 for HPGMX_F64 and float32 for HPGMX_F32, HPGMX_F16
 *    and HPGMX_BF16 (the 16-bit types describe how the matrix is stored; the
 *    vectors stay float32), and binary16 / bfloat16 for HPGMX_F16_MG /
 *    HPGMX_BF16_MG, except the output of hpgmx_spmv, which is float32 (the
 *    SpMV of the solver feeds the FP32 Krylov basis).  The batched entry
 *    points accept HPGMX_F64 .. HPGMX_BF16 only.
 *  - The caller owns every pointer it passes.  The library owns its
 *    matrices, hierarchy and Krylov workspace: they live in memory the caller
 *    bound with hpgmx_bind_workspace, or else in memory the library
 *    allocates itself and frees in hpgmx_destroy.
 *  - Work is enqueued on the HIP stream given to hpgmx_setup_problem.
 *    hpgmx_spmv, hpgmx_smooth, hpgmx_vcycle, hpgmx_restrict_residual,
 *    hpgmx_prolong_add and hpgmx_rhs_from_x are stream-ordered and return
 *    before the work finishes.  hpgmx_gmres_ir_solve returns after the solve
 *    has finished, because it reads the residual estimate every iteration.
 *  - Errors are returned, never thrown: a negative hpgmx_status.  EINVAL
 *    (bad argument) leaves the handle usable.  EHIP (a HIP runtime error)
 *    poisons the handle: every later call except hpgmx_last_error and
 *    hpgmx_destroy returns ESTATE.  hpgmx_last_error gives a message.
 *  - A solve that does not reach the tolerance within max_iters is not an
 *    error: it returns HPGMX_OK with stats->converged = 0.
 *  - One handle must not be used from two host threads at once.
 */
#ifndef HPGMX_H
#define HPGMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hpgmx_ctx *hpgmx_handle;

typedef enum {
    HPGMX_OK = 0,
    HPGMX_EINVAL = -1,     /* invalid argument; the handle stays usable      */
    HPGMX_ENOMEM = -2,     /* device memory or bound workspace exhausted      */
    HPGMX_EHIP = -3,       /* HIP runtime error; the handle is poisoned       */
    HPGMX_ESTATE = -4,     /* call out of order, or handle poisoned           */
    HPGMX_ENONFINITE = -5  /* NaN or Inf in the right-hand side or residual  */
} hpgmx_status;

/* Precisions.  HPGMX_F64: everything in FP64.  HPGMX_F32: FP32 matrices,
 * multigrid vectors and Krylov basis.  HPGMX_F16 / HPGMX_BF16: the multigrid
 * matrices stored in binary16 / bfloat16, everything else as HPGMX_F32.
 * HPGMX_F16_MG / HPGMX_BF16_MG: the whole multigrid hierarchy in 16 bits --
 * the matrices and the work vectors of every level (the residuals r_l and
 * corrections z_l) -- with FP32 arithmetic and an FP32 Krylov basis (the
 * low-precision preconditioner the paper leaves as future work, Sec. 5). */
typedef enum {
    HPGMX_F64 = 0, HPGMX_F32 = 1, HPGMX_F16 = 2, HPGMX_BF16 = 3,
    HPGMX_F16_MG = 4, HPGMX_BF16_MG = 5
} hpgmx_dtype;

typedef enum {
    HPGMX_GS_FORWARD = 0,   /* colours 0..7: the smoother of Sec. 3           */
    HPGMX_GS_BACKWARD = 1,  /* colours 7..0                                    */
    HPGMX_GS_SYMMETRIC = 2  /* forward then backward, eqs. (1)-(2) (Sec. 2)    */
} hpgmx_sweep;

/* The operator (Sec. 2, Sec. 3): 27-point stencil on an nx*ny*nz grid with
 * Dirichlet truncation at the boundary; diagonal 26, off-diagonal -1, except
 * that every entry coupling to an x-neighbour at i-1 is -1-beta and at i+1 is
 * -1+beta (beta = 0 is the symmetric matrix of Sec. 3). */
typedef struct {
    int nx, ny, nz;
    double beta;
} hpgmx_problem_desc;

/* A general 27-point stencil: coef[t] multiplies the neighbour at offset
 * (di,dj,dk) with t = 9(dk+1) + 3(dj+1) + (di+1) (t = 13 is the diagonal,
 * which must be nonzero); entries outside the grid are dropped as for the
 * beta family.  The beta family is coef = 26 on the diagonal, -1-beta at
 * di = -1, -1+beta at di = +1, -1 elsewhere.  The stencil of A^T is coef
 * reversed (coef[26 - t]).  Used for the adjoint (gradients with respect to
 * the 27 entries). */
typedef struct {
    int nx, ny, nz;
    double coef[27];
} hpgmx_stencil_desc;

/* The V-cycle (Sec. 2 Fig. 1 applied recursively; Sec. 3): `levels` grids,
 * each coarser one half the size in every dimension (coarse point (I,J,K) is
 * fine point (2I,2J,2K)); pre/post smoothing sweeps on every level but the
 * coarsest, which gets coarsest_sweeps sweeps; `sweep` is an hpgmx_sweep.
 * Every dimension must be divisible by 2^(levels-1) and the coarsest level
 * must be at least 2 in every dimension.  1 <= levels <= 8. */
typedef struct {
    int levels, pre_sweeps, post_sweeps, coarsest_sweeps;
    int sweep;
} hpgmx_mg_desc;

/* Solve flags. */
#define HPGMX_SOLVE_PROFILE 1  /* time every kernel launch with HIP events   */
#define HPGMX_SOLVE_GRAPH 2    /* replay each inner step as a captured hipGraph
                                  (on a private stream ordered after and before
                                  the handle's stream; ignored with PROFILE) */

/* Alg. 3 parameters.  restart = m (1..63), max_iters counts inner steps over
 * all restarts, tol is the relative residual ||b - A x|| / ||b|| to reach
 * (strict "<").  inner_dtype selects the precision of the steps Alg. 3
 * allows in low precision: HPGMX_F64 gives the plain FP64 GMRES-MG,
 * HPGMX_F32 the FP32-inner GMRES-IR, HPGMX_F16 / HPGMX_BF16 the FP32-inner
 * solver with the multigrid matrices stored in 16 bits, HPGMX_F16_MG /
 * HPGMX_BF16_MG with the whole multigrid hierarchy in 16 bits (the V-cycle's
 * input is the Krylov vector times a power of two that brings its entries
 * near 1, inside binary16's range; the SpMV and the update undo it).  The outer residual
 * and the solution update are always FP64.  If res_hist_host is not NULL the
 * estimated relative residual after each inner step is written there (host
 * memory, res_hist_len entries at most). */
typedef struct {
    int restart, max_iters;
    double tol;
    int inner_dtype;
    double *res_hist_host;
    int res_hist_len;
    int flags;
} hpgmx_solve_desc;

typedef struct {
    int iters;          /* inner steps, summed over restarts                 */
    int restarts;       /* completed restart cycles                          */
    int converged;      /* final relative residual < tol                     */
    int breakdown;      /* a new Krylov vector had norm <= 1e-300            */
    double rho0;        /* ||b||                                             */
    double final_rel_res; /* ||b - A x|| / ||b|| in FP64 at exit             */
    double est_rel_res; /* last Givens estimate |t_{k+1}| / ||b||             */
    double solve_ms;    /* device time of the whole solve (HIP events)       */
} hpgmx_solve_stats;

/* Creates a handle for one problem on the current HIP device.  hip_stream
 * is a hipStream_t (NULL = the null stream); the library enqueues all of its
 * work there.  No device memory is touched until hpgmx_mg_setup. */
hpgmx_status hpgmx_setup_problem(const hpgmx_problem_desc *desc, void *hip_stream,
                                 hpgmx_handle *out);

/* As hpgmx_setup_problem for a general 27-point stencil (every multigrid
 * level uses the same stencil).  EINVAL for non-finite entries or a zero
 * diagonal. */
hpgmx_status hpgmx_setup_problem_stencil(const hpgmx_stencil_desc *desc, void *hip_stream,
                                         hpgmx_handle *out);

/* Storage of the ELL column indices of every level (Sec. 3.2 "ELLPACK matrix
 * format").  HPGMX_COLS_INT32 (the default): one int32 column index per slot.
 * HPGMX_COLS_OFFSET16: the index of slot s of a row p of colour c stored as
 * the 16-bit offset col - p - D[c][s], with D a table of 8 x 26 offsets taken
 * from interior rows of the generated matrix; padded slots hold a reserved
 * value.  It halves the index bytes every ELL pass moves (the paper notes
 * that index fetches limit the mixed-precision gain of the smoother and the
 * SpMV, Sec. 4); hpgmx_mg_setup fails with EINVAL if an offset does not fit
 * 16 bits (odd level extents of a few hundred and more).  The batched entry
 * points need int32 indices.  Must precede hpgmx_mg_setup. */
#define HPGMX_COLS_INT32 0
#define HPGMX_COLS_OFFSET16 1
hpgmx_status hpgmx_set_column_format(hpgmx_handle h, int format);

/* Data layout and work order, for layout studies and tests; the defaults
 * are the tuned ones and a production solve needs no call.  The choice
 * changes where data sits, in which order workgroups take row tiles and
 * how a sweep is cut into launches, never the arithmetic: results are
 * bit-identical under every setting.
 *   tile_order     0 = tiles in launch order, 1 = each of the eight XCDs
 *                  takes one contiguous range of row tiles, 3 = as 1, plus
 *                  the plane order for the full-grid SpMVs (each XCD takes
 *                  a slab of grid planes and walks it plane by plane through
 *                  all eight colours), 2 (default) = as 1, plus the order
 *                  measured fastest for each full-grid SpMV: the slab order
 *                  (each XCD takes one eighth of every colour block) for the
 *                  FP32 and 16-bit SpMV, the plane order for the batched
 *                  SpMV, the XCD-contiguous order for the FP64 SpMV.  With
 *                  2 and 3 the batched SpMV over the whole rows of the
 *                  colour pair (0, 1) or (6, 7) walks each XCD's slab plane
 *                  by plane through both colours (the plane-pair order).
 *   ell_chunk_log2 rows per ELL chunk as a power of two, 0..16 (0 =
 *                  slot-major over the whole level; default 8).
 *   ldq_pad        elements added between Krylov basis columns, even,
 *                  0..2^20 (default 1088).
 *   pair_rows      a Gauss-Seidel sweep from a zero guess relaxes two
 *                  colours (c, c ^ 1) per launch on levels with an even x
 *                  extent: the first two pairs of the sweep on levels with
 *                  at most pair_rows rows per colour, the last two on
 *                  levels with at most pair_rows / 64; 0 = never (default
 *                  2^17).
 *   spmv_in_sweep  how the solver's SpMV w = A z after each V-cycle shares
 *                  work with the V-cycle's last level-0 sweep.  0: one SpMV
 *                  over all rows.  1: the sweep's last colour launch (whose
 *                  neighbours are all final) also writes its colour's rows
 *                  of w, and the SpMV covers the other seven colours (same
 *                  bits as 0).  2 (default): as 1, and the launches of the
 *                  sweep's third to seventh colours also write, for their
 *                  rows, the sum over the slots to colours relaxed before
 *                  them, so the SpMV reads only the remaining 20, 18, 8, 6
 *                  and 2 slots of those rows.
 *                  3: the row sums of 2, all formed by the SpMV (same bits
 *                  as 2; differs from 0 and 1 in rounding only).  Batched
 *                  solves follow 0, 2 and 3 (1 runs as 0) with FP32 or FP64
 *                  matrices, and 0 with 16-bit ones.
 * A negative argument keeps that default.  Orders 2 and 3 fall back to 1 on
 * levels with an odd extent.  EINVAL for values out of range;
 * ESTATE after hpgmx_mg_setup (must precede it, and hpgmx_workspace_bytes
 * when a workspace is bound). */
hpgmx_status hpgmx_set_layout(hpgmx_handle h, int tile_order, int ell_chunk_log2, int ldq_pad,
                              long long pair_rows, int spmv_in_sweep);

/* Device bytes the hierarchy of `mg` plus the Krylov workspace for a
 * restart length `restart` need, for every inner dtype whose bit
 * (1 << hpgmx_dtype) is set in dtype_mask. */
hpgmx_status hpgmx_workspace_bytes(hpgmx_handle h, const hpgmx_mg_desc *mg, int restart,
                                   unsigned dtype_mask, size_t *bytes);

/* Hands the library a caller-owned device region (e.g. a torch tensor) to
 * carve all of its buffers from.  Must precede hpgmx_mg_setup; the region
 * must stay alive until hpgmx_destroy.  Without it the library allocates. */
hpgmx_status hpgmx_bind_workspace(hpgmx_handle h, void *dev_ptr, size_t bytes);

/* Builds the multigrid hierarchy on the device: for every level the ELL
 * matrix (26 off-diagonal slots of values and int32 column indices plus the
 * diagonal, Sec. 3.2 "ELLPACK matrix format") in FP64, FP32, FP16 and BF16
 * values, in the colour-blocked order of the multicolour smoother
 * (Sec. 3.2).  Blocks until done. */
hpgmx_status hpgmx_mg_setup(hpgmx_handle h, const hpgmx_mg_desc *mg);

/* Alg. 3.  b: FP64 right-hand side (device, natural order, N = nx*ny*nz).
 * x: FP64 initial guess on entry, solution on exit.  stats may be NULL.
 * Returns ENONFINITE if b or an outer residual is not finite. */
hpgmx_status hpgmx_gmres_ir_solve(hpgmx_handle h, const double *b, double *x,
                                  const hpgmx_solve_desc *desc, hpgmx_solve_stats *stats);

/* y = A_level x with the level's matrix stored in `dtype` (the SpMV of
 * Alg. 3).  x and y must not overlap. */
hpgmx_status hpgmx_spmv(hpgmx_handle h, int level, int dtype, const void *x, void *y);

/* One Gauss-Seidel sweep of kind `sweep` (an hpgmx_sweep) for A_level z = r,
 * in place on z (relaxation form of eq. (1), multicolour order of Sec. 3.2).
 * zero_guess != 0 treats z as zero on entry (its contents are ignored). */
hpgmx_status hpgmx_smooth(hpgmx_handle h, int level, int dtype, int sweep, const void *r,
                          void *z, int zero_guess);

/* z = M^{-1} r: one V-cycle from z = 0 on level 0 (Sec. 2 Fig. 1, Sec. 3). */
hpgmx_status hpgmx_vcycle(hpgmx_handle h, int dtype, const void *r, void *z);

/* r_coarse = R (r - A_level z): the fused residual-restriction of eq. (6),
 * evaluated only at the coarse points.  r, z on `level`, r_coarse on
 * level + 1 (level < levels - 1). */
hpgmx_status hpgmx_restrict_residual(hpgmx_handle h, int level, int dtype, const void *r,
                                     const void *z, void *r_coarse);

/* The first half of one V-cycle level exactly as the V-cycle runs it
 * (Sec. 2 Fig. 1, Sec. 3.2): z <- nsweeps Gauss-Seidel sweeps of kind
 * `sweep` from z = 0 on `level`, then r_coarse = R (r - A_level z), the fused
 * residual-restriction of eq. (6).  After a single forward or backward sweep
 * the restriction takes the V-cycle's shortcut: relaxing the injection
 * colour (colour 4) left r - A z = 0 on its rows while the colours relaxed
 * after it were still zero, so r - A z at an injection point is minus its
 * couplings to those colours (8 slots forward, 18 backward; equal to eq. (6)
 * in exact arithmetic).  Otherwise eq. (6) is evaluated in full.  r: input on
 * `level`; z: output on `level`; r_coarse: output on level + 1 (level <
 * levels - 1); 0 <= nsweeps <= 16.  Stream-ordered. */
hpgmx_status hpgmx_presmooth_restrict(hpgmx_handle h, int level, int dtype, int sweep, int nsweeps,
                                      const void *r, void *z, void *r_coarse);

/* Test export of the Krylov state of Alg. 3: the last restart cycle of the
 * last hpgmx_gmres_ir_solve run with inner dtype `dtype`.  *k = inner steps
 * that cycle took.  Q (device, FP64, (k+1) vectors of N entries one after
 * the other, natural order): the stored basis columns; basis vector
 * q_j = scale[j] * Q[j] (the library stores the columns unnormalised, with
 * their scale).  scale (host, k+1 doubles).  Hbar (host, FP64, (k+1) x k
 * column-major, leading dimension k+1): the Hessenberg matrix before the
 * Givens rotations, in the basis q_j.  y (host, k doubles): the projected
 * solution of the cycle, y = H^{-1} t.  Any of Q, scale, Hbar, y may be NULL.
 * Blocks.  ESTATE if no such solve has run. */
hpgmx_status hpgmx_krylov_cycle_get(hpgmx_handle h, int dtype, int *k, double *Q, double *scale, double *Hbar,
                                    double *y);

/* z += P z_coarse with P = R^T (eq. (3)): z on `level`, z_coarse on
 * level + 1. */
hpgmx_status hpgmx_prolong_add(hpgmx_handle h, int level, int dtype, const void *z_coarse,
                               void *z);

/* b = A x on level 0 in FP64 (device, natural order). */
hpgmx_status hpgmx_rhs_from_x(hpgmx_handle h, const double *x, double *b);

/* Adjoint gradient of the stencil entries: out27[t] = sum over grid points i
 * whose neighbour i + d_t lies in the grid of lam_i * x_{i + d_t}, in FP64.
 * If x = A^{-1} b and A^T lam = dL/dx, then dL/dcoef[t] = -out27[t] and
 * dL/db = lam.  lam, x: FP64 device vectors (natural order, level 0); out27:
 * 27 doubles of device memory.  Stream-ordered. */
hpgmx_status hpgmx_stencil_grad(hpgmx_handle h, const double *lam, const double *x, double *out27);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the result of
 * hpgmx_stencil_grad (same arguments, same meaning, FP64 sums in another
 * order) computed without allocating anything.  Its only scratch is a fixed
 * device array of the library (1024 x 27 partial sums, 216 KiB per GPU, held
 * until the process ends), which serves every grid size the handle accepts;
 * lam and x are read in the natural order, without staging copies.  All
 * calls on one GPU share that array: calls that overlap on one GPU (other
 * streams or host threads) race, calls on one stream are safe.  Works
 * before any solve has run.  Stream-ordered. */
hpgmx_status hpgmx_stencil_grad_noalloc(hpgmx_handle h, const double *lam, const double *x, double *out27);

/* Per-kernel timing of the last solve run with HPGMX_SOLVE_PROFILE.
 * Kernel ids are HPGMX_K_*; `level` selects the grid for the per-level
 * kernels (ignored otherwise).  Returns the summed device time in ms and the
 * number of launches. */
#define HPGMX_K_GS 0           /* one colour of a Gauss-Seidel sweep          */
#define HPGMX_K_GS_ZERO 1      /* one colour of a sweep from a zero guess     */
#define HPGMX_K_RESTRICT 2     /* fused residual-restriction                  */
#define HPGMX_K_PROLONG 3      /* prolongation-correction                    */
#define HPGMX_K_SPMV_DOT 4     /* reserved (a fused SpMV + GEMVT; not launched) */
#define HPGMX_K_CGS_DOT 5      /* h2 = Q^T (w - Q h1)                         */
#define HPGMX_K_CGS_NORM 6     /* w -= Q (h1 + h2), ||w||^2 and Givens        */
#define HPGMX_K_NORMALIZE 7    /* reserved (the basis is stored unnormalised)  */
#define HPGMX_K_RESID64 8      /* r = b - A x in FP64 with ||r||^2            */
#define HPGMX_K_CAST 9         /* q_1 = r / rho (cast to the inner dtype)      */
#define HPGMX_K_TRSM 10        /* y = H^{-1} t                                */
#define HPGMX_K_GEMV 11        /* u = Q y                                      */
#define HPGMX_K_UPDATE 12      /* x += z in FP64                              */
#define HPGMX_K_PERMUTE 13     /* natural <-> colour-blocked order            */
#define HPGMX_K_SPMV 14        /* w = A z                                     */
#define HPGMX_K_DOT 15         /* h1 = Q^T w                                  */
#define HPGMX_K_FINISH 16      /* one-workgroup sums of the reduction passes' partial sums
                                  (and the Givens step after the norm pass)  */
#define HPGMX_K_COUNT 17
hpgmx_status hpgmx_profile_get(hpgmx_handle h, int kernel, int level, double *total_ms,
                               long long *launches);

/* ---- several right-hand sides at once --------------------------------------
 * A batch of nrhs <= 8 right-hand sides shares one pass over the matrix: the
 * SpMV, the Gauss-Seidel sweeps and the fused restriction read each matrix
 * row once for all of them (Sec. 3.2's kernels, generalised to a block of
 * vectors), while every right-hand side keeps its own Krylov basis,
 * Hessenberg matrix, rotations and convergence test.  Batched vectors are
 * passed as nrhs contiguous vectors one after the other, [nrhs][N] in the
 * natural order of the level (a row-major (nrhs, N) tensor).  Internally
 * the batch is padded to K = 2, 4 or 8 interleaved vectors; padded entries
 * are zero.  dtype is the matrix precision as for the single-vector calls
 * (vectors FP64 for HPGMX_F64, FP32 otherwise; tile tables are kept per
 * dtype).
 *
 * Tile shapes.  The batched stencil kernels run R of the K right-hand sides
 * of a row per lane (R = 1, 2, 4 or 8, R <= K; K / R lanes share a row).
 * hpgmx_batch_autotune times every R for every kernel kind and level on the
 * device and keeps the fastest; without it the library uses a fixed rule
 * (R = K on levels with at least 2^22 / K rows, R = 1 below).  The choice
 * never changes results: per (row, right-hand side) the arithmetic is the
 * same for every R. */
#define HPGMX_BK_SPMV 0      /* batched SpMV                                  */
#define HPGMX_BK_GS 1        /* one colour of a batched GS sweep              */
#define HPGMX_BK_GS_ZERO 2   /* one colour of a batched sweep from zero       */
#define HPGMX_BK_RESTRICT 3  /* batched fused residual-restriction            */
#define HPGMX_BK_RESID64 4   /* batched FP64 outer residual (level 0)         */
#define HPGMX_BK_COUNT 5
typedef struct {
    int rhs_per_lane[HPGMX_BK_COUNT][8]; /* R per kernel kind and level (0 = rule) */
    double ms[HPGMX_BK_COUNT][8];        /* autotune: time of the chosen R (ms;
                                            a full sweep for the GS kinds)     */
} hpgmx_batch_tuning;

/* Times every tile shape for a batch of nrhs right-hand sides with matrices
 * in `dtype`, adopts the fastest, and writes the table to *out (may be
 * NULL).  Blocks.  Overwrites the handle's batched work vectors. */
hpgmx_status hpgmx_batch_autotune(hpgmx_handle h, int nrhs, int dtype, hpgmx_batch_tuning *out);

/* Adopts a tile table (entries 0 use the fixed rule; others must divide the
 * padded batch width K).  hpgmx_batch_get_tuning reads the table in use. */
hpgmx_status hpgmx_batch_set_tuning(hpgmx_handle h, int nrhs, int dtype, const hpgmx_batch_tuning *in);
hpgmx_status hpgmx_batch_get_tuning(hpgmx_handle h, int nrhs, int dtype, hpgmx_batch_tuning *out);

/* Extra device bytes the batched state for nrhs right-hand sides, the
 * hierarchy `mg`, restart length `restart` and the inner dtypes in
 * dtype_mask (bits 1 << hpgmx_dtype) needs on top of hpgmx_workspace_bytes
 * for the same mask (a bound workspace must hold both). */
hpgmx_status hpgmx_workspace_bytes_batched(hpgmx_handle h, const hpgmx_mg_desc *mg, int nrhs, int restart,
                                           unsigned dtype_mask, size_t *bytes);

/* Y[j] = A_level X[j] for j < nrhs (X, Y: [nrhs][N_level], must not overlap). */
hpgmx_status hpgmx_spmv_batched(hpgmx_handle h, int level, int dtype, int nrhs, const void *X, void *Y);

/* One Gauss-Seidel sweep of kind `sweep` for every right-hand side
 * (as hpgmx_smooth; R, Z: [nrhs][N_level], Z updated in place). */
hpgmx_status hpgmx_smooth_batched(hpgmx_handle h, int level, int dtype, int sweep, int nrhs,
                                  const void *R, void *Z, int zero_guess);

/* hpgmx_presmooth_restrict for every right-hand side (R: [nrhs][N_level]
 * input, Z: [nrhs][N_level] output, R_coarse: [nrhs][N_{level+1}] output). */
hpgmx_status hpgmx_presmooth_restrict_batched(hpgmx_handle h, int level, int dtype, int sweep, int nsweeps,
                                              int nrhs, const void *R, void *Z, void *R_coarse);

/* Z[j] = M^{-1} R[j]: one batched V-cycle per right-hand side (as
 * hpgmx_vcycle; R, Z: [nrhs][N]). */
hpgmx_status hpgmx_vcycle_batched(hpgmx_handle h, int dtype, int nrhs, const void *R, void *Z);

/* Alg. 3 for nrhs right-hand sides in lockstep.  B: FP64 [nrhs][N]; X: FP64
 * [nrhs][N], initial guesses on entry, solutions on exit; stats: nrhs
 * entries (may be NULL).  desc->inner_dtype as for hpgmx_gmres_ir_solve;
 * desc->res_hist_host, if set, holds nrhs rows of res_hist_len entries.
 * Right-hand side j follows exactly the sequence of steps its own
 * hpgmx_gmres_ir_solve would take: it stops taking Krylov steps in a cycle
 * when its estimate drops below tol, when its new Krylov vector breaks down,
 * or when its own iteration count reaches max_iters; the others carry on,
 * and a right-hand side that has stopped leaves its solution untouched
 * (its extra lockstep work is discarded).  The call returns when every
 * right-hand side has converged or run out of iterations.  Flag
 * HPGMX_SOLVE_AUTOTUNE runs hpgmx_batch_autotune first if this (nrhs,
 * dtype) has no table yet. */
#define HPGMX_SOLVE_AUTOTUNE 4
hpgmx_status hpgmx_gmres_ir_solve_batched(hpgmx_handle h, int nrhs, const double *B, double *X,
                                          const hpgmx_solve_desc *desc, hpgmx_solve_stats *stats);

/* Streaming copy of `bytes` (multiple of 16) from src to dst, `reps` times,
 * timed with HIP events: the measured-bandwidth reference for the roofline
 * and the scale for hardware byte counters.  Blocks; *ms = average per copy. */
hpgmx_status hpgmx_stream_copy(hpgmx_handle h, const void *src, void *dst, size_t bytes,
                               int reps, double *ms);

hpgmx_status hpgmx_destroy(hpgmx_handle h);
const char *hpgmx_last_error(hpgmx_handle h);

#ifdef __cplusplus
}
#endif
#endif /* HPGMX_H */
