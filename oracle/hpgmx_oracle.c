/*
 * hpgmx_oracle.c -- plain FP64 CPU oracle for the HPG-MxP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product path (the
 * HIP library under paper_2507_11512_amd/) never calls it, and the two share
 * no code, headers, tables or generators.
 *
 * Everything is computed directly from the definitions in the paper, on the
 * natural lexicographic ordering I = i + nx*(j + ny*k) (0-based, i fastest),
 * with no stored matrix: each stencil entry is evaluated where it is used.
 * The paper sections followed are cited per function (Kashi et al., "Scaling
 * the memory wall using mixed-precision - HPG-MxP on an exascale machine",
 * SC'25, arXiv 2507.11512).
 *
 * Readings taken where the paper is silent or garbled are restated at the
 * point of use below.
 *
 * Parity status: every exported function is pinned by a test in
 * tests/test_oracle_pins.py against an independent construction (Kronecker
 * products, scipy triangular solves, dense LU, lstsq, closed forms).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t idx_t;

/* Threads the OpenMP loops of this library use. */
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ------------------------------------------------------------------------- */
/* Problem definition: the 27-point stencil (Sec. 2 "Background": 27 nonzeros */
/* per interior row, fewer on boundary rows; Sec. 3: diagonal 26, other       */
/* entries -1, optional nonsymmetric variant).                                */
/* ------------------------------------------------------------------------- */

/* Nonsymmetric variant (Sec. 3 mentions the option without values).  Reading:
 * the entry coupling to an x-neighbour at di = -1 is -1-beta, at di = +1 it is
 * -1+beta, all other off-diagonal entries are -1, the diagonal is 26.
 * faces_only = 0: every entry with di = -1 / +1 (9 each) carries the shift.
 * faces_only = 1: only the two face neighbours (dj = dk = 0) carry it.       */
double or_coef(double beta, int faces_only, int di, int dj, int dk)
{
    if (di == 0 && dj == 0 && dk == 0) return 26.0;
    if (faces_only && (dj != 0 || dk != 0)) return -1.0;
    if (di == -1) return -1.0 - beta;
    if (di == +1) return -1.0 + beta;
    return -1.0;
}

/* The stencil as a table of 27 entries in slot order
 * s = 9(dk+1) + 3(dj+1) + (di+1); s = 13 is the diagonal.  Every routine
 * below works from such a table; the beta family above fills it, and the
 * *_c entry points accept any table (used by the adjoint tests, where each
 * entry is a parameter). */
void or_stencil_from_beta(double beta, int faces_only, double *c27)
{
    for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di)
                c27[9 * (dk + 1) + 3 * (dj + 1) + (di + 1)] = or_coef(beta, faces_only, di, dj, dk);
}

static inline double cf(const double *c27, int di, int dj, int dk)
{
    return c27[9 * (dk + 1) + 3 * (dj + 1) + (di + 1)];
}

static inline idx_t lex(int nx, int ny, int i, int j, int k)
{
    return (idx_t)i + (idx_t)nx * ((idx_t)j + (idx_t)ny * (idx_t)k);
}

/* One row of y = A x: sum over the 27 offsets in slot order
 * s = 9(dk+1) + 3(dj+1) + (di+1), dropping offsets outside the grid
 * (Dirichlet truncation of the stencil at the domain boundary).             */
static double row_apply(int nx, int ny, int nz, const double *c27,
                        const double *x, int i, int j, int k)
{
    double acc = 0.0;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                int ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                acc += cf(c27, di, dj, dk) * x[lex(nx, ny, ii, jj, kk)];
            }
    return acc;
}

/* Sum of the off-diagonal terms of one row against z (slot order, diagonal
 * skipped).  Used by the Gauss-Seidel relaxation form.                      */
static double row_offdiag(int nx, int ny, int nz, const double *c27,
                          const double *z, int i, int j, int k)
{
    double acc = 0.0;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                if (di == 0 && dj == 0 && dk == 0) continue;
                int ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                acc += cf(c27, di, dj, dk) * z[lex(nx, ny, ii, jj, kk)];
            }
    return acc;
}

/* y = A x (the SpMV of Alg. 3 and the FP64 outer residual's product). */
void or_spmv_c(int nx, int ny, int nz, const double *c27, const double *x, double *y)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                y[lex(nx, ny, i, j, k)] = row_apply(nx, ny, nz, c27, x, i, j, k);
}

void or_spmv(int nx, int ny, int nz, double beta, int fo, const double *x, double *y)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
    or_spmv_c(nx, ny, nz, c27, x, y);
}

/* Selected rows of y = A x, for sampled checks at sizes where a full product
 * is not wanted.  rows[] are natural indices.                                */
void or_spmv_rows(int nx, int ny, int nz, double beta, int fo, const double *x,
                  const idx_t *rows, idx_t nrows, double *y)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
#pragma omp parallel for schedule(static)
    for (idx_t t = 0; t < nrows; ++t) {
        idx_t I = rows[t];
        int i = (int)(I % nx), j = (int)((I / nx) % ny), k = (int)(I / ((idx_t)nx * ny));
        y[t] = row_apply(nx, ny, nz, c27, x, i, j, k);
    }
}

/* |A| |x| per row: the scale of the dot-product forward-error bound used by
 * the parity tolerances (row sums of |a_ij| |x_j|).                         */
void or_absrow(int nx, int ny, int nz, double beta, int fo, const double *x, double *y)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int dk = -1; dk <= 1; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                            acc += fabs(cf(c27, di, dj, dk)) * fabs(x[lex(nx, ny, ii, jj, kk)]);
                        }
                y[lex(nx, ny, i, j, k)] = acc;
            }
}

/* ------------------------------------------------------------------------- */
/* Multicolour ordering (Sec. 3.2 "Multicolor Gauss-Seidel iteration",        */
/* Fig. 2: 8 independent sets for the 27-point stencil).                     */
/* ------------------------------------------------------------------------- */

/* Colour of point (i,j,k).  Two points of equal parity in all three
 * coordinates are never stencil neighbours, so each parity class is an
 * independent set.  Reading of the (unstated) colour order: the class whose
 * coordinates are all even -- the injection points of the restriction --
 * takes colour 4, i.e. it is relaxed fifth in a forward sweep.  Placing it
 * first would discard the coarse-grid correction in the post-smoother and
 * placing it last would make the restricted residual vanish.               */
int or_color(int i, int j, int k)
{
    return (i & 1) + 2 * (j & 1) + 4 * ((k + 1) & 1);
}

/* One relaxation over all rows of colour c:
 * z_I <- (r_I - sum_{J != I} a_IJ z_J) / a_II   (relaxation form of the
 * forward Gauss-Seidel step, eq. (1) and Sec. 3.2).  Rows of one colour do
 * not couple, so their order does not matter; natural order is used.       */
static void relax_color(int nx, int ny, int nz, const double *c27,
                        const double *r, double *z, int c)
{
    int pi = c & 1, pj = (c >> 1) & 1, pk = ((c >> 2) & 1) ^ 1;
    double diag = cf(c27, 0, 0, 0);
#pragma omp parallel for schedule(static)
    for (int k = pk; k < nz; k += 2)
        for (int j = pj; j < ny; j += 2)
            for (int i = pi; i < nx; i += 2) {
                idx_t I = lex(nx, ny, i, j, k);
                z[I] = (r[I] - row_offdiag(nx, ny, nz, c27, z, i, j, k)) / diag;
            }
}

/* One Gauss-Seidel sweep in place on z.
 * sweep = 0: forward (colours 0..7), the smoother of the paper (Sec. 3).
 * sweep = 1: backward (colours 7..0), the second half of eq. (2).
 * sweep = 2: symmetric = forward then backward (eqs. (1)-(2), HPCG's smoother).
 * The backward half starts by relaxing colour 7 again with unchanged
 * neighbours; this reproduces the value the forward half gave it, exactly
 * as the two triangular solves of eqs. (1)-(2) do.                          */
void or_gs_c(int nx, int ny, int nz, const double *c27, int sweep, const double *r, double *z)
{
    if (sweep == 0 || sweep == 2)
        for (int c = 0; c < 8; ++c) relax_color(nx, ny, nz, c27, r, z, c);
    if (sweep == 1 || sweep == 2)
        for (int c = 7; c >= 0; --c) relax_color(nx, ny, nz, c27, r, z, c);
}

void or_gs(int nx, int ny, int nz, double beta, int fo, int sweep,
           const double *r, double *z)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
    or_gs_c(nx, ny, nz, c27, sweep, r, z);
}

/* ------------------------------------------------------------------------- */
/* Grid transfers (Sec. 3: injection restriction eq. (3), P = R^T;           */
/* Sec. 3.2 "Fused SpMV-restriction", eqs. (4)-(6)).                          */
/* Coarse point (I,J,K) is fine point (2I,2J,2K): the even-index points.     */
/* Fine dimensions must be even; coarse dimensions are half of them.        */
/* ------------------------------------------------------------------------- */

/* (R v)_i = v_{c_f(i)}, eq. (3). */
void or_inject(int nx, int ny, int nz, const double *v, double *vc)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I)
                vc[lex(cx, cy, I, J, K)] = v[lex(nx, ny, 2 * I, 2 * J, 2 * K)];
}

/* z <- z + P zc with P = R^T: adds each coarse value to its fine point and
 * leaves the other fine points unchanged. */
void or_prolong_add(int nx, int ny, int nz, const double *zc, double *z)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I)
                z[lex(nx, ny, 2 * I, 2 * J, 2 * K)] += zc[lex(cx, cy, I, J, K)];
}

/* Fused residual-restriction, eq. (6):
 * rc_i = r_{f(i)} - sum_j A_{f(i) j} z_j, evaluated only at coarse points.
 * The sum uses the same slot order as or_spmv, so the result equals
 * R (r - A z) computed with or_spmv and or_inject bit for bit.              */
static void restrict_fused_c(int nx, int ny, int nz, const double *c27,
                             const double *r, const double *z, double *rc)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                idx_t f = lex(nx, ny, 2 * I, 2 * J, 2 * K);
                double Az = row_apply(nx, ny, nz, c27, z, 2 * I, 2 * J, 2 * K);
                rc[lex(cx, cy, I, J, K)] = r[f] - Az;
            }
}

void or_restrict_fused(int nx, int ny, int nz, double beta, int fo,
                       const double *r, const double *z, double *rc)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
    restrict_fused_c(nx, ny, nz, c27, r, z, rc);
}

/* ------------------------------------------------------------------------- */
/* Low-precision storage emulation (the argument `f32`, a storage mode).     */
/*   0: everything binary64 (the plain method);                               */
/*   1: every vector element that the mixed-precision method keeps in low    */
/*      precision (Alg. 3, steps in blue) is rounded to binary32 (round to   */
/*      nearest even) when stored; arithmetic stays in binary64.  Stored in  */
/*      binary32: q_1, the multigrid work vectors after every sweep,         */
/*      restriction and correction, z = M^{-1} q_k, w = A z, each            */
/*      Gram-Schmidt update, q_{k+1} and the end-of-cycle u = Q y.  Inner    */
/*      products, H, the rotations and x stay binary64;                      */
/*   2, 3: as 1, but the multigrid work vectors of every level (the V-cycle's */
/*      input, each sweep, restriction and correction, and its output z) are  */
/*      rounded to binary16 (2) or bfloat16 (3) instead: the whole multigrid  */
/*      hierarchy in 16 bits.  The V-cycle is applied to sigma q (q a unit    */
/*      vector, sigma the power of two nearest sqrt(N), so that the entries  */
/*      are of order one, inside binary16's range) and its result divided by */
/*      sigma: w = A z / sigma; at the end of a cycle to sigma u with sigma  */
/*      the power of two nearest sqrt(N) / ||y||, and x += z / sigma.  The    */
/*      powers of two make the scalings exact.                                */
/* Pinned by rebuilding each stored quantity of a cycle from independent     */
/* pieces with the same rounding (tests/test_oracle_pins.py, "storage").     */
/* ------------------------------------------------------------------------- */

/* Round to nearest (ties to even) in a binary format with p significand bits
 * (leading one included), smallest normal exponent emin and largest finite
 * value maxv (IEEE 754): the quantum of x is 2^(e - p + 1) with 2^e the
 * leading bit of |x| (fixed at 2^(emin - p + 1) below the normal range). */
static double round_format(double x, int p, int emin, double maxv)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e); /* |x| = f 2^e, f in [0.5, 1): leading bit 2^(e-1) */
    int lead = e - 1 < emin ? emin : e - 1;
    double r = ldexp(nearbyint(ldexp(x, -(lead - (p - 1)))), lead - (p - 1));
    return fabs(r) > maxv ? copysign(INFINITY, x) : r;
}

static inline double fl32(double v) { return (double)(float)v; }
static inline double fl16(double v) { return round_format(v, 11, -14, 65504.0); }
static inline double flbf16(double v) { return round_format(v, 8, -126, 0x1.fep127); }

/* a stored Krylov quantity (binary32 in every low-precision mode) */
static inline double st(double v, int f32) { return f32 ? fl32(v) : v; }

static void round_vec(double *v, idx_t n, int f32)
{
    if (!f32) return;
#pragma omp parallel for schedule(static)
    for (idx_t i = 0; i < n; ++i) v[i] = fl32(v[i]);
}

/* a stored multigrid work vector */
static inline double st_mg(double v, int mode)
{
    return mode == 1 ? fl32(v) : mode == 2 ? fl16(v) : mode == 3 ? flbf16(v) : v;
}

static void round_mg(double *v, idx_t n, int mode)
{
    if (!mode) return;
#pragma omp parallel for schedule(static)
    for (idx_t i = 0; i < n; ++i) v[i] = st_mg(v[i], mode);
}

static double pow2_near(double v)
{
    if (!(v > 0.0) || !isfinite(v)) return 1.0;
    return ldexp(1.0, (int)nearbyint(log2(v)));
}

/* ------------------------------------------------------------------------- */
/* Geometric multigrid V-cycle (Sec. 2 Fig. 1 two-grid cycle applied          */
/* recursively; Sec. 3: forward GS smoother, injection, P = R^T; coarse      */
/* operators by re-discretising the same stencil on each coarser mesh).      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int levels, pre, post, coarsest, sweep;
    const double *c27;
    int f32;
} mgparam;

/* z <- M^{-1} r on level l with dimensions (nx,ny,nz).  The V-cycle starts
 * from z = 0 on every level (so M^{-1} is a fixed linear operator, as right
 * preconditioning requires).  The defect is d = r - A z (the sign printed in
 * Fig. 1 is read as a typo; eq. (6) has this sign).                         */
static void mg_apply(const mgparam *p, int l, int nx, int ny, int nz,
                     const double *r, double *z)
{
    idx_t n = (idx_t)nx * ny * nz;
    memset(z, 0, (size_t)n * sizeof(double));
    if (l == p->levels - 1) {
        for (int s = 0; s < p->coarsest; ++s) {
            or_gs_c(nx, ny, nz, p->c27, p->sweep, r, z);
            round_mg(z, n, p->f32);
        }
        return;
    }
    for (int s = 0; s < p->pre; ++s) {
        or_gs_c(nx, ny, nz, p->c27, p->sweep, r, z);
        round_mg(z, n, p->f32);
    }
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    idx_t nc = (idx_t)cx * cy * cz;
    double *rc = (double *)malloc((size_t)nc * sizeof(double));
    double *zc = (double *)malloc((size_t)nc * sizeof(double));
    restrict_fused_c(nx, ny, nz, p->c27, r, z, rc);
    round_mg(rc, nc, p->f32);
    mg_apply(p, l + 1, cx, cy, cz, rc, zc);
    or_prolong_add(nx, ny, nz, zc, z);
    round_mg(z, n, p->f32);
    for (int s = 0; s < p->post; ++s) {
        or_gs_c(nx, ny, nz, p->c27, p->sweep, r, z);
        round_mg(z, n, p->f32);
    }
    free(rc);
    free(zc);
}

void or_vcycle(int nx, int ny, int nz, double beta, int fo, int levels, int pre,
               int post, int coarsest, int sweep, int f32, const double *r, double *z)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
    mgparam p = {levels, pre, post, coarsest, sweep, c27, f32};
    mg_apply(&p, 0, nx, ny, nz, r, z);
}

/* The V-cycle for any stencil table (every level uses the same table). */
void or_vcycle_c(int nx, int ny, int nz, const double *c27, int levels, int pre, int post,
                 int coarsest, int sweep, int f32, const double *r, double *z)
{
    mgparam p = {levels, pre, post, coarsest, sweep, c27, f32};
    mg_apply(&p, 0, nx, ny, nz, r, z);
}

/* ------------------------------------------------------------------------- */
/* GMRES-IR with CGS2 and Givens rotations (Alg. 3).                         */
/* ------------------------------------------------------------------------- */
static double dot(const double *a, const double *b, idx_t n)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (idx_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

typedef struct {
    int iters, restarts, converged, breakdown;
    double rho0, final_rel_res, est_rel_res;
} or_stats;

/*
 * Solves A x = b.  x holds the initial guess on entry and the result on exit.
 *   levels >= 1 : right preconditioner M^{-1} = one V-cycle (levels deep);
 *   levels == 0 : no preconditioner (M = I), used by the finite-termination pin.
 *   f32         : storage mode 0..3 (see "Low-precision storage emulation"):
 *                 1 rounds the low-precision quantities of Alg. 3 to
 *                 binary32, 2 / 3 in addition keep the multigrid hierarchy's
 *                 vectors in binary16 / bfloat16.
 * Readings (Alg. 3): rho0 = ||b||; convergence tests are strict "<"; the
 * projected system is solved over the k steps actually taken (the loop may
 * end early); the Givens rotations of earlier columns are applied through
 * temporaries (each rotation uses the not-yet-rotated entries); c_k and s_k
 * are formed from H_kk and H_{k+1,k} before H_kk is overwritten; the basis
 * holds m+1 vectors.  iters counts inner steps summed over restarts.
 * A breakdown (new vector of norm <= 1e-300) ends the cycle: the Krylov space
 * is then invariant and the projected solution is exact.
 * Optional outputs for the first cycle (NULL to skip): Q1 (n x (m+1),
 * column-major), Hbar1 ((m+1) x m column-major, before rotations), y1 (m),
 * k1 = number of steps in that cycle.  hist (length hist_len) receives the
 * estimated relative residual after each inner step.
 */
int or_gmres_ir_c(int nx, int ny, int nz, const double *c27, int levels, int pre,
                  int post, int coarsest, int sweep, int f32, int restart, int max_iters,
                  double tol, const double *b, double *x, or_stats *stats,
                  double *Q1, double *Hbar1, double *y1, int *k1,
                  double *hist, int hist_len)
{
    idx_t n = (idx_t)nx * ny * nz;
    int m = restart;
    mgparam mp = {levels, pre, post, coarsest, sweep, c27, f32};
    memset(stats, 0, sizeof(*stats));
    if (m < 1) return -1;

    double *Q = (double *)malloc((size_t)n * (m + 1) * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *t = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *cs = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *sn = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *y = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    double *hc = (double *)malloc((size_t)(m + 1) * sizeof(double));
    int rc_status = 0;
    if (!Q || !H || !t || !cs || !sn || !y || !r || !z || !hc) { rc_status = -2; goto done; }

    double rho0 = sqrt(dot(b, b, n));
    const double sig = pow2_near(sqrt((double)n)); /* 16-bit hierarchy: V-cycle input scale */
    stats->rho0 = rho0;
    if (rho0 == 0.0) {
        memset(x, 0, (size_t)n * sizeof(double));
        stats->converged = 1;
        goto done;
    }
    int its = 0, first = 1;
    stats->final_rel_res = 1.0;
    for (;;) {
        /* FP64 outer residual (Alg. 3, residual step; required in double). */
        or_spmv_c(nx, ny, nz, c27, x, r);
        for (idx_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double rho = sqrt(dot(r, r, n));
        stats->final_rel_res = rho / rho0;
        if (rho / rho0 < tol) { stats->converged = 1; break; }
        if (its >= max_iters) break;
        if (!isfinite(rho)) { rc_status = -5; break; }

        for (idx_t i = 0; i < n; ++i) Q[i] = st(r[i] / rho, f32);
        memset(t, 0, (size_t)(m + 1) * sizeof(double));
        memset(H, 0, (size_t)(m + 1) * m * sizeof(double));
        t[0] = rho;
        int kk = 0;
        for (int k = 0; k < m; ++k) {
            if (rho / rho0 < tol) break;
            double *qk = Q + (size_t)k * n, *w = Q + (size_t)(k + 1) * n;
            /* z = M^{-1} q_k ; w = A z */
            if (f32 >= 2 && levels >= 1) {
                /* 16-bit hierarchy: the cycle runs on sigma q_k */
                for (idx_t i = 0; i < n; ++i) r[i] = st_mg(sig * qk[i], f32);
                mg_apply(&mp, 0, nx, ny, nz, r, z);
                or_spmv_c(nx, ny, nz, c27, z, w);
                for (idx_t i = 0; i < n; ++i) w[i] = fl32(w[i] / sig);
            } else {
                if (levels >= 1) mg_apply(&mp, 0, nx, ny, nz, qk, z);
                else memcpy(z, qk, (size_t)n * sizeof(double));
                round_vec(z, n, f32);
                or_spmv_c(nx, ny, nz, c27, z, w);
                round_vec(w, n, f32);
            }
            /* CGS2: two classical Gram-Schmidt passes, H(1:k,k) = h1 + h2. */
            for (int j = 0; j <= k; ++j) H[(size_t)k * (m + 1) + j] = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int j = 0; j <= k; ++j) hc[j] = dot(Q + (size_t)j * n, w, n);
#pragma omp parallel for schedule(static)
                for (idx_t i = 0; i < n; ++i) {
                    double acc = w[i];
                    for (int j = 0; j <= k; ++j) acc -= Q[(size_t)j * n + i] * hc[j];
                    w[i] = st(acc, f32);
                }
                for (int j = 0; j <= k; ++j) H[(size_t)k * (m + 1) + j] += hc[j];
            }
            double bet = sqrt(dot(w, w, n));
            H[(size_t)k * (m + 1) + k + 1] = bet;
            if (first && Hbar1)
                for (int j = 0; j <= k + 1; ++j) Hbar1[(size_t)k * (m + 1) + j] = H[(size_t)k * (m + 1) + j];
            int brk = !(bet > 1e-300);
            if (!brk)
                for (idx_t i = 0; i < n; ++i) w[i] = st(w[i] / bet, f32);
            /* Givens: rotate column k by the earlier rotations, then form the
             * rotation that annihilates H(k+1,k). */
            double *hk = H + (size_t)k * (m + 1);
            for (int j = 0; j < k; ++j) {
                double a = hk[j], bb = hk[j + 1];
                hk[j] = cs[j] * a + sn[j] * bb;
                hk[j + 1] = -sn[j] * a + cs[j] * bb;
            }
            double mu = sqrt(hk[k] * hk[k] + hk[k + 1] * hk[k + 1]);
            cs[k] = hk[k] / mu;
            sn[k] = hk[k + 1] / mu;
            hk[k] = mu;
            hk[k + 1] = 0.0;
            t[k + 1] = -sn[k] * t[k];
            t[k] = cs[k] * t[k];
            rho = fabs(t[k + 1]);
            kk = k + 1;
            ++its;
            if (hist && its - 1 < hist_len) hist[its - 1] = rho / rho0;
            stats->est_rel_res = rho / rho0;
            if (brk) { stats->breakdown = 1; break; }
            if (its >= max_iters) break;
        }
        /* y = H(1:kk,1:kk)^{-1} t(1:kk) by back substitution. */
        for (int i = kk - 1; i >= 0; --i) {
            double acc = t[i];
            for (int j = i + 1; j < kk; ++j) acc -= H[(size_t)j * (m + 1) + i] * y[j];
            y[i] = acc / H[(size_t)i * (m + 1) + i];
        }
        if (first) {
            if (Q1) memcpy(Q1, Q, (size_t)n * (kk + 1) * sizeof(double));
            if (y1) memcpy(y1, y, (size_t)kk * sizeof(double));
            if (k1) *k1 = kk;
            first = 0;
        }
        /* u = Q y ; x <- x + M^{-1} u (the update itself in FP64). */
#pragma omp parallel for schedule(static)
        for (idx_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < kk; ++j) acc += Q[(size_t)j * n + i] * y[j];
            r[i] = st(acc, f32);
        }
        if (f32 >= 2 && levels >= 1) {
            double y2 = 0.0;
            for (int j = 0; j < kk; ++j) y2 += y[j] * y[j];
            const double su = pow2_near(sqrt((double)n) / sqrt(y2));
            for (idx_t i = 0; i < n; ++i) r[i] = st_mg(su * r[i], f32);
            mg_apply(&mp, 0, nx, ny, nz, r, z);
            for (idx_t i = 0; i < n; ++i) x[i] += z[i] / su;
        } else {
            if (levels >= 1) mg_apply(&mp, 0, nx, ny, nz, r, z);
            else memcpy(z, r, (size_t)n * sizeof(double));
            round_vec(z, n, f32);
            for (idx_t i = 0; i < n; ++i) x[i] += z[i];
        }
        stats->restarts += 1;
    }
    stats->iters = its;
done:
    free(Q); free(H); free(t); free(cs); free(sn); free(y); free(r); free(z); free(hc);
    return rc_status;
}

int or_gmres_ir(int nx, int ny, int nz, double beta, int fo, int levels, int pre,
                int post, int coarsest, int sweep, int f32, int restart, int max_iters,
                double tol, const double *b, double *x, or_stats *stats,
                double *Q1, double *Hbar1, double *y1, int *k1,
                double *hist, int hist_len)
{
    double c27[27];
    or_stencil_from_beta(beta, fo, c27);
    return or_gmres_ir_c(nx, ny, nz, c27, levels, pre, post, coarsest, sweep, f32, restart,
                         max_iters, tol, b, x, stats, Q1, Hbar1, y1, k1, hist, hist_len);
}

/* Adjoint quantities for a stencil parameterised by its 27 entries (the
 * gradient of a loss through x = A^{-1} b): for each offset s,
 * out[s] = sum over rows i with neighbour i+d_s inside the grid of
 * lam_i * x_{i+d_s}.  The gradient of L with respect to entry s is -out[s]
 * when lam solves A^T lam = dL/dx. */
void or_stencil_correlation(int nx, int ny, int nz, const double *lam, const double *x,
                            double *out27)
{
    for (int s = 0; s < 27; ++s) {
        int di = s % 3 - 1, dj = (s / 3) % 3 - 1, dk = s / 9 - 1;
        double acc = 0.0;
#pragma omp parallel for collapse(2) reduction(+ : acc) schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                    acc += lam[lex(nx, ny, i, j, k)] * x[lex(nx, ny, ii, jj, kk)];
                }
        out27[s] = acc;
    }
}
