// Internal declarations of the hpgmx library (gfx950 HIP).
//
// Data layout in HBM (per multigrid level):
//  * Rows are stored in a colour-blocked order.  The 8 colours of the
//    multicolour Gauss-Seidel smoother (Sec. 3.2) are the 8 parity classes of
//    (i, j, k); colour c = (i&1) + 2(j&1) + 4((k+1)&1), so the class of
//    all-even points -- the injection points of the restriction, eq. (3) --
//    is colour 4.  Each colour is one contiguous block, lexicographic in
//    (i>>1, j>>1, k>>1) inside the block.  A colour launch therefore streams
//    a contiguous slice of every array, every stencil neighbour of a row sits
//    at a regular offset in another block (gathers stay coalesced across a
//    wavefront), and the colour-4 block of a fine level is exactly the coarse
//    level in its natural order.
//  * The matrix is ELLPACK (Sec. 3.2) with the diagonal split off: 26
//    off-diagonal slots (layout: see ell_row) plus a diagonal array.  Rows
//    with fewer neighbours pad with value 0 and column N: every vector the
//    kernels gather from holds N + 1 entries and keeps entry N at zero, so a
//    padded slot contributes 0 * 0 whatever the rest of the vector holds.
//    Column indices are shared by all value precisions (FP64, FP32, FP16,
//    BF16): int32 (the default), or compressed to 16-bit offsets (see
//    ColMap), chosen per handle before the hierarchy is built.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hpgmx.h"

namespace hpgmx {

using i64 = long long;

constexpr int kSlots = 26;        // off-diagonal ELL slots
constexpr int kMaxLevels = 8;
constexpr int kMaxRestart = 63;   // m; the basis holds m + 1 vectors
constexpr int kMaxBasis = 64;     // kMaxRestart + 1
constexpr int kBlock = 256;       // threads per workgroup (4 wavefronts)
constexpr int kMaxBatch = 8;      // right-hand sides of one batched solve
constexpr int kMaxRedBlocks = 1024;  // workgroups of the grid-stride reductions
constexpr int kDefaultEllChunkLog2 = 8;  // ELL chunking default (see ell_row)
// Extra elements between Krylov basis columns, so that columns do not start
// on the same large power-of-two boundary (DRAM channel/bank aliasing).
constexpr int kDefaultLdqPad = 1088;
// Tile orders of the row-per-lane launches: 0 the launch order, 1 each XCD
// owns one contiguous range of tiles; for the full-grid SpMV also
// kRemapSlab (see slab_perm) or kRemapPlanes (see plane_row); for a launch
// over the whole rows of a colour pair, kRemapPlanePair (see
// plane_pair_row).
constexpr int kRemapSlab = 2;
constexpr int kRemapPlanes = 3;
constexpr int kRemapPlanePair = 4;
constexpr long long kDefaultPairRows = 1 << 17;

// Data layout and tile order of a handle.  The defaults are the tuned
// ones; hpgmx_set_layout changes them for layout studies and tests.
struct Layout {
    int order = kRemapSlab;
    int clog2 = kDefaultEllChunkLog2;  // ELL chunking (see ell_row)
    int ldq_pad = kDefaultLdqPad;      // elements between Krylov basis columns
    // Sweeps from a zero guess relax two colours per launch on levels with
    // at most this many rows per colour (launch_gs_pair_zero).
    long long pair_rows = kDefaultPairRows;
};

using bf16 = __hip_bfloat16;

// Colour-blocked geometry of one level.
struct Geom {
    int nx, ny, nz;
    int bx[8], by[8], bz[8];  // block extents per colour
    i64 off[9];               // block offsets; off[8] = N
    i64 N;
};

__host__ __device__ inline int colour_of(int i, int j, int k)
{
    return (i & 1) + 2 * (j & 1) + 4 * ((k + 1) & 1);
}

__host__ __device__ inline i64 to_internal(const Geom &g, int i, int j, int k)
{
    const int c = colour_of(i, j, k);
    return g.off[c] + (i >> 1) + (i64)g.bx[c] * ((j >> 1) + (i64)g.by[c] * (k >> 1));
}

__host__ __device__ inline void from_internal(const Geom &g, i64 p, int &i, int &j, int &k)
{
    int c = 0;
    while (c < 7 && p >= g.off[c + 1]) ++c;
    const i64 q = p - g.off[c];
    const int ii = (int)(q % g.bx[c]);
    const int jj = (int)((q / g.bx[c]) % g.by[c]);
    const int kk = (int)(q / ((i64)g.bx[c] * g.by[c]));
    i = 2 * ii + (c & 1);
    j = 2 * jj + ((c >> 1) & 1);
    k = 2 * kk + (((c >> 2) & 1) ^ 1);
}

Geom make_geom(int nx, int ny, int nz);

// Neighbour colour of slot s for a row of colour c (slot s enumerates the 26
// off-diagonal offsets (di,dj,dk) in the order dk, dj, di = -1..1 with the
// centre skipped).
__host__ __device__ inline void slot_offset(int s, int &di, int &dj, int &dk)
{
    const int t = s < 13 ? s : s + 1;
    di = t % 3 - 1;
    dj = (t / 3) % 3 - 1;
    dk = t / 9 - 1;
}

// Bit s set when slot s of a colour-c row couples to a colour relaxed before c
// in the given direction (forward: lower colour index first).
__host__ __device__ constexpr unsigned zero_guess_mask(int c, bool forward)
{
    unsigned m = 0;
    for (int s = 0; s < kSlots; ++s) {
        const int t = s < 13 ? s : s + 1;
        const int di = t % 3 - 1, dj = (t / 3) % 3 - 1, dk = t / 9 - 1;
        const int flip = (di & 1) | ((dj & 1) << 1) | ((dk & 1) << 2);
        const int cn = c ^ flip;
        if (forward ? cn < c : cn > c) m |= 1u << s;
    }
    return m;
}

// Gauss-Seidel colour-pass modes.
constexpr int kGsFull = 0;          // every slot
constexpr int kGsZeroForward = 1;   // forward sweep from z = 0
constexpr int kGsZeroBackward = 2;  // backward sweep from z = 0

// Position of slot s of row p in the ELL arrays.  clog2 = 0: slot-major over
// the whole matrix ([s*N + p]).  clog2 > 0: rows are grouped in chunks of
// C = 2^clog2 and each chunk is slot-major on its own (SELL-C with sigma = 1):
// a wavefront's 26 slots then lie in one contiguous 26*C-entry region.
// The 16-bit column offsets are stored in pairs: slots 2t and 2t + 1 of a
// row share one 32-bit word (low half slot 2t), the 13 pair words laid out
// as the values (pbase + t * pstride), so a row's offsets take 13 loads.
constexpr int kPairs = kSlots / 2;
struct EllRow {
    i64 base, stride;    // values: slot s at base + s * stride
    i64 pbase, pstride;  // offset pairs: pair t at pbase + t * pstride (32-bit words)
};
__host__ __device__ inline EllRow ell_row(i64 p, i64 N, int clog2)
{
    if (clog2 == 0) return {p, N, p, N};
    const i64 lane = p & ((1ll << clog2) - 1), chunk = p >> clog2;
    return {chunk * ((i64)kSlots << clog2) + lane, 1ll << clog2, chunk * ((i64)kPairs << clog2) + lane,
            1ll << clog2};
}
// Entries each off-diagonal ELL array holds (the last chunk is padded).
__host__ __device__ inline i64 ell_entries(i64 N, int clog2)
{
    if (clog2 == 0) return (i64)kSlots * N;
    const i64 C = 1ll << clog2;
    return (i64)kSlots * ((N + C - 1) / C) * C;
}

// Compressed column indices (optional).  Slot s of row p, a row of colour c,
// stores the 16-bit offset d = col - p - D[c][s] with D a per-matrix table of
// 8 x 26 column offsets (the offsets of an interior row of that colour); a
// padded slot stores kPadOffset and reads column N.  Any matrix whose
// offsets all fit 16 bits is stored exactly (mg_setup checks every entry and
// fails otherwise).  This halves the index bytes of every ELL pass, which
// are 104 of the 224 bytes of an FP32 Gauss-Seidel row with int32 indices.
constexpr int kPadOffset = -32768;
constexpr int kColMapSize = 8 * kSlots;
struct ColMap {
    int d[8][kSlots];
};
ColMap make_colmap(const Geom &g);

struct Matrix {
    Geom g;
    int clog2 = 0;         // ELL chunking (see ell_row)
    int order = kRemapSlab;   // tile order of its launches (Layout::order)
    bool c16 = false;         // column format: int32 indices, or 16-bit offsets
    void *col = nullptr;      // int32 [laid out as the values], or 16-bit offset pairs (see ell_row)
    int *cmap = nullptr;      // the ColMap D[c][s] on the device (16-bit offsets)
    double *v64 = nullptr, *d64 = nullptr;
    float *v32 = nullptr, *d32 = nullptr;
    __half *v16 = nullptr, *d16 = nullptr;
    bf16 *vb16 = nullptr, *db16 = nullptr;
};

// Precision of a call.  Matrix values: double (P64), float (P32), __half
// (P16, P16V) or bf16 (PB16, PB16V).  Multigrid vectors: double for P64,
// float for P32, P16 and PB16, and the 16-bit type of the matrix for P16V and
// PB16V (the whole hierarchy in 16 bits).  Arithmetic is FP64 for P64 and
// FP32 otherwise; the Krylov basis is FP64 for P64 and FP32 otherwise.
enum Prec {
    P64 = HPGMX_F64, P32 = HPGMX_F32, P16 = HPGMX_F16, PB16 = HPGMX_BF16,
    P16V = HPGMX_F16_MG, PB16V = HPGMX_BF16_MG
};
constexpr int kNumPrec = 6;
inline bool mg16(Prec p) { return p == P16V || p == PB16V; }
// Multigrid vector bytes.
inline size_t vec_bytes(Prec p) { return p == P64 ? 8 : mg16(p) ? 2 : 4; }
// Precision of the Krylov vectors (basis, u) and of the kernels on them.
inline Prec basis_prec(Prec p) { return p == P64 ? P64 : P32; }
// Which value array of the matrix a precision reads.
inline Prec matrix_prec(Prec p) { return p == P16V ? P16 : p == PB16V ? PB16 : p; }

// Device-side control block of one Krylov cycle (FP64): Hessenberg matrix
// (rotated) and its unrotated copy, Givens rotations, right-hand side t,
// projected solution y, CGS2 coefficients and scalars.
//
// Basis columns are stored unnormalised: column j holds w_j, and the basis
// vector of Alg. 3 is q_j = colscale[j] * w_j (colscale[0] = 1, since q_1 is
// cast already divided by rho; colscale[j+1] = 1 / ||w_{j+1}|| from the
// Givens step).  Every consumer applies the scale: the SpMV of the step
// multiplies its output by the scale of the column it was fed, the inner
// products and the staged CGS2 / basis-combination coefficients carry it.
// In exact arithmetic this is Alg. 3; it saves the normalisation pass (a
// read and a write of one vector per step).
struct Ctrl {
    double H[kMaxBasis * kMaxRestart];
    double Hbar[kMaxBasis * kMaxRestart];
    double t[kMaxBasis], cs[kMaxBasis], sn[kMaxBasis], y[kMaxBasis];
    double h1[kMaxBasis], h2[kMaxBasis];
    double colscale[kMaxBasis];
    // scalars read back by the host after every inner step (keep together)
    double rho, inv_rho, beta, inv_beta, nrm2, rho0;
    int breakdown, nonfinite;
    double corr[27];  // stencil correlation of the adjoint gradient
    // 16-bit multigrid hierarchy (P16V, PB16V): the V-cycle's input is the
    // Krylov vector times a power of two sigma that brings its entries near
    // 1 in magnitude (binary16's range); the consumers undo sigma.
    double mg_post;   // SpMV output scale of the inner step: colscale[k] / sigma
    double mg_inv;    // 1 / sigma of the end-of-cycle V-cycle (the update)
};

// What the finish kernel of a reduction does with the summed partials.
constexpr int kFinishH1 = 0;          // h1 = Q^T w
constexpr int kFinishH2 = 1;          // h2 = Q^T w (reorthogonalisation)
constexpr int kFinishNormGivens = 2;  // ||w||^2, then the Givens step of column k
constexpr int kFinishResid = 3;       // rho = ||b - A x||, start of a cycle
constexpr int kFinishRho0 = 4;        // rho0 = ||b||
constexpr int kFinishCorr = 5;        // the 27 stencil correlations

// ---- launchers (stream-ordered) -------------------------------------------
// The operator's 27 stencil entries in slot order t = 9(dk+1) + 3(dj+1) + (di+1)
// (t = 13 is the diagonal), passed to kernels by value.
struct Stencil {
    double c[27];
};
Stencil stencil_from_beta(double beta);
// Writes the values of the precisions A has arrays for and, if A.col is set,
// the column offsets (A.cmap must hold make_colmap(A.g)); an offset that does
// not fit 16 bits sets *overflow (device int, may be null if A.col is null).
void launch_generate(const Matrix &A, const Stencil &st, int *overflow, hipStream_t s);
// out[t] = sum over rows of lam_p * x_{neighbour t of p} (x, lam in internal
// order, x gathered with its zero entry at N); `partials` as for the
// Krylov reductions.
void launch_stencil_correlation(const Matrix &A, const double *lam, const double *x,
                                double *partials, Ctrl *ctrl, hipStream_t s);
// The same correlations from lam and x in the natural order, with the
// per-workgroup partial sums in a fixed device array of this library
// (noalloc_scratch_bytes() bytes per device; noalloc_setup(device) must have
// run with `device` current).  Allocates nothing.
hipError_t noalloc_setup(int device);
size_t noalloc_scratch_bytes();
void launch_stencil_correlation_noalloc(int device, const Geom &g, const double *lam, const double *x,
                                        double *out27, hipStream_t s);
void launch_nat2int(const Geom &g, Prec src, const void *nat, Prec dst, void *in, hipStream_t s);
void launch_int2nat(const Geom &g, Prec src, const void *in, Prec dst, void *nat, hipStream_t s);
// y = A x; with ctrl, y = (A x) * ctrl->colscale[k] (the SpMV of inner step
// k, fed with the unnormalised basis column k), or for the 16-bit hierarchy
// y = (A x) * ctrl->mg_post.  x in the multigrid vector type of p, y in the
// Krylov type (FP32 for the 16-bit hierarchy).
// With skip = 0 or 7 the rows of that colour are left out (they come from the
// last colour launch of the V-cycle, see SpmvOut).
void launch_spmv(const Matrix &A, Prec p, const void *x, void *y, hipStream_t s,
                 const Ctrl *ctrl = nullptr, int k = 0, int skip = -1);
// The scale launch_spmv applies to its output (null without ctrl).
const double *spmv_scale(Prec p, const Ctrl *ctrl, int k);
// The SpMV after a V-cycle whose last level-0 sweep (direction `forward`)
// wrote the rows of its last colour (7 forward, 0 backward) and, for the
// colours at sweep positions 2-6, the partial sums `part` (fused = true);
// the rows of those colours are (A z)_p = a_pp z_p + (part_p + the sum over
// the remaining slots).  With fused = false the same values are formed from z
// alone (part unused) and the last colour's rows are computed too.
void launch_spmv_split(const Matrix &A, Prec p, const void *x, void *y, const void *part, bool forward,
                       bool fused, hipStream_t s, const Ctrl *ctrl, int k);
// What a Gauss-Seidel colour launch of the last level-0 sweep writes for the
// SpMV that follows: with w, the SpMV rows of its colour (y of launch_spmv,
// Krylov type, and its scale); with part, the partial sums of its rows over
// the slots to colours relaxed before it in direction `forward` (Krylov
// type, indexed by row; see launch_spmv_split).  Neither: nothing.
struct SpmvOut {
    void *w = nullptr;
    const double *scale = nullptr;
    void *part = nullptr;
    bool forward = true;
};
// One colour of a Gauss-Seidel sweep: rows of colour c, slots per `mode`.
// With out.w (full mode only) the launch also writes (A z)_p for the rows of
// its colour, valid when every neighbour of the colour is final (the last
// colour launch of a V-cycle).
void launch_gs_colour(const Matrix &A, Prec p, int c, int mode, const void *r, void *z,
                      hipStream_t s, SpmvOut out = {});
// Colours a and a ^ 1 of a sweep from a zero guess in one launch (a even
// for a forward sweep, odd for a backward one); same result bit for bit.
// Needs gs_pair_possible(A) (equal blocks: an even x extent).
void launch_gs_pair_zero(const Matrix &A, Prec p, int a, bool forward, const void *r, void *z,
                         hipStream_t s);
bool gs_pair_possible(const Matrix &A);
void launch_restrict(const Matrix &Af, const Geom &gc, Prec p, const void *r, const void *z,
                     void *rc, hipStream_t s);
// The same result when z is the outcome of a single Gauss-Seidel sweep from
// z = 0 in direction `forward` (see k_restrict_after_sweep): reads only the
// slots of the injection rows that couple to colours relaxed after colour 4.
void launch_restrict_after_sweep(const Matrix &Af, const Geom &gc, Prec p, bool forward, const void *z,
                                 void *rc, hipStream_t s);
void launch_prolong(const Geom &gf, const Geom &gc, Prec p, const void *zc, void *z,
                    hipStream_t s);

// Krylov kernels.  Q is column-major with leading dimension ldq >= N.
//
// The vector kernels take M elements of K interleaved right-hand sides
// (M = rows * K; element e is row e / K of right-hand side e % K) and one
// control block per right-hand side (ctrl[0..K)).  K is 1 for the single
// solve and 2, 4 or 8 for a batch; a column of a batched basis holds M
// elements.
int red_blocks(i64 N);
// The finish kernel: one workgroup per right-hand side adds partial columns
// i * K + j (i < kb) over nb workgroups and applies `mode` to ctrl[j].
void launch_finish(const double *partials, int nb, int kb, int K, int mode, Ctrl *ctrl, int k, int m,
                   hipStream_t s);
// Profiling of the reduction passes: when set (on the calling host thread),
// launch_finish calls finish_hook(finish_hook_arg) before it enqueues the
// finish kernel, so that a pass and its finish kernel can be timed apart.
extern thread_local void (*finish_hook)(void *);
extern thread_local void *finish_hook_arg;
// h1 = Q^T w alone (the first GEMVT when the SpMV runs as its own kernel).
void launch_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, const void *w, double *partials,
                Ctrl *ctrl, hipStream_t s);
// h2 = Q^T (w - Q h1); w is not written.
void launch_cgs_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                    Ctrl *ctrl, hipStream_t s);
// w <- w - Q (h1 + h2), ||w||^2 and the Givens step of column k.
void launch_cgs_norm(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                     Ctrl *ctrl, int k, int m, hipStream_t s);
void launch_resid64(const Matrix &A, const double *x, const double *b, double *r,
                    double *partials, Ctrl *ctrl, int m, hipStream_t s);
// ||v_j||^2 per right-hand side, then the finish `mode` (kFinishRho0 or
// kFinishResid with restart length m).
void launch_norm64(i64 M, int K, const double *v, double *partials, Ctrl *ctrl, int mode, int m,
                   hipStream_t s);
void launch_cast(i64 M, int K, Prec p, const double *r, const Ctrl *ctrl, void *q, hipStream_t s);
// Completed Krylov steps per right-hand side (the size of each back-solve).
struct KCount {
    int v[kMaxBatch];
};
void launch_trsm(Ctrl *ctrl, const KCount &kc, int K, int m, hipStream_t s);
void launch_gemv(i64 M, int K, Prec p, const void *Q, i64 ldq, int kk, const Ctrl *ctrl, void *u,
                 hipStream_t s);
// x += z in FP64 (z in the multigrid vector type of p); for the 16-bit
// hierarchy x += z * ctrl->mg_inv.
void launch_update(i64 M, Prec p, const void *z, double *x, hipStream_t s, const Ctrl *ctrl = nullptr);
// The V-cycle input of the 16-bit hierarchy: r0 = sigma * v rounded to the
// 16-bit type of p, with v an FP32 Krylov vector and sigma a power of two.
// end_of_cycle = false: v is basis column k (norm 1 / colscale[k]), sigma is
// the power of two nearest sqrt(N) colscale[k], and ctrl->mg_post =
// colscale[k] / sigma.  end_of_cycle = true: v = Q y (norm about ||y||,
// y = ctrl->y[0..kk)), sigma the power of two nearest sqrt(N) / ||y||, and
// ctrl->mg_inv = 1 / sigma.
void launch_cast_mg(i64 N, Prec p, const float *v, Ctrl *ctrl, bool end_of_cycle, int k, void *r0,
                    hipStream_t s);
void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// ---- batched stencil kernels (K interleaved right-hand sides, K = 2, 4, 8) ----
// Vectors hold N * K entries ([p * K + j]); a vector that is gathered from
// holds (N + 1) * K with row N zero.  R right-hand sides per lane (R divides
// K): the tile shape chosen per kernel and level by the autotuner.  p is the
// matrix precision (vectors FP64 for P64, FP32 otherwise).
bool batch_shape_ok(int K, int R);
// Y = A X; with ctrl, vector j is scaled by ctrl[j].colscale[k].
void launch_bspmv(const Matrix &A, Prec p, int K, int R, const void *x, void *y, hipStream_t s,
                  const Ctrl *ctrl = nullptr, int k = 0);
// What a batched colour launch of the last level-0 sweep writes for the
// batched SpMV (as SpmvOut, K interleaved right-hand sides): with y, the
// SpMV rows of its colour, right-hand side j scaled by ctrl[j].colscale[k];
// with part, the partial sums over the slots to colours relaxed before it.
struct BSpmvOut {
    void *y = nullptr;
    const Ctrl *ctrl = nullptr;
    int k = 0;
    void *part = nullptr;
    bool forward = true;
};
void launch_bgs_colour(const Matrix &A, Prec p, int K, int R, int c, int mode, const void *r,
                       void *z, hipStream_t s, BSpmvOut out = {});
// launch_spmv_split for K interleaved right-hand sides (the batched solver).
void launch_bspmv_split(const Matrix &A, Prec p, int K, int R, const void *x, void *y, const void *part,
                        bool forward, bool fused, hipStream_t s, const Ctrl *ctrl, int k);
void launch_brestrict(const Matrix &Af, const Geom &gc, Prec p, int K, int R, const void *r,
                      const void *z, void *rc, hipStream_t s);
void launch_brestrict_after_sweep(const Matrix &Af, const Geom &gc, Prec p, int K, int R, bool forward,
                                  const void *z, void *rc, hipStream_t s);
void launch_bprolong(const Geom &gf, const Geom &gc, Prec p, int K, const void *zc, void *z,
                     hipStream_t s);
// r = b - A x in FP64 for K right-hand sides, then rho_j = ||r_j|| into
// ctrl[j] (start of a cycle, as launch_resid64) by the norm kernel.
void launch_bresid64(const Matrix &A, int K, int R, const double *x, const double *b, double *r,
                     double *partials, Ctrl *ctrl, int m, hipStream_t s);
// [nrhs][N] natural order <-> [N][K] colour-blocked interleaved (right-hand
// sides nrhs..K-1 are zero-filled on the way in and dropped on the way out).
void launch_bnat2int(const Geom &g, Prec src, Prec dst, int K, int nrhs, const void *nat, void *in,
                     hipStream_t s);
void launch_bint2nat(const Geom &g, Prec src, Prec dst, int K, int nrhs, const void *in, void *nat,
                     hipStream_t s);

}  // namespace hpgmx
