// Stencil-side kernels: matrix generation, ordering permutations, ELL SpMV,
// one colour of a multicolour Gauss-Seidel sweep, fused residual-restriction
// and prolongation-correction.  All are HBM-bandwidth bound (no dense
// contraction anywhere), so they are written for coalesced streaming: one
// row per lane, slot-major ELL arrays read with non-temporal loads (each
// matrix entry is used once per launch) and vector entries gathered through
// the caches (each is reused by up to 26 rows).
#include "ell_device.hpp"

#include <cstdlib>
#include <stdexcept>
#include <type_traits>

namespace hpgmx {

static bool even_extents(const Geom &g) { return g.nx % 2 == 0 && g.ny % 2 == 0 && g.nz % 2 == 0; }

int plane_order(const Matrix &A)
{
    return even_extents(A.g) && A.g.N < (1LL << 32) ? kRemapPlanes : 1;
}

int full_grid_order(const Matrix &A, int lanes)
{
    if (A.order < kRemapSlab) return A.order != 0 ? 1 : 0;
    const Geom &g = A.g;
    const bool even = even_extents(g);
    if (A.order == kRemapPlanes) return plane_order(A);
    const i64 lanes_total = g.N * lanes;
    const bool whole = lanes_total % ((i64)kBlock * kXcds * kXcds) == 0;
    return even && whole ? kRemapSlab : 1;
}

// ---- geometry -----------------------------------------------------------------
Geom make_geom(int nx, int ny, int nz)
{
    Geom g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    i64 o = 0;
    for (int c = 0; c < 8; ++c) {
        const int pi = c & 1, pj = (c >> 1) & 1, pk = ((c >> 2) & 1) ^ 1;
        g.bx[c] = (nx - pi + 1) / 2;
        g.by[c] = (ny - pj + 1) / 2;
        g.bz[c] = (nz - pk + 1) / 2;
        g.off[c] = o;
        o += (i64)g.bx[c] * g.by[c] * g.bz[c];
    }
    g.off[8] = o;
    g.N = o;
    return g;
}

// ---- generation -----------------------------------------------------------------
// The 27-point operator of Sec. 2 / Sec. 3: 26 on the diagonal, -1 off it,
// with the x-neighbour entries shifted to -1-beta (i-1) and -1+beta (i+1).
Stencil stencil_from_beta(double beta)
{
    Stencil st{};
    for (int t = 0; t < 27; ++t) {
        const int di = t % 3 - 1, dj = (t / 3) % 3 - 1, dk = t / 9 - 1;
        double a = -1.0;
        if (di == 0 && dj == 0 && dk == 0) a = 26.0;
        else if (di < 0) a = -1.0 - beta;
        else if (di > 0) a = -1.0 + beta;
        st.c[t] = a;
    }
    return st;
}

// IEEE round-to-nearest-even of x to a binary format with p significand bits
// (the leading one included), smallest normal exponent emin and largest
// finite value maxv, in one step from FP64: the value is scaled so that the
// format's last significand bit (fixed at 2^(emin-p+1) below the normal
// range) becomes the unit, rounded to an integer with ties to even, and
// scaled back; a value that rounds above maxv overflows to infinity.  The
// result is exactly representable in the format (and in FP32), so the
// conversions that store it are exact and the entry is rounded once.
__device__ double round_to_format(double x, int p, int emin, double maxv)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);  // |x| = f 2^e with f in [0.5, 1): leading bit 2^(e-1)
    const int lead = e - 1 < emin ? emin : e - 1;
    const int q = lead - (p - 1);
    const double r = ldexp(rint(ldexp(x, -q)), q);
    return fabs(r) > maxv ? copysign(INFINITY, x) : r;
}
__device__ __half to_half_rne(double x) { return __float2half((float)round_to_format(x, 11, -14, 65504.0)); }
__device__ bf16 to_bf16_rne(double x)
{
    return __float2bfloat16((float)round_to_format(x, 8, -126, 3.3895313892515355e38));
}

// Column-offset table of a geometry (see ColMap): for each colour, the
// offsets col - p of an interior row of that colour (every row of that colour
// in a grid of even extents); 0 where the colour has no interior row.
ColMap make_colmap(const Geom &g)
{
    ColMap m{};
    for (int c = 0; c < 8; ++c) {
        const int i0 = (c & 1) ? 1 : 2, j0 = ((c >> 1) & 1) ? 1 : 2, k0 = (((c >> 2) & 1) ^ 1) ? 1 : 2;
        if (i0 + 1 >= g.nx || j0 + 1 >= g.ny || k0 + 1 >= g.nz) continue;
        const i64 p0 = to_internal(g, i0, j0, k0);
        for (int s = 0; s < kSlots; ++s) {
            int di, dj, dk;
            slot_offset(s, di, dj, dk);
            m.d[c][s] = (int)(to_internal(g, i0 + di, j0 + dj, k0 + dk) - p0);
        }
    }
    return m;
}

__global__ __launch_bounds__(kBlock) void k_generate(Geom g, int clog2, Stencil st, void *col, int c16,
                                                     const int *__restrict__ cmap, int *overflow, double *v64,
                                                     double *d64, float *v32, float *d32,
                                                     __half *v16, __half *d16, bf16 *vb16,
                                                     bf16 *db16)
{
    const i64 p = gtid();
    if (p >= g.N) return;
    int i, j, k;
    from_internal(g, p, i, j, k);
    const i64 N = g.N;
    const int c = colour_of(i, j, k);
    const EllRow er = ell_row(p, N, clog2);
    for (int s = 0; s < kSlots; ++s) {
        int di, dj, dk;
        slot_offset(s, di, dj, dk);
        const int ii = i + di, jj = j + dj, kk = k + dk;
        const bool in = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
        const double a = in ? st.c[9 * (dk + 1) + 3 * (dj + 1) + (di + 1)] : 0.0;
        const i64 e = er.base + (i64)s * er.stride;
        if (col && !c16) static_cast<int *>(col)[e] = in ? (int)to_internal(g, ii, jj, kk) : (int)N;
        if (col && c16) {
            short o = (short)kPadOffset;
            if (in) {
                const i64 d = to_internal(g, ii, jj, kk) - p - cmap[c * kSlots + s];
                if (d < -32767 || d > 32767) atomicOr(overflow, 1);
                else o = (short)d;
            }
            // slot s is the low (even s) or high half of pair word s / 2
            static_cast<short *>(col)[2 * (er.pbase + (i64)(s >> 1) * er.pstride) + (s & 1)] = o;
        }
        if (v64) v64[e] = a;
        if (v32) v32[e] = (float)a;
        if (v16) v16[e] = to_half_rne(a);
        if (vb16) vb16[e] = to_bf16_rne(a);
    }
    const double dg = st.c[13];
    if (d64) d64[p] = dg;
    if (d32) d32[p] = (float)dg;
    if (d16) d16[p] = to_half_rne(dg);
    if (db16) db16[p] = to_bf16_rne(dg);
}

void launch_generate(const Matrix &A, const Stencil &st, int *overflow, hipStream_t s)
{
    if (A.col && A.c16 && (!A.cmap || !overflow))
        throw std::runtime_error("launch_generate: column map or flag missing");
    hipLaunchKernelGGL(k_generate, dim3(grid_for(A.g.N)), dim3(kBlock), 0, s, A.g, A.clog2, st, A.col, (int)A.c16,
                       A.cmap, overflow, A.v64, A.d64, A.v32, A.d32, A.v16, A.d16, A.vb16, A.db16);
    HPGMX_LAUNCH_CHECK();
}

// ---- natural <-> colour-blocked order ---------------------------------------------
// Element conversions between vector types go through FP32 for the 16-bit
// types (exact for widening; rounding to nearest even when narrowing).
template <typename To, typename Ti> __device__ __forceinline__ To cvt(Ti v)
{
    if constexpr (std::is_same<To, Ti>::value) return v;
    else if constexpr (std::is_same<Ti, double>::value) return from_t<To>((float)v);
    else if constexpr (std::is_same<To, double>::value) return (double)to_t<float>(v);
    else return from_t<To>(to_t<float>(v));
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_nat2int(Geom g, const Ti *__restrict__ nat, To *__restrict__ in)
{
    const i64 I = gtid();
    if (I >= g.N) return;
    const int i = (int)(I % g.nx), j = (int)((I / g.nx) % g.ny), k = (int)(I / ((i64)g.nx * g.ny));
    in[to_internal(g, i, j, k)] = cvt<To>(nat[I]);
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_int2nat(Geom g, const Ti *__restrict__ in, To *__restrict__ nat)
{
    const i64 I = gtid();
    if (I >= g.N) return;
    const int i = (int)(I % g.nx), j = (int)((I / g.nx) % g.ny), k = (int)(I / ((i64)g.nx * g.ny));
    nat[I] = cvt<To>(in[to_internal(g, i, j, k)]);
}

// Calls f(tag) with a value of the multigrid vector type of p.
template <typename F> static void with_vec(Prec p, F &&f)
{
    switch (p) {
    case P64: f(double{}); break;
    case P16V: f(__half{}); break;
    case PB16V: f(bf16{}); break;
    default: f(float{}); break;
    }
}

void launch_nat2int(const Geom &g, Prec src, const void *nat, Prec dst, void *in, hipStream_t s)
{
    const dim3 gr(grid_for(g.N)), bl(kBlock);
    with_vec(src, [&](auto ti) {
        with_vec(dst, [&](auto to) {
            using Ti = decltype(ti);
            using To = decltype(to);
            hipLaunchKernelGGL((k_nat2int<Ti, To>), gr, bl, 0, s, g, (const Ti *)nat, (To *)in);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_int2nat(const Geom &g, Prec src, const void *in, Prec dst, void *nat, hipStream_t s)
{
    const dim3 gr(grid_for(g.N)), bl(kBlock);
    with_vec(src, [&](auto ti) {
        with_vec(dst, [&](auto to) {
            using Ti = decltype(ti);
            using To = decltype(to);
            hipLaunchKernelGGL((k_int2nat<Ti, To>), gr, bl, 0, s, g, (const Ti *)in, (To *)nat);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

// Matrix value type V and multigrid vector type S of each precision, with the
// value arrays of the matrix: calls f(v, d, S{}).
template <typename F> static void with_matrix(const Matrix &A, Prec p, F &&f)
{
    switch (p) {
    case P64: f(A.v64, A.d64, double{}); break;
    case P32: f(A.v32, A.d32, float{}); break;
    case P16: f(A.v16, A.d16, float{}); break;
    case PB16: f(A.vb16, A.db16, float{}); break;
    case P16V: f(A.v16, A.d16, __half{}); break;
    case PB16V: f(A.vb16, A.db16, bf16{}); break;
    }
}

// ---- SpMV -------------------------------------------------------------------------------
// y = A x over all N rows (Sec. 3.2 ELL SpMV); with `scale`, y = (A x) * *scale
// (the unnormalised-basis scale of the column x was computed from).  x is a
// multigrid vector (type S), y a Krylov vector (type T).
template <typename V, typename S, bool C16>
__global__ __launch_bounds__(kBlock) void k_spmv(Geom g, i64 row0, i64 cnt, int nb, int clog2, int remap,
                                                 const V *__restrict__ offv,
                                                 const void *__restrict__ offc, const int *__restrict__ cmap,
                                                 const V *__restrict__ diag,
                                                 const S *__restrict__ x,
                                                 typename VecT<V>::T *__restrict__ y,
                                                 const double *scale)
{
    using T = typename VecT<V>::T;
    __shared__ int cm[C16 ? kColMapSize : 1];
    if constexpr (C16) stage_colmap(cm, cmap);
    const i64 N = g.N;
    i64 p = gtid_xcd(remap, nb);
    if (p >= cnt) return;
    p = remap == kRemapPlanes ? plane_row(p, g) : row0 + p;
    const EllRow er = ell_row(p, N, clog2);
    const T d = to_t<T>(ld_stream(diag + p)), xp = to_t<T>(x[p]);
    const int *Dc = C16 ? cm + row_colour(g, p) * kSlots : nullptr;
    const T acc = ell_row_dot<T, V, kAllSlots, C16>(offv, offc, x, er, p, Dc, N);
    __builtin_nontemporal_store(spmv_row_value<T>(d, xp, acc, scale), y + p);
}

// Order of the single-vector SpMV.  With the default (kRemapSlab) the FP32
// and 16-bit SpMV take the slab order and the FP64 one the XCD-contiguous
// order.  The plane order brings the fetched bytes of the 320^3 SpMV down to
// the algorithmic ones (FP32: 1.13x -> 1.00x), but it ran 5 % (FP32) and 1 %
// (FP64) slower: the redundant fetches of the other orders are served by
// the last-level cache, not HBM.  Over nb < 8 colour blocks (one colour's
// rows come from the last Gauss-Seidel launch) the plane order gives way to
// the XCD-contiguous one.
static int spmv_order(const Matrix &A, bool fp64, int nb)
{
    if (fp64 && A.order == kRemapSlab) return tile_remap(A);
    const int o = full_grid_order(A, 1);
    return nb < 8 && o == kRemapPlanes ? 1 : o;
}

const double *spmv_scale(Prec p, const Ctrl *ctrl, int k)
{
    return !ctrl ? nullptr : mg16(p) ? &ctrl->mg_post : ctrl->colscale + k;
}

void launch_spmv(const Matrix &A, Prec p, const void *x, void *y, hipStream_t s, const Ctrl *ctrl, int k,
                 int skip)
{
    const double *scale = spmv_scale(p, ctrl, k);
    // rows of every colour but `skip`: a contiguous range when skip is the
    // first or the last colour
    i64 row0 = 0, cnt = A.g.N;
    int nb = 8;
    if (skip == 0) { row0 = A.g.off[1]; cnt = A.g.N - row0; nb = 7; }
    else if (skip == 7) { cnt = A.g.off[7]; nb = 7; }
    else if (skip >= 0) throw std::runtime_error("launch_spmv: only the first or the last colour can be left out");
    if (cnt == 0) return;
    with_matrix(A, p, [&](auto *v, auto *d, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using S = decltype(sv);
        using T = typename VecT<V>::T;
        with_cols(A, [&](auto c16) {
            hipLaunchKernelGGL((k_spmv<V, S, decltype(c16)::value>), dim3(grid_for(cnt)), dim3(kBlock), 0, s, A.g,
                               row0, cnt, nb, A.clog2, spmv_order(A, std::is_same<V, double>::value, nb),
                               (const V *)v, (const void *)A.col, A.cmap, (const V *)d, (const S *)x, (T *)y, scale);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

// ---- SpMV after the last sweep of a V-cycle ---------------------------------------------------
// In sweep order, the colours at positions 2-6 (forward: 2 ... 6; backward:
// 5 ... 1) have their row sums split in two: E, the slots to the colours
// relaxed before them in the sweep, and L, the others, each summed in slot
// order, and (A z)_p = a_pp z_p + (sum_E + sum_L).  FUSED: sum_E comes from
// part (written by the colour's own launch, k_gs with kWoutPart) and only
// the L slots are read here -- 20, 18, 8, 6 and 2 of 26 -- and the rows of
// the sweep's last colour were written by its launch, so they are left out;
// otherwise both sums are formed here from z, and every row is.  The rows
// of the first two colours are whole k_spmv rows (position 1 would save 2
// slots for the 4 bytes of a partial sum written and read again).  The two
// forms give the same bits.
template <typename T, typename V, typename S, int C, bool FWD, bool FUSED, bool C16>
__device__ __forceinline__ T split_row_sum(const V *__restrict__ offv, const void *__restrict__ offc,
                                           const S *x, const EllRow &er, i64 p, const int *Dc, i64 N,
                                           const T *__restrict__ part)
{
    constexpr unsigned E = zero_guess_mask(C, FWD), L = kAllSlots & ~E;
    T se = (T)0;
    if constexpr (FUSED) se = part[p];
    const T sl = ell_row_dot<T, V, L, C16>(offv, offc, x, er, p, Dc, N);
    if constexpr (!FUSED) se = ell_row_dot<T, V, E, C16>(offv, offc, x, er, p, Dc, N);
    return se + sl;
}

// One colour block of the split rows (compile-time slot masks; a launch per
// colour keeps the short rows of the late colours from running at the
// occupancy the whole rows need).
template <typename V, typename S, bool C16, int C, bool FWD, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_spmv_colour(i64 row0, i64 cnt, i64 N, int clog2, int remap,
                                                        const V *__restrict__ offv,
                                                        const void *__restrict__ offc,
                                                        const int *__restrict__ cmapc,
                                                        const V *__restrict__ diag,
                                                        const S *__restrict__ x,
                                                        typename VecT<V>::T *__restrict__ y,
                                                        const typename VecT<V>::T *__restrict__ part,
                                                        const double *scale)
{
    using T = typename VecT<V>::T;
    const i64 t = gtid_xcd(remap);
    if (t >= cnt) return;
    const i64 p = row0 + t;
    const EllRow er = ell_row(p, N, clog2);
    const T d = to_t<T>(ld_stream(diag + p)), xp = to_t<T>(x[p]);
    const T acc = split_row_sum<T, V, S, C, FWD, FUSED, C16>(offv, offc, x, er, p, cmapc, N, part);
    __builtin_nontemporal_store(spmv_row_value<T>(d, xp, acc, scale), y + p);
}

template <typename V, typename S, bool C16, int POS, bool FWD, bool FUSED>
static void spmv_colour_launch(const Matrix &A, const V *v, const V *d, const void *x, void *y, const void *part,
                               const double *scale, hipStream_t s)
{
    using T = typename VecT<V>::T;
    constexpr int C = FWD ? POS : 7 - POS;
    const i64 row0 = A.g.off[C], cnt = A.g.off[C + 1] - row0;
    if (cnt == 0) return;
    hipLaunchKernelGGL((k_spmv_colour<V, S, C16, C, FWD, FUSED>), dim3(grid_for(cnt)), dim3(kBlock), 0, s, row0, cnt,
                       A.g.N, A.clog2, tile_remap(A), v, (const void *)A.col, C16 ? A.cmap + C * kSlots : nullptr, d,
                       (const S *)x, (T *)y, (const T *)part, scale);
}

// Whole rows of the colours in [c0, c1) (consecutive blocks) with k_spmv.
template <typename V, typename S, bool C16>
static void spmv_rows_launch(const Matrix &A, const V *v, const V *d, int c0, int c1, const void *x, void *y,
                             const double *scale, hipStream_t s)
{
    using T = typename VecT<V>::T;
    const i64 row0 = A.g.off[c0], cnt = A.g.off[c1] - row0;
    if (cnt == 0) return;
    const int nb = c1 - c0;
    int order = spmv_order(A, std::is_same<V, double>::value, nb);
    if (order == kRemapPlanes) order = 1;
    hipLaunchKernelGGL((k_spmv<V, S, C16>), dim3(grid_for(cnt)), dim3(kBlock), 0, s, A.g, row0, cnt, nb, A.clog2,
                       order, v, (const void *)A.col, A.cmap, d, (const S *)x, (T *)y, scale);
}

void launch_spmv_split(const Matrix &A, Prec p, const void *x, void *y, const void *part, bool forward,
                       bool fused, hipStream_t s, const Ctrl *ctrl, int k)
{
    const double *scale = spmv_scale(p, ctrl, k);
    with_matrix(A, p, [&](auto *v, auto *d, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using S = decltype(sv);
        with_cols(A, [&](auto c16) {
            constexpr bool C = decltype(c16)::value;
            // sweep positions 0 and 1 (and 7 when it is not fused): whole rows
            if (forward) {
                spmv_rows_launch<V, S, C>(A, v, d, 0, 2, x, y, scale, s);
                if (!fused) spmv_rows_launch<V, S, C>(A, v, d, 7, 8, x, y, scale, s);
            } else {
                spmv_rows_launch<V, S, C>(A, v, d, 6, 8, x, y, scale, s);
                if (!fused) spmv_rows_launch<V, S, C>(A, v, d, 0, 1, x, y, scale, s);
            }
            auto split = [&](auto fwd, auto fus) {
                constexpr bool F = decltype(fwd)::value, U = decltype(fus)::value;
                spmv_colour_launch<V, S, C, 2, F, U>(A, v, d, x, y, part, scale, s);
                spmv_colour_launch<V, S, C, 3, F, U>(A, v, d, x, y, part, scale, s);
                spmv_colour_launch<V, S, C, 4, F, U>(A, v, d, x, y, part, scale, s);
                spmv_colour_launch<V, S, C, 5, F, U>(A, v, d, x, y, part, scale, s);
                spmv_colour_launch<V, S, C, 6, F, U>(A, v, d, x, y, part, scale, s);
            };
            if (forward) {
                if (fused) split(std::true_type{}, std::true_type{});
                else split(std::true_type{}, std::false_type{});
            } else {
                if (fused) split(std::false_type{}, std::true_type{});
                else split(std::false_type{}, std::false_type{});
            }
        });
    });
    HPGMX_LAUNCH_CHECK();
}

// ---- Gauss-Seidel, one colour ---------------------------------------------------------------
// Rows p in [row0, row0 + cnt) of one colour:
//   z_p <- (r_p - sum_{s in MASK} a_{p,s} z_{col(p,s)}) / a_pp
// (relaxation form of eq. (1)).  Rows of one colour never couple, so the
// in-place update is race free.  MASK is a compile-time slot set, so the
// unrolled loop issues every load of the row before the first use: the full
// mask for ordinary sweeps, and for a sweep from a zero guess only the slots
// that couple to colours relaxed earlier in the sweep (the others still hold
// zero, and skipping them gives the same result bit for bit).  r and z are
// stored in S and the row is evaluated in T.
//
// The last sweep of a V-cycle's level-0 post-smoothing also prepares the
// SpMV w = A z that follows it (WOUT):
//  * kWoutRow, the sweep's last colour (every neighbour is final once it is
//    relaxed): the launch writes the SpMV rows of its colour,
//    w_p = (A z)_p, from the slot sum it already holds (spmv_row_value,
//    same bits as the SpMV kernels);
//  * kWoutPart, the colours at sweep positions 2-6: the launch writes part_p, the
//    sum over the slots EMASK of the neighbours relaxed before the colour
//    (final from then on); the SpMV adds the remaining slots (launch_spmv_split).
constexpr int kWoutNone = 0, kWoutRow = 1, kWoutPart = 2;
template <typename V, typename S, unsigned MASK, bool C16, int WOUT = kWoutNone, unsigned EMASK = 0>
__global__ __launch_bounds__(kBlock) void k_gs(i64 row0, i64 cnt, i64 N, int clog2, int remap,
                                               const V *__restrict__ offv,
                                               const void *__restrict__ offc, const int *__restrict__ cmapc,
                                               const V *__restrict__ diag,
                                               const S *__restrict__ r, S *z,
                                               typename VecT<V>::T *__restrict__ w, const double *scale)
{
    using T = typename VecT<V>::T;
    const i64 t = gtid_xcd(remap);
    if (t >= cnt) return;
    const i64 p = row0 + t;
    const EllRow er = ell_row(p, N, clog2);
    const T rp = to_t<T>(r[p]);
    const T dg = to_t<T>(ld_stream(diag + p));
    if constexpr (WOUT == kWoutPart) {
        T accE;
        const T acc = ell_row_dot2<T, V, MASK, EMASK, C16>(offv, offc, z, er, p, cmapc, N, accE);
        st_stream(z + p, from_t<S>((rp - acc) / dg));
        __builtin_nontemporal_store(accE, w + p);
    } else {
        const T acc = ell_row_dot<T, V, MASK, C16>(offv, offc, z, er, p, cmapc, N);
        const S zp = from_t<S>((rp - acc) / dg);
        st_stream(z + p, zp);
        if constexpr (WOUT == kWoutRow)
            __builtin_nontemporal_store(spmv_row_value<T>(dg, to_t<T>(zp), acc, scale), w + p);
    }
}

template <typename V, typename S, unsigned MASK, int WOUT = kWoutNone, unsigned EMASK = 0>
static void gs_launch(const Matrix &A, const V *v, const V *d, int c, const void *r, void *z, hipStream_t s,
                      SpmvOut out = {})
{
    using T = typename VecT<V>::T;
    const i64 row0 = A.g.off[c], cnt = A.g.off[c + 1] - A.g.off[c];
    if (cnt == 0) return;
    void *w = WOUT == kWoutPart ? out.part : out.w;
    with_cols(A, [&](auto c16) {
        hipLaunchKernelGGL((k_gs<V, S, MASK, decltype(c16)::value, WOUT, EMASK>), dim3(grid_for(cnt)), dim3(kBlock),
                           0, s, row0, cnt, A.g.N, A.clog2, tile_remap(A), v, (const void *)A.col,
                           A.c16 ? A.cmap + c * kSlots : nullptr, d, (const S *)r, (S *)z, (T *)w, out.scale);
    });
    HPGMX_LAUNCH_CHECK();
}

// The full-slot launch of colour C that also writes its partial SpMV sums
// over the neighbours relaxed before it (direction FWD).
template <typename V, typename S, int C, bool FWD>
static void gs_part_launch(const Matrix &A, const V *v, const V *d, const void *r, void *z, hipStream_t s,
                           SpmvOut out)
{
    gs_launch<V, S, kAllSlots, kWoutPart, zero_guess_mask(C, FWD)>(A, v, d, C, r, z, s, out);
}

#define HPGMX_GS_CASE(C, FWD) \
    case C: gs_launch<V, S, zero_guess_mask(C, FWD)>(A, v, d, c, r, z, s); break;

template <typename V, typename S>
static void gs_t(const Matrix &A, const V *v, const V *d, int c, int mode, const void *r, void *z,
                 hipStream_t s, SpmvOut out)
{
    if (out.w || out.part) {
        if (mode != kGsFull) throw std::runtime_error("the SpMV rows ride only on a full colour launch");
        if (out.w) {
            gs_launch<V, S, kAllSlots, kWoutRow>(A, v, d, c, r, z, s, out);
        } else {
            switch (c + (out.forward ? 0 : 8)) {
            case 2: gs_part_launch<V, S, 2, true>(A, v, d, r, z, s, out); break;
            case 3: gs_part_launch<V, S, 3, true>(A, v, d, r, z, s, out); break;
            case 4: gs_part_launch<V, S, 4, true>(A, v, d, r, z, s, out); break;
            case 5: gs_part_launch<V, S, 5, true>(A, v, d, r, z, s, out); break;
            case 6: gs_part_launch<V, S, 6, true>(A, v, d, r, z, s, out); break;
            case 8 + 1: gs_part_launch<V, S, 1, false>(A, v, d, r, z, s, out); break;
            case 8 + 2: gs_part_launch<V, S, 2, false>(A, v, d, r, z, s, out); break;
            case 8 + 3: gs_part_launch<V, S, 3, false>(A, v, d, r, z, s, out); break;
            case 8 + 4: gs_part_launch<V, S, 4, false>(A, v, d, r, z, s, out); break;
            case 8 + 5: gs_part_launch<V, S, 5, false>(A, v, d, r, z, s, out); break;
            default: throw std::runtime_error("partial SpMV sums: sweep positions 2-6 only");
            }
        }
    } else if (mode == kGsFull) {
        gs_launch<V, S, kAllSlots>(A, v, d, c, r, z, s);
    } else if (mode == kGsZeroForward) {
        switch (c) {
            HPGMX_GS_CASE(0, true) HPGMX_GS_CASE(1, true) HPGMX_GS_CASE(2, true) HPGMX_GS_CASE(3, true)
            HPGMX_GS_CASE(4, true) HPGMX_GS_CASE(5, true) HPGMX_GS_CASE(6, true) HPGMX_GS_CASE(7, true)
        }
    } else {
        switch (c) {
            HPGMX_GS_CASE(0, false) HPGMX_GS_CASE(1, false) HPGMX_GS_CASE(2, false) HPGMX_GS_CASE(3, false)
            HPGMX_GS_CASE(4, false) HPGMX_GS_CASE(5, false) HPGMX_GS_CASE(6, false) HPGMX_GS_CASE(7, false)
        }
    }
}

void launch_gs_colour(const Matrix &A, Prec p, int c, int mode, const void *r, void *z,
                      hipStream_t s, SpmvOut out)
{
    with_matrix(A, p, [&](auto *v, auto *d, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        gs_t<V, decltype(sv)>(A, v, d, c, mode, r, z, s, out);
    });
}

// ---- Gauss-Seidel from a zero guess, two colours per launch ----------------------------------
// Colours a and b = a ^ 1, consecutive in a forward (a even) or backward
// (a odd) sweep, couple only through the x-neighbours (slots 12 and 13), and
// in a sweep from a zero guess a row reads only colours relaxed before it.
// One launch relaxes both: a lane of colour a does what k_gs does; a lane of
// colour b first evaluates its two colour-a neighbours with colour a's own
// expression (same loads, same operations, hence the same bits), then its
// own row with those two values in place of the gathered ones.  Nothing the
// launch writes is read by it, so the result equals the two single-colour
// launches bit for bit.  The price is two extra row evaluations per colour-b
// row, worth paying where a launch is latency bound (the small levels).
// Row tiles alternate between the colours, so each XCD gets the same slab
// of both blocks; the blocks must have equal sizes (even x extent).
template <typename V, typename S, unsigned MA, unsigned MB, bool C16>
__global__ __launch_bounds__(kBlock) void k_gs_pair_zero(i64 rowa, i64 rowb, i64 cnt, i64 N, int clog2,
                                                         int remap, const V *__restrict__ offv,
                                                         const void *__restrict__ offc,
                                                         const int *__restrict__ cmapa,
                                                         const int *__restrict__ cmapb,
                                                         const V *__restrict__ diag,
                                                         const S *__restrict__ r, S *z)
{
    static_assert((MA & kXSlots) == 0 && (MB & kXSlots) == kXSlots, "colours a, b = a ^ 1 in sweep order");
    using T = typename VecT<V>::T;
    const i64 t = gtid_xcd(remap);
    const i64 tile = t / kBlock;
    const i64 u = (tile >> 1) * kBlock + t % kBlock;
    if (u >= cnt) return;
    if ((tile & 1) == 0) {
        const i64 p = rowa + u;
        const EllRow er = ell_row(p, N, clog2);
        const T rp = to_t<T>(r[p]);
        const T dg = to_t<T>(ld_stream(diag + p));
        st_stream(z + p, from_t<S>((rp - ell_row_dot<T, V, MA, C16>(offv, offc, z, er, p, cmapa, N)) / dg));
        return;
    }
    const i64 p = rowb + u;
    const EllRow er = ell_row(p, N, clog2);
    S xn[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const i64 q = ell_slot_col<C16>(offc, er, 12 + m, p, cmapb, N);
        if (q == N) {  // padded slot: the zero entry, as the gather would read it
            xn[m] = z[N];
            continue;
        }
        const EllRow eq = ell_row(q, N, clog2);
        const T rq = to_t<T>(r[q]);
        const T dq = to_t<T>(ld_stream(diag + q));
        xn[m] = from_t<S>((rq - ell_row_dot<T, V, MA, C16>(offv, offc, z, eq, q, cmapa, N)) / dq);
    }
    const T rp = to_t<T>(r[p]);
    const T dg = to_t<T>(ld_stream(diag + p));
    const T acc = ell_row_dot_x<T, V, MB, C16>(offv, offc, z, er, p, cmapb, N, xn[0], xn[1]);
    st_stream(z + p, from_t<S>((rp - acc) / dg));
}

template <typename V, typename S, int A_, bool FWD>
static void gs_pair_launch(const Matrix &A, const V *v, const V *d, const void *r, void *z, hipStream_t s)
{
    constexpr int B_ = A_ ^ 1;
    const i64 rowa = A.g.off[A_], rowb = A.g.off[B_], cnt = A.g.off[A_ + 1] - rowa;
    if (cnt == 0) return;
    with_cols(A, [&](auto c16) {
        hipLaunchKernelGGL((k_gs_pair_zero<V, S, zero_guess_mask(A_, FWD), zero_guess_mask(B_, FWD),
                                           decltype(c16)::value>),
                           dim3(2 * grid_for(cnt)), dim3(kBlock), 0, s, rowa, rowb, cnt, A.g.N, A.clog2,
                           tile_remap(A), v, (const void *)A.col, A.c16 ? A.cmap + A_ * kSlots : nullptr,
                           A.c16 ? A.cmap + B_ * kSlots : nullptr, d, (const S *)r, (S *)z);
    });
    HPGMX_LAUNCH_CHECK();
}

bool gs_pair_possible(const Matrix &A) { return A.g.nx % 2 == 0; }

void launch_gs_pair_zero(const Matrix &A, Prec p, int a, bool forward, const void *r, void *z, hipStream_t s)
{
    if (!gs_pair_possible(A) || (forward ? (a & 1) : !(a & 1)))
        throw std::runtime_error("launch_gs_pair_zero: needs an even x extent and a first colour in sweep order");
    with_matrix(A, p, [&](auto *v, auto *d, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using S = decltype(sv);
        switch (a) {
        case 0: gs_pair_launch<V, S, 0, true>(A, v, d, r, z, s); break;
        case 2: gs_pair_launch<V, S, 2, true>(A, v, d, r, z, s); break;
        case 4: gs_pair_launch<V, S, 4, true>(A, v, d, r, z, s); break;
        case 6: gs_pair_launch<V, S, 6, true>(A, v, d, r, z, s); break;
        case 1: gs_pair_launch<V, S, 1, false>(A, v, d, r, z, s); break;
        case 3: gs_pair_launch<V, S, 3, false>(A, v, d, r, z, s); break;
        case 5: gs_pair_launch<V, S, 5, false>(A, v, d, r, z, s); break;
        case 7: gs_pair_launch<V, S, 7, false>(A, v, d, r, z, s); break;
        default: break;
        }
    });
}

// ---- fused residual-restriction (eq. (6)) ------------------------------------------------------
// The colour-4 block of the fine level holds the injection points in the
// coarse level's natural order: row q of that block is coarse point
// (q % cx, (q / cx) % cy, q / (cx cy)).  Only those rows are evaluated.
template <typename V, typename S, bool C16>
__global__ __launch_bounds__(kBlock) void k_restrict(Geom gf, Geom gc, int clog2, int remap,
                                                     const V *__restrict__ offv,
                                                     const void *__restrict__ offc, const int *__restrict__ cmap4,
                                                     const V *__restrict__ diag,
                                                     const S *__restrict__ r,
                                                     const S *__restrict__ z,
                                                     S *__restrict__ rc)
{
    using T = typename VecT<V>::T;
    const i64 q = gtid_xcd(remap);
    if (q >= gc.N) return;
    const i64 N = gf.N, p = gf.off[4] + q;
    const EllRow er = ell_row(p, N, clog2);
    const T rp = to_t<T>(r[p]);
    const T acc = to_t<T>(ld_stream(diag + p)) * to_t<T>(z[p]) +
                  ell_row_dot<T, V, kAllSlots, C16>(offv, offc, z, er, p, cmap4, N);
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), K = (int)(q / ((i64)gc.nx * gc.ny));
    st_stream(rc + to_internal(gc, I, J, K), from_t<S>(rp - acc));
}

void launch_restrict(const Matrix &Af, const Geom &gc, Prec p, const void *r, const void *z,
                     void *rc, hipStream_t s)
{
    with_matrix(Af, p, [&](auto *v, auto *d, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using S = decltype(sv);
        with_cols(Af, [&](auto c16) {
            hipLaunchKernelGGL((k_restrict<V, S, decltype(c16)::value>), dim3(grid_for(gc.N)), dim3(kBlock), 0, s,
                               Af.g, gc, Af.clog2, tile_remap(Af), (const V *)v, (const void *)Af.col,
                               Af.c16 ? Af.cmap + 4 * kSlots : nullptr, (const V *)d, (const S *)r, (const S *)z,
                               (S *)rc);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

// ---- the fused restriction right after a single sweep from zero -----------------------------------
// When z is the outcome of one Gauss-Seidel sweep from z = 0 (the
// pre-smoother of a V-cycle level with one sweep), the relaxation of colour
// 4 made r - A z vanish at the colour-4 rows while the colours relaxed after
// colour 4 were still zero.  Those colours are the only ones that changed
// since, so at an injection point
//     r - A z = - sum over the slots to colours relaxed after 4 of a z,
// which is eq. (6) evaluated with 8 of the 26 slots (forward sweep; 18
// backward) and without r or the diagonal.  Exact in exact arithmetic; the
// rounding differs from the full formula by the rounding of the colour-4
// relaxation.
template <typename V, typename S, unsigned MASK, bool C16>
__global__ __launch_bounds__(kBlock) void k_restrict_after_sweep(Geom gf, Geom gc, int clog2, int remap,
                                                                 const V *__restrict__ offv,
                                                                 const void *__restrict__ offc,
                                                                 const int *__restrict__ cmap4,
                                                                 const S *__restrict__ z,
                                                                 S *__restrict__ rc)
{
    using T = typename VecT<V>::T;
    const i64 q = gtid_xcd(remap);
    if (q >= gc.N) return;
    const i64 N = gf.N, p = gf.off[4] + q;
    const EllRow er = ell_row(p, N, clog2);
    const T acc = ell_row_dot<T, V, MASK, C16>(offv, offc, z, er, p, cmap4, N);
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), K = (int)(q / ((i64)gc.nx * gc.ny));
    st_stream(rc + to_internal(gc, I, J, K), from_t<S>(-acc));
}

void launch_restrict_after_sweep(const Matrix &Af, const Geom &gc, Prec p, bool forward, const void *z, void *rc,
                                 hipStream_t s)
{
    constexpr unsigned kFwd = kAllSlots & ~zero_guess_mask(4, true);
    constexpr unsigned kBwd = kAllSlots & ~zero_guess_mask(4, false);
    with_matrix(Af, p, [&](auto *v, auto *, auto sv) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using S = decltype(sv);
        with_cols(Af, [&](auto c16) {
            constexpr bool C = decltype(c16)::value;
            const int *cm4 = Af.c16 ? Af.cmap + 4 * kSlots : nullptr;
            if (forward)
                hipLaunchKernelGGL((k_restrict_after_sweep<V, S, kFwd, C>), dim3(grid_for(gc.N)), dim3(kBlock), 0, s,
                                   Af.g, gc, Af.clog2, tile_remap(Af), (const V *)v, (const void *)Af.col, cm4,
                                   (const S *)z, (S *)rc);
            else
                hipLaunchKernelGGL((k_restrict_after_sweep<V, S, kBwd, C>), dim3(grid_for(gc.N)), dim3(kBlock), 0, s,
                                   Af.g, gc, Af.clog2, tile_remap(Af), (const V *)v, (const void *)Af.col, cm4,
                                   (const S *)z, (S *)rc);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

// ---- prolongation-correction: z += P zc, P = R^T -------------------------------------------------
template <typename S>
__global__ __launch_bounds__(kBlock) void k_prolong(Geom gf, Geom gc, const S *__restrict__ zc, S *__restrict__ z)
{
    using T = typename VecT<S>::T;
    const i64 q = gtid();
    if (q >= gc.N) return;
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), K = (int)(q / ((i64)gc.nx * gc.ny));
    const i64 p = gf.off[4] + q;
    st_stream(z + p, from_t<S>(to_t<T>(z[p]) + to_t<T>(zc[to_internal(gc, I, J, K)])));
}

void launch_prolong(const Geom &gf, const Geom &gc, Prec p, const void *zc, void *z, hipStream_t s)
{
    with_vec(p, [&](auto sv) {
        using S = decltype(sv);
        hipLaunchKernelGGL(k_prolong<S>, dim3(grid_for(gc.N)), dim3(kBlock), 0, s, gf, gc, (const S *)zc, (S *)z);
    });
    HPGMX_LAUNCH_CHECK();
}

}  // namespace hpgmx
