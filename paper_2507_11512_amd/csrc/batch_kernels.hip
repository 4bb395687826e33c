// Stencil kernels for K right-hand sides at once: the batched SpMV, one
// colour of a batched Gauss-Seidel sweep, the batched fused
// residual-restriction and prolongation, and the batched FP64 outer residual.
//
// Every one of these is bound by HBM bandwidth, and in the single-vector
// kernels the matrix (values and int32 columns, 216 of the 224 bytes a row
// moves in FP32) dominates the traffic.  Here a row's 26 values, 26 columns
// and diagonal are read once for all K right-hand sides, and each neighbour
// contributes one contiguous run of K vector entries (the batch is stored
// interleaved, [p * K + j]).  A lane handles R of the K right-hand sides of
// one row; K / R lanes share the row's matrix entries (the hardware merges
// their identical addresses into one request).  R is a tile shape: wide
// lanes issue fewer, wider gathers and re-read fewer matrix entries, narrow
// lanes give more parallelism to the small coarse levels.  The autotuner in
// the host code picks R per kernel and level by timing.
//
// Per (row, right-hand side) the arithmetic is that of the single-vector
// kernels: the slots are summed in slot order from zero and the diagonal
// term is added last, so the result for right-hand side j does not depend on
// K or R.
#include "ell_device.hpp"

#include <stdexcept>
#include <type_traits>

namespace hpgmx {

// ---- SpMV --------------------------------------------------------------------------------
// With ctrl, vector j of the output is scaled by ctrl[j].colscale[k] (the
// unnormalised-basis scale of the column x was computed from).
template <typename V, int K, int R>
__global__ __launch_bounds__(kBlock) void k_bspmv(Geom gm, i64 row0, i64 cnt, int clog2, int remap,
                                                  const V *__restrict__ offv,
                                                  const int *__restrict__ offc,
                                                  const V *__restrict__ diag,
                                                  const typename VecT<V>::T *__restrict__ x,
                                                  typename VecT<V>::T *__restrict__ y,
                                                  const Ctrl *ctrl, int k)
{
    using T = typename VecT<V>::T;
    constexpr int L = K / R;
    const i64 N = gm.N;
    const i64 t = gtid_xcd(remap);
    i64 p = t / L;
    if (p >= cnt) return;
    // the plane order over all rows, the pair order over the rows of a colour pair
    p = remap == kRemapPlanes ? plane_row(p, gm) : remap == kRemapPlanePair ? plane_pair_row(p, gm, row0) : row0 + p;
    const int g = (int)(t % L);
    const i64 o = p * K + g * R;
    const EllRow er = ell_row(p, N, clog2);
    const Pack<T, R> xp = ldp<T, R>(x + o);
    const T d = to_t<T>(ld_stream(diag + p));
    T acc[R];
    ell_row_dot_b<T, V, K, R, kAllSlots>(offv, offc, x + g * R, er, acc);
    Pack<T, R> out;
#pragma unroll
    for (int r = 0; r < R; ++r)
        out.v[r] = spmv_row_value<T>(d, xp.v[r], acc[r], ctrl ? ctrl[g * R + r].colscale + k : nullptr);
    stp_stream<T, R>(y + o, out);
}

// ---- SpMV after the last sweep of a V-cycle (see launch_spmv_split) ------------------------------
template <typename T, typename V, int K, int R, int C, bool FWD, bool FUSED>
__device__ __forceinline__ void bsplit_row_sum(const V *__restrict__ offv, const int *__restrict__ offc,
                                               const T *x, const EllRow &er, const T *part, T (&acc)[R])
{
    constexpr unsigned E = zero_guess_mask(C, FWD), L = kAllSlots & ~E;
    Pack<T, R> se;
    if constexpr (FUSED) se = ldp<T, R>(part);
    T sl[R];
    ell_row_dot_b<T, V, K, R, L>(offv, offc, x, er, sl);
    if constexpr (!FUSED) ell_row_dot_b<T, V, K, R, E>(offv, offc, x, er, se.v);
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = se.v[r] + sl[r];
}

// One colour block of the split rows (a launch per colour, as the
// single-vector SpMV; compile-time slot masks).
template <typename V, int K, int R, int C, bool FWD, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_bspmv_colour(i64 row0, i64 cnt, i64 N, int clog2, int remap,
                                                         const V *__restrict__ offv,
                                                         const int *__restrict__ offc,
                                                         const V *__restrict__ diag,
                                                         const typename VecT<V>::T *__restrict__ x,
                                                         typename VecT<V>::T *__restrict__ y,
                                                         const typename VecT<V>::T *__restrict__ part,
                                                         const Ctrl *ctrl, int k)
{
    using T = typename VecT<V>::T;
    constexpr int L = K / R;
    const i64 t = gtid_xcd(remap);
    const i64 q = t / L;
    if (q >= cnt) return;
    const int g = (int)(t % L);
    const i64 p = row0 + q;
    const i64 o = p * K + g * R;
    const EllRow er = ell_row(p, N, clog2);
    const Pack<T, R> xp = ldp<T, R>(x + o);
    const T d = to_t<T>(ld_stream(diag + p));
    T acc[R];
    bsplit_row_sum<T, V, K, R, C, FWD, FUSED>(offv, offc, x + g * R, er, part + o, acc);
    Pack<T, R> out;
#pragma unroll
    for (int r = 0; r < R; ++r)
        out.v[r] = spmv_row_value<T>(d, xp.v[r], acc[r], ctrl ? ctrl[g * R + r].colscale + k : nullptr);
    stp_stream<T, R>(y + o, out);
}

// ---- Gauss-Seidel, one colour (rows [row0, row0 + cnt)) ------------------------------------
// WOUT as in k_gs (stencil_kernels.hip): the last sweep of a V-cycle's
// level-0 post-smoothing also writes the SpMV rows of its last colour
// (kWoutRow, right-hand side j scaled by ctrl[j].colscale[k]) and the
// partial sums of the colours at sweep positions 2-6 (kWoutPart).
constexpr int kBWoutNone = 0, kBWoutRow = 1, kBWoutPart = 2;
template <typename V, int K, int R, unsigned MASK, int WOUT = kBWoutNone, unsigned EMASK = 0>
__global__ __launch_bounds__(kBlock) void k_bgs(i64 row0, i64 cnt, i64 N, int clog2, int remap,
                                                const V *__restrict__ offv,
                                                const int *__restrict__ offc,
                                                const V *__restrict__ diag,
                                                const typename VecT<V>::T *__restrict__ r,
                                                typename VecT<V>::T *z,
                                                typename VecT<V>::T *__restrict__ y, const Ctrl *ctrl, int k)
{
    using T = typename VecT<V>::T;
    constexpr int L = K / R;
    const i64 t = gtid_xcd(remap);
    const i64 q = t / L;
    if (q >= cnt) return;
    const int g = (int)(t % L);
    const i64 p = row0 + q;
    const i64 o = p * K + g * R;
    const EllRow er = ell_row(p, N, clog2);
    const Pack<T, R> rp = ldp<T, R>(r + o);
    const T dg = to_t<T>(ld_stream(diag + p));
    T acc[R];
    Pack<T, R> out;
    if constexpr (WOUT == kBWoutPart) {
        Pack<T, R> pe;
        ell_row_dot_b2<T, V, K, R, MASK, EMASK>(offv, offc, z + g * R, er, acc, pe.v);
#pragma unroll
        for (int i = 0; i < R; ++i) out.v[i] = (rp.v[i] - acc[i]) / dg;
        stp<T, R>(z + o, out);  // plain: re-read by the next colour passes (see st_stream)
        stp_stream<T, R>(y + o, pe);
    } else {
        ell_row_dot_b<T, V, K, R, MASK>(offv, offc, z + g * R, er, acc);
#pragma unroll
        for (int i = 0; i < R; ++i) out.v[i] = (rp.v[i] - acc[i]) / dg;
        stp<T, R>(z + o, out);
        if constexpr (WOUT == kBWoutRow) {
            Pack<T, R> w;
#pragma unroll
            for (int i = 0; i < R; ++i)
                w.v[i] = spmv_row_value<T>(dg, out.v[i], acc[i], ctrl ? ctrl[g * R + i].colscale + k : nullptr);
            stp_stream<T, R>(y + o, w);
        }
    }
}

// ---- fused residual-restriction (eq. (6)) at the colour-4 rows ------------------------------
template <typename V, int K, int R>
__global__ __launch_bounds__(kBlock) void k_brestrict(Geom gf, Geom gc, int clog2, int remap,
                                                      const V *__restrict__ offv,
                                                      const int *__restrict__ offc,
                                                      const V *__restrict__ diag,
                                                      const typename VecT<V>::T *__restrict__ r,
                                                      const typename VecT<V>::T *__restrict__ z,
                                                      typename VecT<V>::T *__restrict__ rc)
{
    using T = typename VecT<V>::T;
    constexpr int L = K / R;
    const i64 t = gtid_xcd(remap);
    const i64 q = t / L;
    if (q >= gc.N) return;
    const int g = (int)(t % L);
    const i64 N = gf.N, p = gf.off[4] + q;
    const i64 o = p * K + g * R;
    const EllRow er = ell_row(p, N, clog2);
    const Pack<T, R> rp = ldp<T, R>(r + o);
    const Pack<T, R> zp = ldp<T, R>(z + o);
    const T d = to_t<T>(ld_stream(diag + p));
    T acc[R];
    ell_row_dot_b<T, V, K, R, kAllSlots>(offv, offc, z + g * R, er, acc);
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), Kc = (int)(q / ((i64)gc.nx * gc.ny));
    Pack<T, R> out;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const T dz = d * zp.v[i];
        out.v[i] = rp.v[i] - (dz + acc[i]);
    }
    stp_stream<T, R>(rc + to_internal(gc, I, J, Kc) * K + g * R, out);
}

// ---- the fused restriction right after a single sweep from zero (see
// k_restrict_after_sweep in stencil_kernels.hip): minus the couplings of the
// injection rows to the colours relaxed after colour 4 ----
template <typename V, int K, int R, unsigned MASK>
__global__ __launch_bounds__(kBlock) void k_brestrict_after_sweep(Geom gf, Geom gc, int clog2, int remap,
                                                                  const V *__restrict__ offv,
                                                                  const int *__restrict__ offc,
                                                                  const typename VecT<V>::T *__restrict__ z,
                                                                  typename VecT<V>::T *__restrict__ rc)
{
    using T = typename VecT<V>::T;
    constexpr int L = K / R;
    const i64 t = gtid_xcd(remap);
    const i64 q = t / L;
    if (q >= gc.N) return;
    const int g = (int)(t % L);
    const i64 N = gf.N, p = gf.off[4] + q;
    const EllRow er = ell_row(p, N, clog2);
    T acc[R];
    ell_row_dot_b<T, V, K, R, MASK>(offv, offc, z + g * R, er, acc);
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), Kc = (int)(q / ((i64)gc.nx * gc.ny));
    Pack<T, R> out;
#pragma unroll
    for (int i = 0; i < R; ++i) out.v[i] = -acc[i];
    stp_stream<T, R>(rc + to_internal(gc, I, J, Kc) * K + g * R, out);
}

// ---- prolongation-correction z += P zc (one lane per element) -------------------------------
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_bprolong(Geom gf, Geom gc, const T *__restrict__ zc,
                                                     T *__restrict__ z)
{
    const i64 e = gtid();
    const i64 q = e / K;
    if (q >= gc.N) return;
    const int j = (int)(e % K);
    const int I = (int)(q % gc.nx), J = (int)((q / gc.nx) % gc.ny), Kc = (int)(q / ((i64)gc.nx * gc.ny));
    const i64 o = (gf.off[4] + q) * K + j;
    __builtin_nontemporal_store(z[o] + zc[to_internal(gc, I, J, Kc) * K + j], z + o);
}

// ---- FP64 outer residual r = b - A x ---------------------------------------------------------
// The norms ||r_j|| are summed by the fixed-layout norm kernel afterwards, so
// that they (and everything that follows from them) do not depend on R.
template <int K, int R>
__global__ __launch_bounds__(kBlock) void k_bresid64(i64 N, int clog2, int remap,
                                                     const double *__restrict__ offv,
                                                     const int *__restrict__ offc,
                                                     const double *__restrict__ diag,
                                                     const double *__restrict__ x,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ r)
{
    constexpr int L = K / R;
    const i64 t = gtid_xcd(remap);
    const i64 p = t / L;
    if (p >= N) return;
    const int g = (int)(t % L);
    const i64 o = p * K + g * R;
    const EllRow er = ell_row(p, N, clog2);
    const Pack<double, R> bp = ldp<double, R>(b + o);
    const Pack<double, R> xp = ldp<double, R>(x + o);
    const double d = ld_stream(diag + p);
    double acc[R];
    ell_row_dot_b<double, double, K, R, kAllSlots>(offv, offc, x + g * R, er, acc);
    Pack<double, R> out;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        out.v[i] = bp.v[i] - spmv_row_value<double>(d, xp.v[i], acc[i], nullptr);
    }
    stp_stream<double, R>(r + o, out);
}

// ---- [nrhs][N] natural order <-> [N][K] colour-blocked --------------------------------------
template <typename Ti, typename To, int K>
__global__ __launch_bounds__(kBlock) void k_bnat2int(Geom g, int nrhs, const Ti *__restrict__ nat,
                                                     To *__restrict__ in)
{
    const i64 I = gtid();
    if (I >= g.N) return;
    const int i = (int)(I % g.nx), j = (int)((I / g.nx) % g.ny), k = (int)(I / ((i64)g.nx * g.ny));
    const i64 q = to_internal(g, i, j, k) * K;
#pragma unroll
    for (int c = 0; c < K; ++c) in[q + c] = c < nrhs ? (To)nat[(i64)c * g.N + I] : (To)0;
}

template <typename Ti, typename To, int K>
__global__ __launch_bounds__(kBlock) void k_bint2nat(Geom g, int nrhs, const Ti *__restrict__ in,
                                                     To *__restrict__ nat)
{
    const i64 I = gtid();
    if (I >= g.N) return;
    const int i = (int)(I % g.nx), j = (int)((I / g.nx) % g.ny), k = (int)(I / ((i64)g.nx * g.ny));
    const i64 q = to_internal(g, i, j, k) * K;
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (c < nrhs) nat[(i64)c * g.N + I] = (To)in[q + c];
}

// =====================================================================================================
// launchers
bool batch_shape_ok(int K, int R)
{
    return (K == 2 || K == 4 || K == 8) && R >= 1 && R <= K && (K % R) == 0 && (R & (R - 1)) == 0;
}

// Calls f(K, R) with both as compile-time constants.
template <typename F> static void with_kr(int K, int R, F &&f)
{
    using std::integral_constant;
#define HPGMX_KR(KK, RR) \
    if (K == KK && R == RR) return f(integral_constant<int, KK>{}, integral_constant<int, RR>{});
    HPGMX_KR(2, 1) HPGMX_KR(2, 2)
    HPGMX_KR(4, 1) HPGMX_KR(4, 2) HPGMX_KR(4, 4)
    HPGMX_KR(8, 1) HPGMX_KR(8, 2) HPGMX_KR(8, 4) HPGMX_KR(8, 8)
#undef HPGMX_KR
    throw std::runtime_error("unsupported batch tile (K, R)");
}

template <typename F> static void with_k(int K, F &&f)
{
    using std::integral_constant;
    if (K == 2) return f(integral_constant<int, 2>{});
    if (K == 4) return f(integral_constant<int, 4>{});
    if (K == 8) return f(integral_constant<int, 8>{});
    throw std::runtime_error("unsupported batch width");
}

// Matrix values of a batched call (the vectors are FP64 for P64, FP32
// otherwise).
template <typename F> static void with_values(const Matrix &A, Prec p, F &&f)
{
    switch (p) {
    case P64: return f(A.v64, A.d64);
    case P32: return f(A.v32, A.d32);
    case P16: return f(A.v16, A.d16);
    case PB16: return f(A.vb16, A.db16);
    default: break;  // 16-bit multigrid vectors are not batched
    }
    throw std::runtime_error("unsupported matrix precision for a batched call");
}

static inline unsigned lanes_grid(i64 rows, int K, int R) { return grid_for(rows * (K / R)); }

void launch_bspmv(const Matrix &A, Prec p, int K, int R, const void *x, void *y, hipStream_t s,
                  const Ctrl *ctrl, int k)
{
    with_values(A, p, [&](auto *v, auto *d) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using T = typename VecT<V>::T;
        with_kr(K, R, [&](auto kc, auto rc) {
            constexpr int KK = decltype(kc)::value, RR = decltype(rc)::value;
            // The default order takes the plane order here: at 192^3 x 8 it
            // cut the fetched bytes from 1.94x to 1.30x the algorithmic ones
            // and the time by 6 % (the slab order ran slower).
            const int order = A.order >= kRemapSlab ? plane_order(A) : tile_remap(A);
            hipLaunchKernelGGL((k_bspmv<V, KK, RR>), dim3(lanes_grid(A.g.N, KK, RR)), dim3(kBlock), 0, s,
                               A.g, (i64)0, A.g.N, A.clog2, order, v, (const int *)A.col, d, (const T *)x, (T *)y,
                               ctrl, k);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

template <typename V, int K, int R, int POS, bool FWD, bool FUSED>
static void bspmv_colour_launch(const Matrix &A, const V *v, const V *d, const void *x, void *y, const void *part,
                                hipStream_t s, const Ctrl *ctrl, int k)
{
    using T = typename VecT<V>::T;
    constexpr int C = FWD ? POS : 7 - POS;
    const i64 row0 = A.g.off[C], cnt = A.g.off[C + 1] - row0;
    if (cnt == 0) return;
    hipLaunchKernelGGL((k_bspmv_colour<V, K, R, C, FWD, FUSED>), dim3(lanes_grid(cnt, K, R)), dim3(kBlock), 0, s,
                       row0, cnt, A.g.N, A.clog2, tile_remap(A), v, (const int *)A.col, d, (const T *)x, (T *)y,
                       (const T *)part, ctrl, k);
}

void launch_bspmv_split(const Matrix &A, Prec p, int K, int R, const void *x, void *y, const void *part,
                        bool forward, bool fused, hipStream_t s, const Ctrl *ctrl, int k)
{
    if (p != P32 && p != P64) throw std::runtime_error("launch_bspmv_split: FP32 and FP64 only");
    with_values(A, p, [&](auto *v, auto *d) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using T = typename VecT<V>::T;
        if constexpr (std::is_same<V, float>::value || std::is_same<V, double>::value) {
            with_kr(K, R, [&](auto kc, auto rc) {
                constexpr int KK = decltype(kc)::value, RR = decltype(rc)::value;
                // sweep positions 0 and 1 (and 7 when it is not fused): whole rows;
                // the colour pair in the plane-interleaved order where it applies
                const int pair_order = A.order >= kRemapSlab && plane_order(A) == kRemapPlanes
                                           ? kRemapPlanePair : tile_remap(A);
                auto rows = [&](int c0, int c1) {
                    const i64 row0 = A.g.off[c0], cnt = A.g.off[c1] - row0;
                    if (cnt == 0) return;
                    const int order = c1 - c0 == 2 ? pair_order : tile_remap(A);
                    hipLaunchKernelGGL((k_bspmv<V, KK, RR>), dim3(lanes_grid(cnt, KK, RR)), dim3(kBlock), 0, s,
                                       A.g, row0, cnt, A.clog2, order, v, (const int *)A.col, d,
                                       (const T *)x, (T *)y, ctrl, k);
                };
                if (forward) { rows(0, 2); if (!fused) rows(7, 8); }
                else { rows(6, 8); if (!fused) rows(0, 1); }
                auto split = [&](auto fwd, auto fus) {
                    constexpr bool F = decltype(fwd)::value, U = decltype(fus)::value;
                    bspmv_colour_launch<V, KK, RR, 2, F, U>(A, v, d, x, y, part, s, ctrl, k);
                    bspmv_colour_launch<V, KK, RR, 3, F, U>(A, v, d, x, y, part, s, ctrl, k);
                    bspmv_colour_launch<V, KK, RR, 4, F, U>(A, v, d, x, y, part, s, ctrl, k);
                    bspmv_colour_launch<V, KK, RR, 5, F, U>(A, v, d, x, y, part, s, ctrl, k);
                    bspmv_colour_launch<V, KK, RR, 6, F, U>(A, v, d, x, y, part, s, ctrl, k);
                };
                if (forward) {
                    if (fused) split(std::true_type{}, std::true_type{});
                    else split(std::true_type{}, std::false_type{});
                } else {
                    if (fused) split(std::false_type{}, std::true_type{});
                    else split(std::false_type{}, std::false_type{});
                }
            });
        }
    });
    HPGMX_LAUNCH_CHECK();
}

template <typename V, int K, int R, unsigned MASK, int WOUT = kBWoutNone, unsigned EMASK = 0>
static void bgs_launch(const Matrix &A, const V *v, const V *d, int c, const void *r, void *z, hipStream_t s,
                       BSpmvOut out = {})
{
    using T = typename VecT<V>::T;
    const i64 row0 = A.g.off[c], cnt = A.g.off[c + 1] - A.g.off[c];
    if (cnt == 0) return;
    void *y = WOUT == kBWoutPart ? out.part : out.y;
    hipLaunchKernelGGL((k_bgs<V, K, R, MASK, WOUT, EMASK>), dim3(lanes_grid(cnt, K, R)), dim3(kBlock), 0, s, row0,
                       cnt, A.g.N, A.clog2, tile_remap(A), v, (const int *)A.col, d, (const T *)r, (T *)z, (T *)y,
                       out.ctrl, out.k);
}

template <typename V, int K, int R, int C, bool FWD>
static void bgs_part_launch(const Matrix &A, const V *v, const V *d, const void *r, void *z, hipStream_t s,
                            BSpmvOut out)
{
    bgs_launch<V, K, R, kAllSlots, kBWoutPart, zero_guess_mask(C, FWD)>(A, v, d, C, r, z, s, out);
}

#define HPGMX_BGS_CASE(C, FWD) \
    case C: bgs_launch<V, K, R, zero_guess_mask(C, FWD)>(A, v, d, c, r, z, s); break;

template <typename V, int K, int R>
static void bgs_kr(const Matrix &A, const V *v, const V *d, int c, int mode, const void *r, void *z,
                   hipStream_t s, BSpmvOut out)
{
    constexpr bool kWide = std::is_same<V, float>::value || std::is_same<V, double>::value;
    if (kWide && (out.y || out.part)) {
        if (mode != kGsFull) throw std::runtime_error("the SpMV rows ride only on a full colour launch");
        if constexpr (!kWide) return;
        else if (out.y) {
            bgs_launch<V, K, R, kAllSlots, kBWoutRow>(A, v, d, c, r, z, s, out);
        } else {
            switch (c + (out.forward ? 0 : 8)) {
            case 2: bgs_part_launch<V, K, R, 2, true>(A, v, d, r, z, s, out); break;
            case 3: bgs_part_launch<V, K, R, 3, true>(A, v, d, r, z, s, out); break;
            case 4: bgs_part_launch<V, K, R, 4, true>(A, v, d, r, z, s, out); break;
            case 5: bgs_part_launch<V, K, R, 5, true>(A, v, d, r, z, s, out); break;
            case 6: bgs_part_launch<V, K, R, 6, true>(A, v, d, r, z, s, out); break;
            case 8 + 1: bgs_part_launch<V, K, R, 1, false>(A, v, d, r, z, s, out); break;
            case 8 + 2: bgs_part_launch<V, K, R, 2, false>(A, v, d, r, z, s, out); break;
            case 8 + 3: bgs_part_launch<V, K, R, 3, false>(A, v, d, r, z, s, out); break;
            case 8 + 4: bgs_part_launch<V, K, R, 4, false>(A, v, d, r, z, s, out); break;
            case 8 + 5: bgs_part_launch<V, K, R, 5, false>(A, v, d, r, z, s, out); break;
            default: throw std::runtime_error("partial SpMV sums: sweep positions 2-6 only");
            }
        }
    } else if (mode == kGsFull) {
        bgs_launch<V, K, R, kAllSlots>(A, v, d, c, r, z, s);
    } else if (mode == kGsZeroForward) {
        switch (c) {
            HPGMX_BGS_CASE(0, true) HPGMX_BGS_CASE(1, true) HPGMX_BGS_CASE(2, true) HPGMX_BGS_CASE(3, true)
            HPGMX_BGS_CASE(4, true) HPGMX_BGS_CASE(5, true) HPGMX_BGS_CASE(6, true) HPGMX_BGS_CASE(7, true)
        }
    } else {
        switch (c) {
            HPGMX_BGS_CASE(0, false) HPGMX_BGS_CASE(1, false) HPGMX_BGS_CASE(2, false) HPGMX_BGS_CASE(3, false)
            HPGMX_BGS_CASE(4, false) HPGMX_BGS_CASE(5, false) HPGMX_BGS_CASE(6, false) HPGMX_BGS_CASE(7, false)
        }
    }
}
#undef HPGMX_BGS_CASE

void launch_bgs_colour(const Matrix &A, Prec p, int K, int R, int c, int mode, const void *r, void *z,
                       hipStream_t s, BSpmvOut out)
{
    if ((out.y || out.part) && p != P32 && p != P64)
        throw std::runtime_error("the batched SpMV rows ride on FP32 and FP64 sweeps only");
    with_values(A, p, [&](auto *v, auto *d) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        with_kr(K, R, [&](auto kc, auto rc) {
            constexpr int KK = decltype(kc)::value, RR = decltype(rc)::value;
            if constexpr (std::is_same<V, float>::value || std::is_same<V, double>::value)
                bgs_kr<V, KK, RR>(A, v, d, c, mode, r, z, s, out);
            else
                bgs_kr<V, KK, RR>(A, v, d, c, mode, r, z, s, BSpmvOut{});
        });
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_brestrict(const Matrix &Af, const Geom &gc, Prec p, int K, int R, const void *r,
                      const void *z, void *rc, hipStream_t s)
{
    with_values(Af, p, [&](auto *v, auto *d) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using T = typename VecT<V>::T;
        with_kr(K, R, [&](auto kc, auto rcn) {
            constexpr int KK = decltype(kc)::value, RR = decltype(rcn)::value;
            hipLaunchKernelGGL((k_brestrict<V, KK, RR>), dim3(lanes_grid(gc.N, KK, RR)), dim3(kBlock), 0, s,
                               Af.g, gc, Af.clog2, tile_remap(Af), v, (const int *)Af.col, d, (const T *)r,
                               (const T *)z, (T *)rc);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_brestrict_after_sweep(const Matrix &Af, const Geom &gc, Prec p, int K, int R, bool forward,
                                  const void *z, void *rc, hipStream_t s)
{
    constexpr unsigned kFwd = kAllSlots & ~zero_guess_mask(4, true);
    constexpr unsigned kBwd = kAllSlots & ~zero_guess_mask(4, false);
    with_values(Af, p, [&](auto *v, auto *d) {
        (void)d;
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        using T = typename VecT<V>::T;
        with_kr(K, R, [&](auto kc, auto rcn) {
            constexpr int KK = decltype(kc)::value, RR = decltype(rcn)::value;
            const dim3 gr(lanes_grid(gc.N, KK, RR)), bl(kBlock);
            if (forward)
                hipLaunchKernelGGL((k_brestrict_after_sweep<V, KK, RR, kFwd>), gr, bl, 0, s, Af.g, gc, Af.clog2,
                                   tile_remap(Af), v, (const int *)Af.col, (const T *)z, (T *)rc);
            else
                hipLaunchKernelGGL((k_brestrict_after_sweep<V, KK, RR, kBwd>), gr, bl, 0, s, Af.g, gc, Af.clog2,
                                   tile_remap(Af), v, (const int *)Af.col, (const T *)z, (T *)rc);
        });
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_bprolong(const Geom &gf, const Geom &gc, Prec p, int K, const void *zc, void *z, hipStream_t s)
{
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        const dim3 gr(grid_for(gc.N * KK));
        if (p == P64)
            hipLaunchKernelGGL((k_bprolong<double, KK>), gr, dim3(kBlock), 0, s, gf, gc, (const double *)zc,
                               (double *)z);
        else
            hipLaunchKernelGGL((k_bprolong<float, KK>), gr, dim3(kBlock), 0, s, gf, gc, (const float *)zc,
                               (float *)z);
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_bresid64(const Matrix &A, int K, int R, const double *x, const double *b, double *r,
                     double *partials, Ctrl *ctrl, int m, hipStream_t s)
{
    with_kr(K, R, [&](auto kc, auto rc) {
        constexpr int KK = decltype(kc)::value, RR = decltype(rc)::value;
        hipLaunchKernelGGL((k_bresid64<KK, RR>), dim3(lanes_grid(A.g.N, KK, RR)), dim3(kBlock), 0, s, A.g.N,
                           A.clog2, tile_remap(A), A.v64, (const int *)A.col, A.d64, x, b, r);
    });
    HPGMX_LAUNCH_CHECK();
    launch_norm64(A.g.N * K, K, r, partials, ctrl, kFinishResid, m, s);
}

void launch_bnat2int(const Geom &g, Prec src, Prec dst, int K, int nrhs, const void *nat, void *in,
                     hipStream_t s)
{
    const dim3 gr(grid_for(g.N)), bl(kBlock);
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        const bool s64 = src == P64, d64 = dst == P64;
        if (s64 && d64) hipLaunchKernelGGL((k_bnat2int<double, double, KK>), gr, bl, 0, s, g, nrhs, (const double *)nat, (double *)in);
        else if (s64) hipLaunchKernelGGL((k_bnat2int<double, float, KK>), gr, bl, 0, s, g, nrhs, (const double *)nat, (float *)in);
        else if (d64) hipLaunchKernelGGL((k_bnat2int<float, double, KK>), gr, bl, 0, s, g, nrhs, (const float *)nat, (double *)in);
        else hipLaunchKernelGGL((k_bnat2int<float, float, KK>), gr, bl, 0, s, g, nrhs, (const float *)nat, (float *)in);
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_bint2nat(const Geom &g, Prec src, Prec dst, int K, int nrhs, const void *in, void *nat,
                     hipStream_t s)
{
    const dim3 gr(grid_for(g.N)), bl(kBlock);
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        const bool s64 = src == P64, d64 = dst == P64;
        if (s64 && d64) hipLaunchKernelGGL((k_bint2nat<double, double, KK>), gr, bl, 0, s, g, nrhs, (const double *)in, (double *)nat);
        else if (s64) hipLaunchKernelGGL((k_bint2nat<double, float, KK>), gr, bl, 0, s, g, nrhs, (const double *)in, (float *)nat);
        else if (d64) hipLaunchKernelGGL((k_bint2nat<float, double, KK>), gr, bl, 0, s, g, nrhs, (const float *)in, (double *)nat);
        else hipLaunchKernelGGL((k_bint2nat<float, float, KK>), gr, bl, 0, s, g, nrhs, (const float *)in, (float *)nat);
    });
    HPGMX_LAUNCH_CHECK();
}

}  // namespace hpgmx
