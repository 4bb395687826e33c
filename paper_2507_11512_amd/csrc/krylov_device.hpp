// Device templates of the Krylov vector passes, shared by the single-solve
// and the batched translation units: the first GEMVT of a batch, the two
// fused CGS2 update passes and the reduction helpers they use.
//
// The vector kernels serve K right-hand sides stored interleaved (element
// e = p * K + j is row p of right-hand side j).  They run one lane per
// element; since K divides the workgroup size, a lane's right-hand side is
// threadIdx.x % K for the whole grid-stride loop, and each right-hand side
// has its own control block ctrl[j] (coefficients, Hessenberg matrix,
// rotations).  K = 1 is the single solve.
#pragma once

#include "ell_device.hpp"

namespace hpgmx {

// ---- reduction helpers -------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int K> __device__ __forceinline__ int rhs_of_thread() { return (int)(threadIdx.x & (K - 1)); }

// Coefficient arrays of the control block staged by the CGS and GEMV passes.
enum CoefSel { kCoefH1, kCoefH12, kCoefY };

// c[i * K + j] = coefficient i of right-hand side j for the stored
// (unnormalised) column i: the coefficient of q_i times colscale[i]
// (0 for i >= kb).
template <int KB, int K>
__device__ __forceinline__ void stage_coefs(double *c, const Ctrl *ctrl, int kb, CoefSel sel)
{
    for (int t = threadIdx.x; t < KB * K; t += kBlock) {
        const int i = t / K, j = t % K;
        double v = 0.0;
        if (i < kb) {
            const Ctrl &cj = ctrl[j];
            v = sel == kCoefH1 ? cj.h1[i] : sel == kCoefH12 ? cj.h1[i] + cj.h2[i] : cj.y[i];
            v *= cj.colscale[i];
        }
        c[t] = v;
    }
    __syncthreads();
}

// Column j of the basis for a kernel compiled for KB columns: loads are
// issued for all KB columns unconditionally (so they can all be in flight at
// once); columns at or beyond kb re-read column kb-1 from cache and carry a
// zero coefficient.  The passes stream the basis and w with nontemporal
// loads: neither is reused before it has left the caches, and the hint lets
// a streaming read run about 11 % faster on MI355X.
__device__ __forceinline__ i64 col_off(int j, int kb, i64 ldq) { return (i64)(j < kb ? j : kb - 1) * ldq; }

// FP32 passes take two consecutive elements per lane (8-byte loads, about
// 5 % faster than 4-byte ones on a 30-column pass).  For K = 1 both belong
// to the one right-hand side; for K >= 2 (K even, entries interleaved) they
// are right-hand sides 2g and 2g + 1 with g = lane % (K / 2), so a lane keeps
// two sets of accumulators.  The update pass (one accumulator per
// right-hand side) does so for every K; the two GEMVT passes (kb
// accumulators per right-hand side) only for K = 1: twice kb FP64
// accumulators leave one or two wavefronts per SIMD, and the batched passes
// gained nothing.  Basis columns start at even offsets (even leading
// dimension); an odd length (K = 1 only) leaves its last element to lane 0
// of workgroup 0.  FP64 passes keep one element per lane.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T, int K, bool PER_COLUMN> constexpr bool pair_lanes()
{
    return sizeof(T) == 4 && (K == 1 || !PER_COLUMN);
}
template <int K> constexpr int rhs_per_lane() { return K == 1 ? 1 : 2; }
// First right-hand side of the lane's pair.
template <int K> __device__ __forceinline__ int pair_rhs0() { return K == 1 ? 0 : 2 * (int)(threadIdx.x % (K / 2)); }
template <typename T> __device__ __forceinline__ f32x2 ld_pair(const T *col, i64 pe)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(col) + pe);
}
// Partial sums of a pair-lane pass: accumulator a = NR i + r holds
// coefficient i of right-hand side pair_rhs0 + r (column i K + j).
template <int NA, int K>
__device__ __forceinline__ void store_pair_partials(const double (&acc)[NA], int na, double *partials)
{
    if constexpr (K == 1) store_partials_g<NA, 1, 1>(acc, na, partials);
    else store_partials_g<NA, K / 2, 2>(acc, na, partials);
}

// ---- h1 = Q_{1:kb}^T w per right-hand side (the first GEMVT of a batch, whose
// SpMV runs in its own kernel) ----
template <typename T, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_dot(i64 M, const T *__restrict__ Q, i64 ldq, int kb,
                                                const T *__restrict__ w, double *partials)
{
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K, true>()) {  // K = 1
        double acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0.0;
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j].x * (double)x.x + (double)q[j].y * (double)x.y;
        }
        if ((M & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const double x = (double)w[M - 1];
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)Q[col_off(j, kb, ldq) + M - 1] * x;
        }
        store_partials_g<KB, 1, 1>(acc, kb, partials);
    } else {
        double acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0.0;
        for (; e < M; e += stride) {
            T q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_stream(Q + col_off(j, kb, ldq) + e);
            const double vd = (double)ld_stream(w + e);
            sched_fence();
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j] * vd;
        }
        store_partials_g<KB, K, 1>(acc, kb, partials);
    }
}

// ---- h2 = Q^T (w - Q h1) (the reorthogonalisation GEMV and GEMVT) ----
// w - Q h1 is kept in FP64 in registers and not stored: the norm pass forms
// w - Q (h1 + h2) from the original w, which is the same vector in exact
// arithmetic, rounds to the storage type once instead of twice, and saves
// one write of w per step.
template <typename T, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_cgs_dot(i64 M, const T *__restrict__ Q, i64 ldq, int kb,
                                                    const T *__restrict__ w, double *partials,
                                                    const Ctrl *ctrl)
{
    __shared__ double c[KB * K];
    stage_coefs<KB, K>(c, ctrl, kb, kCoefH1);
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K, true>()) {  // K = 1
        double acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0.0;
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
            double v0 = (double)x.x, v1 = (double)x.y;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                v0 -= c[j] * (double)q[j].x;
                v1 -= c[j] * (double)q[j].y;
            }
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j].x * v0 + (double)q[j].y * v1;
        }
        if ((M & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            double v = (double)w[M - 1];
#pragma unroll
            for (int j = 0; j < KB; ++j) v -= c[j] * (double)Q[col_off(j, kb, ldq) + M - 1];
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)Q[col_off(j, kb, ldq) + M - 1] * v;
        }
        store_partials_g<KB, 1, 1>(acc, kb, partials);
    } else {
        const double *cj = c + rhs_of_thread<K>();
        double acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0.0;
        for (; e < M; e += stride) {
            T q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_stream(Q + col_off(j, kb, ldq) + e);
            double v = (double)ld_stream(w + e);
            sched_fence();
#pragma unroll
            for (int j = 0; j < KB; ++j) v -= cj[j * K] * (double)q[j];
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j] * v;
        }
        store_partials_g<KB, K, 1>(acc, kb, partials);
    }
}

// ---- w -= Q (h1 + h2) fused with ||w||^2, then the Givens step ----------------------------
template <typename T, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_cgs_norm(i64 M, const T *__restrict__ Q, i64 ldq, int kb,
                                                     T *__restrict__ w, double *partials,
                                                     const Ctrl *ctrl)
{
    __shared__ double c[KB * K];
    stage_coefs<KB, K>(c, ctrl, kb, kCoefH12);
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K, false>()) {
        constexpr int NR = rhs_per_lane<K>();
        const double *c0 = c + pair_rhs0<K>(), *c1 = c0 + (NR - 1);
        double acc[NR];
#pragma unroll
        for (int a = 0; a < NR; ++a) acc[a] = 0.0;
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
            double v0 = (double)x.x, v1 = (double)x.y;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                v0 -= c0[j * K] * (double)q[j].x;
                v1 -= c1[j * K] * (double)q[j].y;
            }
            f32x2 o;
            o.x = (float)v0;
            o.y = (float)v1;
            __builtin_nontemporal_store(o, reinterpret_cast<f32x2 *>(w) + e);
            acc[0] += (double)o.x * (double)o.x;
            acc[NR - 1] += (double)o.y * (double)o.y;
        }
        if (K == 1 && (M & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            double v = (double)w[M - 1];
#pragma unroll
            for (int j = 0; j < KB; ++j) v -= c0[j * K] * (double)Q[col_off(j, kb, ldq) + M - 1];
            const T vt = (T)v;
            w[M - 1] = vt;
            acc[0] += (double)vt * (double)vt;
        }
        store_pair_partials<NR, K>(acc, NR, partials);
    } else {
        const double *cj = c + rhs_of_thread<K>();
        double acc[1] = {0.0};
        for (; e < M; e += stride) {
            T q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_stream(Q + col_off(j, kb, ldq) + e);
            double v = (double)ld_stream(w + e);
            sched_fence();
#pragma unroll
            for (int j = 0; j < KB; ++j) v -= cj[j * K] * (double)q[j];
            const T vt = (T)v;
            __builtin_nontemporal_store(vt, w + e);
            acc[0] += (double)vt * (double)vt;
        }
        store_partials_g<1, K, 1>(acc, 1, partials);
    }
}

// Batched instances (K = 2, 4, 8) of the Krylov passes, compiled in
// krylov_batch.hip; each launches its finish kernel as the single-solve
// launchers do.
void batch_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, const void *w, double *partials,
               Ctrl *ctrl, hipStream_t s);
void batch_cgs_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                   Ctrl *ctrl, hipStream_t s);
void batch_cgs_norm(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                    Ctrl *ctrl, int k, int m, hipStream_t s);

}  // namespace hpgmx
