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

// The single FP32 solve (K = 1) runs the passes with two consecutive elements
// per lane (8-byte loads, about 5 % faster than 4-byte ones on a 30-column
// pass); the basis columns start at even offsets (even leading dimension),
// and an odd length leaves its last element to lane 0 of workgroup 0.
// Batches keep one element per lane, so that a lane stays on one
// right-hand side.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T, int K> constexpr bool pair_lanes() { return K == 1 && sizeof(T) == 4; }
template <typename T> __device__ __forceinline__ f32x2 ld_pair(const T *col, i64 pe)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(col) + pe);
}

// ---- h1 = Q_{1:kb}^T w per right-hand side (the first GEMVT of a batch, whose
// SpMV runs in its own kernel) ----
template <typename T, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_dot(i64 M, const T *__restrict__ Q, i64 ldq, int kb,
                                                const T *__restrict__ w, double *partials)
{
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K>()) {
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j].x * (double)x.x + (double)q[j].y * (double)x.y;
        }
        e = (M & 1) && blockIdx.x == 0 && threadIdx.x == 0 ? M - 1 : M;
    }
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
    const double *cj = c + rhs_of_thread<K>();
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K>()) {
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
            double v0 = (double)x.x, v1 = (double)x.y;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                v0 -= cj[j * K] * (double)q[j].x;
                v1 -= cj[j * K] * (double)q[j].y;
            }
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += (double)q[j].x * v0 + (double)q[j].y * v1;
        }
        e = (M & 1) && blockIdx.x == 0 && threadIdx.x == 0 ? M - 1 : M;
    }
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

// ---- w -= Q (h1 + h2) fused with ||w||^2, then the Givens step ----------------------------
template <typename T, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_cgs_norm(i64 M, const T *__restrict__ Q, i64 ldq, int kb,
                                                     T *__restrict__ w, double *partials,
                                                     const Ctrl *ctrl)
{
    __shared__ double c[KB * K];
    stage_coefs<KB, K>(c, ctrl, kb, kCoefH12);
    const double *cj = c + rhs_of_thread<K>();
    double acc[1] = {0.0};
    const i64 stride = (i64)gridDim.x * kBlock;
    i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (pair_lanes<T, K>()) {
        for (; e < M / 2; e += stride) {
            f32x2 q[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) q[j] = ld_pair(Q + col_off(j, kb, ldq), e);
            const f32x2 x = ld_pair(w, e);
            sched_fence();
            double v0 = (double)x.x, v1 = (double)x.y;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                v0 -= cj[j * K] * (double)q[j].x;
                v1 -= cj[j * K] * (double)q[j].y;
            }
            f32x2 o;
            o.x = (float)v0;
            o.y = (float)v1;
            __builtin_nontemporal_store(o, reinterpret_cast<f32x2 *>(w) + e);
            acc[0] += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
        }
        e = (M & 1) && blockIdx.x == 0 && threadIdx.x == 0 ? M - 1 : M;
    }
    for (; e < M; e += stride) {
        T q[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) q[j] = ld_stream(Q + col_off(j, kb, ldq) + e);
        double v = (double)ld_stream(w + e);
        sched_fence();
#pragma unroll
        for (int j = 0; j < KB; ++j) v -= cj[j * K] * (double)q[j];
        const T vt = (T)v;
        w[e] = vt;
        acc[0] += (double)vt * (double)vt;
    }
    store_partials_g<1, K, 1>(acc, 1, partials);
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
