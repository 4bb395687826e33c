// Krylov-side kernels of Alg. 3: the first CGS2 inner products, the two
// fused CGS2 update passes (the new basis vector is stored unnormalised, see
// Ctrl), the FP64 outer residual, the projected least-squares solve, the
// basis combination and the mixed-precision solution update.
//
// Reductions (inner products and norms) are deterministic: every workgroup
// of a fixed-size grid-stride launch writes its partial sums, and a finish
// kernel (one workgroup per right-hand side) adds them in workgroup order.
// The kernel boundary makes the partial sums visible, so the streaming
// kernels need no device-scope fences (on gfx950 a device-scope release
// writes back the XCD's L2, which costs far more than the extra launch).
// The Givens update of the Hessenberg column (Alg. 3, "Update QR with
// Given's rotations") runs in FP64 in the finish kernel of the norm pass, so
// the whole inner step needs no host round trip except the small
// residual-estimate read.
//
// The vector passes also serve K interleaved right-hand sides (see
// krylov_device.hpp); the batched instances of the CGS2 passes are compiled
// in krylov_batch.hip.
#include "krylov_device.hpp"

#include <cmath>
#include <cstdlib>
#include <stdexcept>
#include <type_traits>

namespace hpgmx {

int red_blocks(i64 N)
{
    const i64 b = (N + kBlock - 1) / kBlock;
    return (int)(b < kMaxRedBlocks ? (b < 1 ? 1 : b) : kMaxRedBlocks);
}

// Givens update of Hessenberg column k (0-based) in FP64, by one workgroup:
// H(0:k,k) = h1 + h2, H(k+1,k) = beta; rotate by the earlier rotations (each
// rotation reads both entries before writing either); form the rotation that
// annihilates H(k+1,k); update t and the residual estimate rho = |t(k+1)|.
// The inputs are staged in LDS by all threads, the rotation chain runs in one
// thread out of LDS and registers, and the results are written back in
// parallel (a single thread reading global memory would wait on every load).
__device__ void givens_column(Ctrl *c, int k, int m, double nrm2)
{
    __shared__ double hk[kMaxBasis + 1], cs[kMaxBasis], sn[kMaxBasis], tk[2];
    const int t = threadIdx.x;
    const double beta = sqrt(nrm2);
    if (t <= k) hk[t] = c->h1[t] + c->h2[t];
    if (t < k) {
        cs[t] = c->cs[t];
        sn[t] = c->sn[t];
    }
    if (t == 0) {
        hk[k + 1] = beta;
        tk[0] = c->t[k];
    }
    __syncthreads();
    double *Hb = c->Hbar + (i64)k * (m + 1);
    if (t <= k + 1) Hb[t] = hk[t];  // unrotated column
    if (t == 0) {
        double a = hk[0];
        for (int j = 0; j < k; ++j) {
            const double b = hk[j + 1];
            hk[j] = cs[j] * a + sn[j] * b;
            a = -sn[j] * a + cs[j] * b;
        }
        const double bk = hk[k + 1];
        const double mu = sqrt(a * a + bk * bk);
        double ck = 1.0, sk = 0.0;
        if (mu > 0.0) {
            ck = a / mu;
            sk = bk / mu;
        }
        cs[k] = ck;
        sn[k] = sk;
        hk[k] = mu;
        hk[k + 1] = 0.0;
        const double t0 = tk[0];
        tk[0] = ck * t0;
        tk[1] = -sk * t0;
        c->rho = fabs(tk[1]);
        c->beta = beta;
        c->nrm2 = nrm2;
        c->breakdown = !(beta > 1e-300);
        c->inv_beta = c->breakdown ? 0.0 : 1.0 / beta;
        c->colscale[k + 1] = c->inv_beta;  // q_{k+1} = w / beta, stored as w
        c->nonfinite = !isfinite(nrm2);
    }
    __syncthreads();
    double *Hk = c->H + (i64)k * (m + 1);
    if (t <= k + 1) Hk[t] = hk[t];
    if (t == 0) {
        c->cs[k] = cs[k];
        c->sn[k] = sn[k];
        c->t[k] = tk[0];
        c->t[k + 1] = tk[1];
    }
}

// ---- FP64 outer residual r = b - A x with ||r||^2 (Alg. 3, residual step) ----
template <bool C16>
__global__ __launch_bounds__(kBlock) void k_resid64(Geom g, int clog2, int remap, const double *__restrict__ offv,
                                                    const void *__restrict__ offc, const int *__restrict__ cmap,
                                                    const double *__restrict__ diag,
                                                    const double *__restrict__ x,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ r, double *partials)
{
    __shared__ int cm[C16 ? kColMapSize : 1];
    if constexpr (C16) stage_colmap(cm, cmap);
    const i64 N = g.N;
    double acc[1] = {0.0};
    RowLoop rl = row_loop(N, remap);
    i64 p;
    while (rl.next(p)) {
        const EllRow er = ell_row(p, N, clog2);
        const double bp = b[p];
        const int *Dc = C16 ? cm + row_colour(g, p) * kSlots : nullptr;
        const double rv = bp - spmv_row_value<double>(ld_stream(diag + p), x[p],
                                                      ell_row_dot<double, double, kAllSlots, C16>(offv, offc, x, er, p, Dc, N),
                                                      nullptr);
        __builtin_nontemporal_store(rv, r + p);
        acc[0] += rv * rv;
    }
    store_partials_g<1, 1, 1>(acc, 1, partials);
}

// ---- rho0 = ||b|| (Alg. 3, first step) -----------------------------------------------------------
template <int K>
__global__ __launch_bounds__(kBlock) void k_norm64(i64 M, const double *__restrict__ v, double *partials)
{
    double acc[1] = {0.0};
    const i64 stride = (i64)gridDim.x * kBlock;
    for (i64 e = (i64)blockIdx.x * kBlock + threadIdx.x; e < M; e += stride) acc[0] += v[e] * v[e];
    store_partials_g<1, K, 1>(acc, 1, partials);
}

// ---- finish kernel: add the partial sums of nb workgroups in order -------------------------
constexpr int kFinishThreads = 1024;

// Workgroup j finishes right-hand side j: partial columns i * K + j for
// i < kb, control block ctrl[j].  Wave w sums columns i = w, w + 16, ...;
// lane l adds workgroups l, l + 64, ... with four independent accumulators,
// then the wave adds its lanes.
__global__ __launch_bounds__(kFinishThreads) void k_finish(const double *__restrict__ partials,
                                                           int nb, int kb, int K, int mode, Ctrl *ctrl,
                                                           int k, int m)
{
    __shared__ double tot[kMaxBasis];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rhs = blockIdx.x;
    Ctrl *c = ctrl + rhs;
    for (int j = wave; j < kb; j += kFinishThreads / 64) {
        const double *col = partials + (i64)(j * K + rhs) * kMaxRedBlocks;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int b = lane;
        for (; b + 192 < nb; b += 256) {
            s0 += col[b];
            s1 += col[b + 64];
            s2 += col[b + 128];
            s3 += col[b + 192];
        }
        for (; b < nb; b += 64) s0 += col[b];
        const double s = wave_sum((s0 + s1) + (s2 + s3));
        if (lane == 0) tot[j] = s;
    }
    __syncthreads();
    switch (mode) {
    case kFinishH1:  // the sums are over stored columns: apply their scales
        if ((int)threadIdx.x < kb) c->h1[threadIdx.x] = tot[threadIdx.x] * c->colscale[threadIdx.x];
        break;
    case kFinishH2:
        if ((int)threadIdx.x < kb) c->h2[threadIdx.x] = tot[threadIdx.x] * c->colscale[threadIdx.x];
        break;
    case kFinishNormGivens:
        givens_column(c, k, m, tot[0]);
        break;
    case kFinishResid:
        // start of a cycle: rho = ||r||, t = (rho, 0, ..., 0)
        if ((int)threadIdx.x < kMaxBasis) c->t[threadIdx.x] = threadIdx.x == 0 ? sqrt(tot[0]) : 0.0;
        if (threadIdx.x == 0) {
            const double rho = sqrt(tot[0]);
            c->nrm2 = tot[0];
            c->rho = rho;
            c->inv_rho = rho > 0.0 ? 1.0 / rho : 0.0;
            c->nonfinite = !isfinite(rho);
            c->breakdown = 0;
            c->colscale[0] = 1.0;  // q_1 is cast already divided by rho
        }
        break;
    case kFinishRho0:
        if (threadIdx.x == 0) {
            c->nrm2 = tot[0];
            c->rho0 = sqrt(tot[0]);
            c->nonfinite = !isfinite(c->rho0);
        }
        break;
    case kFinishCorr:
        if ((int)threadIdx.x < kb) c->corr[threadIdx.x] = tot[threadIdx.x];
        break;
    }
}

thread_local void (*finish_hook)(void *) = nullptr;
thread_local void *finish_hook_arg = nullptr;

void launch_finish(const double *partials, int nb, int kb, int K, int mode, Ctrl *ctrl, int k, int m,
                   hipStream_t s)
{
    if (finish_hook) finish_hook(finish_hook_arg);
    hipLaunchKernelGGL(k_finish, dim3(K), dim3(kFinishThreads), 0, s, partials, nb, kb, K, mode, ctrl,
                       k, m);
    HPGMX_LAUNCH_CHECK();
}

// ---- stencil correlation for the adjoint gradient -------------------------------------------
// acc[t] = sum_p lam_p x_{col(p,t)} for the 26 off-diagonal slots and
// acc[13] = sum_p lam_p x_p; padded slots read the zero entry x_N.
template <bool C16>
__global__ __launch_bounds__(kBlock) void k_stencil_corr(Geom g, int clog2, const void *__restrict__ offc,
                                                         const int *__restrict__ cmap,
                                                         const double *__restrict__ lam,
                                                         const double *__restrict__ x,
                                                         double *partials)
{
    __shared__ int cm[C16 ? kColMapSize : 1];
    if constexpr (C16) stage_colmap(cm, cmap);
    const i64 N = g.N;
    double acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.0;
    const i64 stride = (i64)gridDim.x * kBlock;
    for (i64 p = (i64)blockIdx.x * kBlock + threadIdx.x; p < N; p += stride) {
        const EllRow er = ell_row(p, N, clog2);
        const double l = lam[p];
        int ci[kSlots];
        if constexpr (C16) {
            const int *Dc = cm + row_colour(g, p) * kSlots;
            unsigned w[kPairs];
            load_pairs<kAllSlots>(static_cast<const unsigned *>(offc), er, w);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) ci[s] = ell_col(pair_half(w[s >> 1], s), p, Dc[s], N);
        } else {
#pragma unroll
            for (int s = 0; s < kSlots; ++s)
                ci[s] = ld_stream(static_cast<const int *>(offc) + er.base + (i64)s * er.stride);
        }
        const double xp = x[p];
        sched_fence();
        double xv[kSlots];
#pragma unroll
        for (int s = 0; s < kSlots; ++s) xv[s] = x[ci[s]];
        sched_fence();
        acc[13] += l * xp;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) acc[s < 13 ? s : s + 1] += l * xv[s];
    }
    store_partials_g<27, 1, 1>(acc, 27, partials);
}

// ---- q_1 = r / rho in the inner dtype --------------------------------------------------------------
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_cast(i64 M, const double *__restrict__ r,
                                                 const Ctrl *ctrl, T *__restrict__ q)
{
    const double s = ctrl[rhs_of_thread<K>()].inv_rho;
    const i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if (e < M) __builtin_nontemporal_store((T)(r[e] * s), q + e);
}

// ---- y = H(0:kk,0:kk)^{-1} t(0:kk) by back substitution (FP64) ----
// Workgroup j solves for right-hand side j with kk = kc.v[j] columns.
// Column-oriented: y_i = t_i / H_ii, then every row above subtracts H_ji y_i
// in parallel; the triangle and t live in LDS.  Entries kk..kMaxBasis-1 of
// y are set to zero, so a basis combination over more columns than kk adds
// nothing for them.
__global__ __launch_bounds__(kMaxBasis) void k_trsm(Ctrl *ctrl, KCount kc, int m)
{
    __shared__ double Hs[kMaxBasis][kMaxBasis + 1], ts[kMaxBasis], ys[kMaxBasis];
    Ctrl *c = ctrl + blockIdx.x;
    const int kk = kc.v[blockIdx.x];
    const int t = threadIdx.x;
    for (int j = 0; j < kk; ++j)
        if (t <= j) Hs[t][j] = c->H[(i64)j * (m + 1) + t];
    if (t < kk) ts[t] = c->t[t];
    __syncthreads();
    for (int i = kk - 1; i >= 0; --i) {
        const double yi = ts[i] / Hs[i][i];  // ts[i] is not written in this step
        if (t < i) ts[t] -= Hs[t][i] * yi;
        if (t == 0) ys[i] = yi;
        __syncthreads();
    }
    c->y[t] = t < kk ? ys[t] : 0.0;
}

// ---- u = Q(:,0:kk) y ------------------------------------------------------------------------------
// Runs once per restart cycle, so the column count is a runtime loop.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_gemv(i64 M, const T *__restrict__ Q, i64 ldq, int kk,
                                                 const Ctrl *ctrl, T *__restrict__ u)
{
    __shared__ double c[kMaxBasis * K];
    stage_coefs<kMaxBasis, K>(c, ctrl, kk, kCoefY);
    const double *cj = c + rhs_of_thread<K>();
    const i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if (e >= M) return;
    double v = 0.0;
#pragma unroll 8
    for (int j = 0; j < kk; ++j) v += cj[j * K] * (double)ld_stream(Q + (i64)j * ldq + e);
    __builtin_nontemporal_store((T)v, u + e);
}

// ---- x += z with the sum in FP64 (Alg. 3: the update must be double) ----
// For the 16-bit hierarchy z is the correction times sigma: x += z / sigma
// (a power of two, so the product is exact).
template <typename T> __device__ __forceinline__ double widen(T v) { return (double)to_t<float>(v); }
template <> __device__ __forceinline__ double widen<double>(double v) { return v; }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(i64 M, const T *__restrict__ z, double *__restrict__ x,
                                                   const double *inv)
{
    const i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if (e >= M) return;
    const double v = widen(z[e]);
    __builtin_nontemporal_store(x[e] + (inv ? v * *inv : v), x + e);
}

// ---- the V-cycle input of the 16-bit hierarchy -----------------------------------------------
// r0 = sigma v rounded to S, sigma = 2^e the power of two nearest
// sqrt(N) / ||v||, so that r0's entries are of order one: binary16 has 11
// significant bits but its normal range starts at 2^-14, below which entries
// of a unit vector of millions of entries would lose their precision.  The
// product sigma v is exact (a power of two), so each entry is rounded once.
__device__ __forceinline__ double pow2_near(double v)
{
    if (!(v > 0.0) || !isfinite(v)) return 1.0;
    return ldexp(1.0, (int)rint(log2(v)));
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_cast_mg(i64 N, const float *__restrict__ v, Ctrl *ctrl, int end,
                                                    int k, double sqrtN, S *__restrict__ r0)
{
    double sigma;
    if (!end) {
        const double cs = ctrl->colscale[k];  // ||v|| = 1 / colscale[k]
        sigma = pow2_near(sqrtN * cs);
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->mg_post = cs / sigma;
    } else {
        double y2 = 0.0;  // v = Q y with orthonormal q_j: ||v|| = ||y|| up to rounding
        for (int j = 0; j < k; ++j) y2 += ctrl->y[j] * ctrl->y[j];
        sigma = pow2_near(sqrtN / sqrt(y2));
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->mg_inv = 1.0 / sigma;
    }
    const float sg = (float)sigma;
    const i64 e = (i64)blockIdx.x * kBlock + threadIdx.x;
    if (e < N) st_stream(r0 + e, from_t<S>(v[e] * sg));  // read by the V-cycle that follows
}

// ---- streaming copy (bandwidth reference) -------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// One 16-byte element per lane over a full grid: consecutive workgroups write
// consecutive 4 KB runs, the pattern that streams fastest on MI355X.
__global__ __launch_bounds__(kBlock) void k_copy(i64 n16, const u32x4 *__restrict__ src, u32x4 *__restrict__ dst)
{
    const i64 i = (i64)blockIdx.x * kBlock + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// =====================================================================================================
// launchers
static inline unsigned grid_n(i64 n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Basis counts: kernels are compiled for every KB = 1..32 columns (restart
// lengths up to 31 never read a column they do not use) and for buckets
// KB = 36, 40, ..., 64 above, where columns kb..KB-1 re-read column kb-1
// from cache.  (Buckets of four throughout cost the 30-step cycle's passes
// about 4 % of their bandwidth.)
#define HPGMX_KB_EXACT(N_)                  \
    case N_: {                              \
        constexpr int KB = N_;              \
        HPGMX_KB_BODY;                      \
    } break;
#define HPGMX_KB_CASE(N_)                   \
    case N_: {                              \
        constexpr int KB = 4 * N_;          \
        HPGMX_KB_BODY;                      \
    } break;
#define HPGMX_KB_SWITCH(kb)                                                                       \
    if ((kb) >= 1 && (kb) <= 32) {                                                                \
        switch (kb) {                                                                             \
            HPGMX_KB_EXACT(1) HPGMX_KB_EXACT(2) HPGMX_KB_EXACT(3) HPGMX_KB_EXACT(4)               \
            HPGMX_KB_EXACT(5) HPGMX_KB_EXACT(6) HPGMX_KB_EXACT(7) HPGMX_KB_EXACT(8)               \
            HPGMX_KB_EXACT(9) HPGMX_KB_EXACT(10) HPGMX_KB_EXACT(11) HPGMX_KB_EXACT(12)            \
            HPGMX_KB_EXACT(13) HPGMX_KB_EXACT(14) HPGMX_KB_EXACT(15) HPGMX_KB_EXACT(16)           \
            HPGMX_KB_EXACT(17) HPGMX_KB_EXACT(18) HPGMX_KB_EXACT(19) HPGMX_KB_EXACT(20)           \
            HPGMX_KB_EXACT(21) HPGMX_KB_EXACT(22) HPGMX_KB_EXACT(23) HPGMX_KB_EXACT(24)           \
            HPGMX_KB_EXACT(25) HPGMX_KB_EXACT(26) HPGMX_KB_EXACT(27) HPGMX_KB_EXACT(28)           \
            HPGMX_KB_EXACT(29) HPGMX_KB_EXACT(30) HPGMX_KB_EXACT(31) HPGMX_KB_EXACT(32)           \
        }                                                                                         \
    } else {                                                                                      \
        switch (((kb) + 3) / 4) {                                                                 \
            HPGMX_KB_CASE(9) HPGMX_KB_CASE(10) HPGMX_KB_CASE(11) HPGMX_KB_CASE(12)                \
            HPGMX_KB_CASE(13) HPGMX_KB_CASE(14) HPGMX_KB_CASE(15) HPGMX_KB_CASE(16)               \
        default: throw std::runtime_error("basis size out of range");                             \
        }                                                                                         \
    }

// Interleave widths: K = 1 (single solve) and the batch widths 2, 4, 8.
template <typename F> static void with_k(int K, F &&f)
{
    switch (K) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: throw std::runtime_error("unsupported batch width");
    }
}

// The FP32 passes load element pairs (pair_lanes): columns must start on
// 8-byte boundaries.
static void check_pair_layout(Prec p, const void *Q, i64 ldq, const void *w)
{
    if (p == P64) return;
    if ((ldq & 1) || ((uintptr_t)Q & 7) || ((uintptr_t)w & 7))
        throw std::runtime_error("Krylov basis columns must start on 8-byte boundaries");
}

void launch_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, const void *w, double *partials,
                Ctrl *ctrl, hipStream_t s)
{
    check_pair_layout(p, Q, ldq, w);
    if (K > 1) return batch_dot(M, K, p, Q, ldq, kb, w, partials, ctrl, s);
    const dim3 gr(red_blocks(M)), bl(kBlock);
    if (p == P64) {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_dot<double, KB, 1>), gr, bl, 0, s, M, (const double *)Q, ldq, kb, (const double *)w, partials)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    } else {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_dot<float, KB, 1>), gr, bl, 0, s, M, (const float *)Q, ldq, kb, (const float *)w, partials)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    }
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, kb, 1, kFinishH1, ctrl, 0, 0, s);
}

void launch_cgs_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                    Ctrl *ctrl, hipStream_t s)
{
    check_pair_layout(p, Q, ldq, w);
    if (K > 1) return batch_cgs_dot(M, K, p, Q, ldq, kb, w, partials, ctrl, s);
    const dim3 gr(red_blocks(M)), bl(kBlock);
    if (p == P64) {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_dot<double, KB, 1>), gr, bl, 0, s, M, (const double *)Q, ldq, kb, (const double *)w, partials, ctrl)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    } else {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_dot<float, KB, 1>), gr, bl, 0, s, M, (const float *)Q, ldq, kb, (const float *)w, partials, ctrl)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    }
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, kb, 1, kFinishH2, ctrl, 0, 0, s);
}

void launch_cgs_norm(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                     Ctrl *ctrl, int k, int m, hipStream_t s)
{
    check_pair_layout(p, Q, ldq, w);
    if (K > 1) return batch_cgs_norm(M, K, p, Q, ldq, kb, w, partials, ctrl, k, m, s);
    const dim3 gr(red_blocks(M)), bl(kBlock);
    if (p == P64) {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_norm<double, KB, 1>), gr, bl, 0, s, M, (const double *)Q, ldq, kb, (double *)w, partials, ctrl)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    } else {
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_norm<float, KB, 1>), gr, bl, 0, s, M, (const float *)Q, ldq, kb, (float *)w, partials, ctrl)
        HPGMX_KB_SWITCH(kb)
#undef HPGMX_KB_BODY
    }
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, 1, 1, kFinishNormGivens, ctrl, k, m, s);
}

void launch_resid64(const Matrix &A, const double *x, const double *b, double *r,
                    double *partials, Ctrl *ctrl, int m, hipStream_t s)
{
    const unsigned nb = (unsigned)red_blocks(A.g.N);
    with_cols(A, [&](auto c16) {
        hipLaunchKernelGGL(k_resid64<decltype(c16)::value>, dim3(nb), dim3(kBlock), 0, s, A.g, A.clog2,
                           tile_remap(A), A.v64, (const void *)A.col, A.cmap, A.d64, x, b, r, partials);
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)nb, 1, 1, kFinishResid, ctrl, 0, m, s);
}

void launch_norm64(i64 M, int K, const double *v, double *partials, Ctrl *ctrl, int mode, int m,
                   hipStream_t s)
{
    const unsigned nb = (unsigned)red_blocks(M);
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        hipLaunchKernelGGL((k_norm64<KK>), dim3(nb), dim3(kBlock), 0, s, M, v, partials);
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)nb, 1, K, mode, ctrl, 0, m, s);
}

void launch_stencil_correlation(const Matrix &A, const double *lam, const double *x,
                                double *partials, Ctrl *ctrl, hipStream_t s)
{
    const unsigned nb = (unsigned)red_blocks(A.g.N);
    with_cols(A, [&](auto c16) {
        hipLaunchKernelGGL(k_stencil_corr<decltype(c16)::value>, dim3(nb), dim3(kBlock), 0, s, A.g, A.clog2,
                           (const void *)A.col, A.cmap, lam, x, partials);
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)nb, 27, 1, kFinishCorr, ctrl, 0, 0, s);
}

void launch_cast(i64 M, int K, Prec p, const double *r, const Ctrl *ctrl, void *q, hipStream_t s)
{
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (p == P64) hipLaunchKernelGGL((k_cast<double, KK>), dim3(grid_n(M)), dim3(kBlock), 0, s, M, r, ctrl, (double *)q);
        else hipLaunchKernelGGL((k_cast<float, KK>), dim3(grid_n(M)), dim3(kBlock), 0, s, M, r, ctrl, (float *)q);
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_trsm(Ctrl *ctrl, const KCount &kc, int K, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_trsm, dim3(K), dim3(kMaxBasis), 0, s, ctrl, kc, m);
    HPGMX_LAUNCH_CHECK();
}

void launch_gemv(i64 M, int K, Prec p, const void *Q, i64 ldq, int kk, const Ctrl *ctrl, void *u,
                 hipStream_t s)
{
    if (kk < 0 || kk > kMaxBasis) throw std::runtime_error("basis size out of range");
    const dim3 gr(grid_n(M)), bl(kBlock);
    with_k(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (p == P64)
            hipLaunchKernelGGL((k_gemv<double, KK>), gr, bl, 0, s, M, (const double *)Q, ldq, kk, ctrl, (double *)u);
        else
            hipLaunchKernelGGL((k_gemv<float, KK>), gr, bl, 0, s, M, (const float *)Q, ldq, kk, ctrl, (float *)u);
    });
    HPGMX_LAUNCH_CHECK();
}

void launch_update(i64 M, Prec p, const void *z, double *x, hipStream_t s, const Ctrl *ctrl)
{
    const dim3 gr(grid_n(M)), bl(kBlock);
    const double *inv = ctrl && mg16(p) ? &ctrl->mg_inv : nullptr;
    switch (p) {
    case P64: hipLaunchKernelGGL(k_update<double>, gr, bl, 0, s, M, (const double *)z, x, inv); break;
    case P16V: hipLaunchKernelGGL(k_update<__half>, gr, bl, 0, s, M, (const __half *)z, x, inv); break;
    case PB16V: hipLaunchKernelGGL(k_update<bf16>, gr, bl, 0, s, M, (const bf16 *)z, x, inv); break;
    default: hipLaunchKernelGGL(k_update<float>, gr, bl, 0, s, M, (const float *)z, x, inv); break;
    }
    HPGMX_LAUNCH_CHECK();
}

void launch_cast_mg(i64 N, Prec p, const float *v, Ctrl *ctrl, bool end_of_cycle, int k, void *r0, hipStream_t s)
{
    const double sqrtN = std::sqrt((double)N);
    if (p == P16V)
        hipLaunchKernelGGL(k_cast_mg<__half>, dim3(grid_n(N)), dim3(kBlock), 0, s, N, v, ctrl, (int)end_of_cycle, k,
                           sqrtN, (__half *)r0);
    else if (p == PB16V)
        hipLaunchKernelGGL(k_cast_mg<bf16>, dim3(grid_n(N)), dim3(kBlock), 0, s, N, v, ctrl, (int)end_of_cycle, k,
                           sqrtN, (bf16 *)r0);
    else
        throw std::runtime_error("launch_cast_mg: not a 16-bit hierarchy precision");
    HPGMX_LAUNCH_CHECK();
}

void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const i64 n16 = (i64)(bytes / 16);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n16 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n16,
                       (const u32x4 *)src, (u32x4 *)dst);
    HPGMX_LAUNCH_CHECK();
}

}  // namespace hpgmx
