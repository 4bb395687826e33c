// Device-side helpers shared by the stencil and Krylov kernels: element loads
// and the ELL row product.
//
// Every kernel here is bound by HBM bandwidth, so what matters is how many
// loads each wavefront keeps in flight.  Left alone, the AMDGPU machine
// scheduler trades memory-level parallelism for registers and interleaves
// each load with its first use (load, wait, use, load, wait, ...), which
// serialises the memory latency of a row.  The helpers therefore issue all
// loads of a row first and fence them off with a scheduling barrier:
// values and column indices, then the gathers that depend on the indices,
// then the arithmetic.
#pragma once

#include "hpgmx_internal.hpp"

#include <stdexcept>
#include <type_traits>

namespace hpgmx {

template <typename V> struct VecT { using T = float; };
template <> struct VecT<double> { using T = double; };

// Matrix entries are read once per launch: non-temporal loads.
template <typename V> __device__ __forceinline__ V ld_stream(const V *p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ __half ld_stream<__half>(const __half *p)
{
    return __ushort_as_half(__builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p)));
}
template <> __device__ __forceinline__ bf16 ld_stream<bf16>(const bf16 *p)
{
    return __ushort_as_bfloat16(__builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p)));
}

// Results that a later kernel reads are written with nontemporal stores.  On
// MI355X a pass that streams data written just before with plain stores runs
// far below the streaming rate: a 4 GB read pass (31 Krylov columns) that
// includes a 131 MB vector written by the preceding kernel took 715 us after
// plain stores and 588 us after nontemporal ones, which cost the writing
// kernel 3 us.  Measured on whole solves (bit-identical): the 320^3 mixed-
// precision solve 1305 -> 1288 ms, FP64 2331 -> 2260 ms, the 192^3 x 8 batch
// 1106 -> 1081 ms.  The one exception is the batched smoother's z, which the
// next colour passes re-read: there plain stores measured faster.
template <typename S> __device__ __forceinline__ void st_stream(S *p, S v) { __builtin_nontemporal_store(v, p); }
template <> __device__ __forceinline__ void st_stream<__half>(__half *p, __half v)
{
    __builtin_nontemporal_store(__half_as_ushort(v), reinterpret_cast<unsigned short *>(p));
}
template <> __device__ __forceinline__ void st_stream<bf16>(bf16 *p, bf16 v)
{
    __builtin_nontemporal_store(__bfloat16_as_ushort(v), reinterpret_cast<unsigned short *>(p));
}

template <typename T, typename V> __device__ __forceinline__ T to_t(V v) { return (T)v; }
template <> __device__ __forceinline__ float to_t<float, __half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float to_t<float, bf16>(bf16 v) { return __bfloat162float(v); }

// Storing an FP32 result in a vector of element type S rounds to nearest
// even (IEEE) for the 16-bit types.
template <typename S, typename T> __device__ __forceinline__ S from_t(T v) { return (S)v; }
template <> __device__ __forceinline__ __half from_t<__half, float>(float v) { return __float2half(v); }
template <> __device__ __forceinline__ bf16 from_t<bf16, float>(float v) { return __float2bfloat16(v); }

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// acc + a x with one rounding.  The row products are written as explicit
// fused multiply-adds so that every kernel that forms a row sum (the SpMV,
// the smoother, their batched and fused variants) rounds it alike.
__device__ __forceinline__ float madd(float a, float x, float acc) { return __builtin_fmaf(a, x, acc); }
__device__ __forceinline__ double madd(double a, double x, double acc) { return __builtin_fma(a, x, acc); }

// Column of a slot from its 16-bit offset d (see ColMap): p + D + d, or the
// zero entry N for a padded slot.
__device__ __forceinline__ int ell_col(short d, i64 p, int D, i64 N)
{
    return d == (short)kPadOffset ? (int)N : (int)(p + D + d);
}

// The 16-bit offset of slot s from the row's pair words.
__device__ __forceinline__ short pair_half(unsigned w, int s)
{
    return (short)(unsigned short)((s & 1) ? (w >> 16) : (w & 0xffffu));
}

// Loads the pair words of the slots in MASK (a pair is loaded when either of
// its slots is in MASK).
template <unsigned MASK>
__device__ __forceinline__ void load_pairs(const unsigned *__restrict__ offc, const EllRow &er, unsigned (&w)[kPairs])
{
#pragma unroll
    for (int t = 0; t < kPairs; ++t)
        if (MASK & (3u << (2 * t))) w[t] = __builtin_nontemporal_load(offc + er.pbase + (i64)t * er.pstride);
}

// Colour block of row p (the number of block starts at or below p).
__device__ __forceinline__ int row_colour(const Geom &g, i64 p)
{
    int c = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i) c += p >= g.off[i] ? 1 : 0;
    return c;
}

// Kernels whose rows are of any colour read the column-offset table from LDS
// (each lane indexes it with its row's colour); call before any early exit.
__device__ __forceinline__ void stage_colmap(int *lds, const int *__restrict__ cmap)
{
    for (int t = threadIdx.x; t < kColMapSize; t += blockDim.x) lds[t] = cmap[t];
    __syncthreads();
}

// sum over the slots in MASK of a(p,s) * x[col(p,s)] (slot order), in the
// arithmetic type T; x may be stored in a narrower type X (the 16-bit
// multigrid vectors), widened after the gathers.  Columns: C16 = false,
// int32 indices (offc: int, laid out as the values); C16 = true, 16-bit
// offsets in pairs (offc: unsigned pair words), decoded with Dc, the column
// offsets D[c][.] of the row's colour, and N, the zero entry.
template <typename T, typename V, unsigned MASK, bool C16, typename X>
__device__ __forceinline__ T ell_row_dot(const V *__restrict__ offv, const void *__restrict__ offc,
                                         const X *x, const EllRow &er, i64 p, const int *Dc, i64 N)
{
    V a[kSlots];
    int ci[kSlots];
    unsigned w[kPairs];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            const i64 e = er.base + (i64)s * er.stride;
            a[s] = ld_stream(offv + e);
            if constexpr (!C16) ci[s] = ld_stream(static_cast<const int *>(offc) + e);
        }
    }
    if constexpr (C16) load_pairs<MASK>(static_cast<const unsigned *>(offc), er, w);
    sched_fence();
    X xv[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            if constexpr (C16) xv[s] = x[ell_col(pair_half(w[s >> 1], s), p, Dc[s], N)];
            else xv[s] = x[ci[s]];
        }
    }
    sched_fence();
    T acc = (T)0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (MASK & (1u << s)) acc = madd(to_t<T>(a[s]), to_t<T>(xv[s]), acc);
    return acc;
}

constexpr unsigned kAllSlots = (1u << kSlots) - 1u;

// One SpMV row from its parts: (a_pp x_p + acc) * scale, acc the slot sum of
// ell_row_dot.  Contraction is off so that the SpMV kernel and the last
// Gauss-Seidel colour launch, which computes the rows of its colour (see
// k_gs), round alike.
template <typename T>
__device__ __forceinline__ T spmv_row_value(T d, T x, T acc, const double *scale)
{
#pragma clang fp contract(off)
    const T v = d * x + acc;
    return scale ? v * (T)*scale : v;
}
// The -x and +x neighbours (slots 12 and 13): the only couplings between
// colours c and c ^ 1.
constexpr unsigned kXSlots = (1u << 12) | (1u << 13);

// Column of slot s of row p, decoded as ell_row_dot decodes it.
template <bool C16>
__device__ __forceinline__ i64 ell_slot_col(const void *__restrict__ offc, const EllRow &er, int s, i64 p,
                                            const int *Dc, i64 N)
{
    if constexpr (C16) {
        const unsigned w = __builtin_nontemporal_load(static_cast<const unsigned *>(offc) + er.pbase +
                                                      (i64)(s >> 1) * er.pstride);
        return ell_col(pair_half(w, s), p, Dc[s], N);
    } else {
        return ld_stream(static_cast<const int *>(offc) + er.base + (i64)s * er.stride);
    }
}

// As ell_row_dot over MASK, returning also accE, the sum over the slots of
// EMASK alone: two accumulations in slot order over the same loads (accE
// equals ell_row_dot over EMASK bit for bit).
template <typename T, typename V, unsigned MASK, unsigned EMASK, bool C16, typename X>
__device__ __forceinline__ T ell_row_dot2(const V *__restrict__ offv, const void *__restrict__ offc,
                                          const X *x, const EllRow &er, i64 p, const int *Dc, i64 N, T &accE)
{
    V a[kSlots];
    int ci[kSlots];
    unsigned w[kPairs];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            const i64 e = er.base + (i64)s * er.stride;
            a[s] = ld_stream(offv + e);
            if constexpr (!C16) ci[s] = ld_stream(static_cast<const int *>(offc) + e);
        }
    }
    if constexpr (C16) load_pairs<MASK>(static_cast<const unsigned *>(offc), er, w);
    sched_fence();
    X xv[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            if constexpr (C16) xv[s] = x[ell_col(pair_half(w[s >> 1], s), p, Dc[s], N)];
            else xv[s] = x[ci[s]];
        }
    }
    sched_fence();
    T acc = (T)0, ae = (T)0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) acc = madd(to_t<T>(a[s]), to_t<T>(xv[s]), acc);
        if (EMASK & MASK & (1u << s)) ae = madd(to_t<T>(a[s]), to_t<T>(xv[s]), ae);
    }
    accE = ae;
    return acc;
}

// As ell_row_dot, with the x-neighbour slots 12 and 13 (both in MASK) taking
// the values x12 and x13 instead of gathered ones; same operations in the
// same order.
template <typename T, typename V, unsigned MASK, bool C16, typename X>
__device__ __forceinline__ T ell_row_dot_x(const V *__restrict__ offv, const void *__restrict__ offc,
                                           const X *x, const EllRow &er, i64 p, const int *Dc, i64 N,
                                           X x12, X x13)
{
    static_assert((MASK & kXSlots) == kXSlots, "both x-neighbour slots must be in the mask");
    constexpr unsigned G = MASK & ~kXSlots;  // the gathered slots
    V a[kSlots];
    int ci[kSlots];
    unsigned w[kPairs];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            const i64 e = er.base + (i64)s * er.stride;
            a[s] = ld_stream(offv + e);
            if constexpr (!C16)
                if (G & (1u << s)) ci[s] = ld_stream(static_cast<const int *>(offc) + e);
        }
    }
    if constexpr (C16) load_pairs<G>(static_cast<const unsigned *>(offc), er, w);
    sched_fence();
    X xv[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (G & (1u << s)) {
            if constexpr (C16) xv[s] = x[ell_col(pair_half(w[s >> 1], s), p, Dc[s], N)];
            else xv[s] = x[ci[s]];
        }
    }
    xv[12] = x12;
    xv[13] = x13;
    sched_fence();
    T acc = (T)0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (MASK & (1u << s)) acc = madd(to_t<T>(a[s]), to_t<T>(xv[s]), acc);
    return acc;
}

// Calls f(std::true_type) for a matrix with 16-bit column offsets, else
// f(std::false_type) (the kernels' C16 parameter).
template <typename F> static void with_cols(const Matrix &A, F &&f)
{
    if (A.c16) f(std::true_type{});
    else f(std::false_type{});
}

// ---- XCD-aware work distribution -------------------------------------------------------
// MI355X dispatches workgroup b to XCD b % 8, and each XCD has its own L2.
// Row tiles that share gathered neighbours should therefore run on the same
// XCD: the remaps below give each XCD one contiguous range of row tiles, so
// the neighbour values a tile gathers are mostly already in that XCD's L2
// (they were fetched for the tiles before it).  Both remaps are permutations
// of the work, so results do not depend on whether the dispatch assumption
// holds.
constexpr unsigned kXcds = 8;

// Tile of a one-row-per-lane launch of nb workgroups.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb, int remap)
{
    if (!remap || nb < kXcds) return b;
    const unsigned x = b % kXcds, j = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + j;
}

// Slab order for the SpMV over all rows of every colour (remap ==
// kRemapSlab).  In the XCD-contiguous order XCD x owns tiles
// [x T/8, (x+1) T/8), which is colour block x when the eight blocks are
// equal: at any moment all eight XCDs work at the same spatial position of
// their blocks and gather the same neighbourhood of the vector.  In the slab
// order XCD x owns the x-th eighth of every colour block (a slab of
// k-planes), so the XCDs work on eight different slabs and spread their
// gathers over the vector.  The L2-to-fabric byte counters read the same in
// both orders (a slab does not fit an XCD's L2); the time does not: the FP32
// and 16-bit SpMV at 320^3 runs 6030 -> 6260 GB/s, while the FP64 SpMV, the
// batched SpMV and the FP64 residuals ran 1-4 % slower and keep the
// XCD-contiguous order; the per-colour kernels are unaffected.  slab_perm
// maps a tile of the XCD-contiguous order to its tile in the slab order; over
// nb equal colour blocks of T/nb tiles each it is a permutation of [0, T)
// when T/nb is a multiple of 8, which the host checks (full_grid_order).
__device__ __forceinline__ i64 slab_perm(i64 t, i64 T, int nb = kXcds)
{
    const i64 per = T / nb, sub = per / kXcds, span = T / kXcds;  // span = nb * sub
    const i64 x = t / span, u = t % span;
    return (u / sub) * per + x * sub + u % sub;
}

// Plane-interleaved order of a full-grid launch (remap == kRemapPlanes).
// Work item v of the XCD-contiguous order is the v-th row of a sequence that
// runs over the lattice planes kk of the colour blocks and, within one kk,
// over the eight colours: the four on grid plane 2kk first, then the four on
// 2kk + 1.  XCD x then owns a slab of consecutive grid planes with every
// colour in it, and the rows it has in flight gather their neighbours from
// two or three adjacent grid planes, which stay in that XCD's L2: each
// vector entry comes from HBM about once per launch rather than once per
// XCD.  Needs equal colour blocks (all extents even) and N < 2^32, which
// the host checks.
__device__ __forceinline__ i64 plane_row(i64 v, const Geom &g)
{
    const unsigned P = (unsigned)g.bx[0] * (unsigned)g.by[0];
    const unsigned q = (unsigned)v / P, local = (unsigned)v - q * P;
    const unsigned c = (q & 7u) ^ 4u, kk = q >> 3;
    return g.off[c] + (i64)kk * P + local;
}

// Plane-interleaved order of a launch over two consecutive, equal colour
// blocks c0 and c0 + 1 starting at row0 (remap == kRemapPlanePair): work
// item v is the v-th row of a sequence that runs over the lattice planes kk
// and, within one kk, over colour c0 then c0 + 1.  The pairs this is used
// for, (0, 1) and (6, 7), differ in the x parity only, so both colours of
// one kk lie on the same grid plane and gather from the same three grid
// planes: XCD x owns a slab of planes and fetches those vector entries once
// for both colours, instead of once per colour when each colour block is a
// separate range.  Needs equal colour blocks and rows below 2^32, which the
// host checks.
__device__ __forceinline__ i64 plane_pair_row(i64 v, const Geom &g, i64 row0)
{
    const unsigned P = (unsigned)g.bx[0] * (unsigned)g.by[0];
    const unsigned q = (unsigned)v / P, local = (unsigned)v - q * P;
    const i64 B = g.off[1] - g.off[0];
    return row0 + (i64)(q & 1u) * B + (i64)(q >> 1) * P + local;
}

// Row loop of a grid-stride launch: the N rows are cut into 256-row tiles,
// XCD x owns tiles [T x / 8, T (x+1) / 8) and its workgroups stride through
// them.  Without remap: the plain grid-stride loop.
struct RowLoop {
    i64 tile, tile_end, tile_step, N;
    __device__ __forceinline__ bool next(i64 &p)
    {
        while (tile < tile_end) {
            p = tile * kBlock + threadIdx.x;
            tile += tile_step;
            if (p < N) return true;
        }
        return false;
    }
};
__device__ __forceinline__ RowLoop row_loop(i64 N, int remap)
{
    const i64 T = (N + kBlock - 1) / kBlock;
    const unsigned nb = gridDim.x, b = blockIdx.x;
    if (!remap || nb < kXcds) return RowLoop{(i64)b, T, (i64)nb, N};
    const unsigned x = b % kXcds, j = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    const unsigned cnt = q + (x < r ? 1 : 0);
    const i64 t0 = T * x / kXcds, t1 = T * (x + 1) / kXcds;
    return RowLoop{t0 + j, t1, (i64)cnt, N};
}

// Whether the launches of a matrix use the XCD-aware tile order.
inline int tile_remap(const Matrix &A) { return A.order != 0 ? 1 : 0; }
// Work order of a full-grid launch over all N rows of every colour with
// `lanes` lanes per row, in T tiles of 256 lanes: the matrix's order when it
// applies -- kRemapPlanes needs all grid extents even (equal colour blocks)
// and N < 2^32, kRemapSlab needs even extents and T a multiple of 64 (then
// slab_perm is a permutation) -- else the XCD-contiguous order (or none,
// when the matrix's order is 0).
int full_grid_order(const Matrix &A, int lanes);
// kRemapPlanes where it applies (even extents, N < 2^32), else 1.
int plane_order(const Matrix &A);

__device__ __forceinline__ i64 gtid() { return (i64)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ i64 gtid_xcd(int remap, int nb = kXcds)
{
    // the row permutation of these two is applied by the kernel (plane_row, plane_pair_row)
    if (remap == kRemapPlanes || remap == kRemapPlanePair) remap = 1;
    i64 t = xcd_tile(blockIdx.x, gridDim.x, remap);
    if (remap == kRemapSlab) t = slab_perm(t, gridDim.x, nb);
    return t * blockDim.x + threadIdx.x;
}

static inline unsigned grid_for(i64 n) { return (unsigned)((n + kBlock - 1) / kBlock); }

#define HPGMX_LAUNCH_CHECK()                                                    \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) throw std::runtime_error(hipGetErrorString(e_));  \
    } while (0)

// ---- deterministic block partial sums ----------------------------------------------
// Lane l of a launch holds NA accumulators acc[a]; lanes with equal l % L
// (L divides 64) belong together.  The workgroup's sum of acc[a] over the
// lanes of group g goes to partial column (a / R) * (L R) + g R + a % R, row
// blockIdx.x of partials (columns kMaxRedBlocks apart, contiguous for the
// finish kernel).  L = R = 1: column a holds the sum over all lanes.  The
// adds run in a fixed order (butterfly within a wavefront, then wavefronts
// in order), so results do not depend on timing.
template <int NA, int L, int R>
__device__ __forceinline__ void store_partials_g(const double (&acc)[NA], int na, double *partials)
{
    __shared__ double red[kBlock / 64][NA * L];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        if (a < na) {
            double v = acc[a];
#pragma unroll
            for (int o = 32; o >= L; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane < L) red[wave][a * L + lane] = v;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < na * L; t += kBlock) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][t];
        const int a = t / L, g = t % L;
        const int col = (a / R) * (L * R) + g * R + a % R;
        partials[(i64)col * kMaxRedBlocks + blockIdx.x] = s;
    }
}

// ---- several right-hand sides per row ----------------------------------------------
// A batch of K vectors is stored interleaved: entry j of row p at [p * K + j],
// so the K values a row needs from one neighbour are one contiguous run.  A
// lane handles R consecutive right-hand sides of one row (K / R lanes share
// the row); R is the tile shape the autotuner chooses.
template <typename T, int R> struct alignas(sizeof(T) * R) Pack {
    T v[R];
};
template <typename T, int R> __device__ __forceinline__ Pack<T, R> ldp(const T *p)
{
    return *reinterpret_cast<const Pack<T, R> *>(p);
}
template <typename T, int R> __device__ __forceinline__ void stp(T *p, const Pack<T, R> &v)
{
    *reinterpret_cast<Pack<T, R> *>(p) = v;
}
// As stp with a nontemporal store (results that a later kernel reads, see
// st_stream).
template <typename T, int R> __device__ __forceinline__ void stp_stream(T *p, const Pack<T, R> &v)
{
    if constexpr (R == 1) {
        __builtin_nontemporal_store(v.v[0], p);
    } else {
        typedef T vt __attribute__((ext_vector_type(R)));
        vt x;
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v.v[r];
        __builtin_nontemporal_store(x, reinterpret_cast<vt *>(p));
    }
}

// Gathered neighbour values in flight per lane: about 256 bytes, so that a
// wide lane (R = 8) stays within the register file.
template <typename T, int R> constexpr int gather_group()
{
    const int g = 256 / (R * (int)sizeof(T));
    return g >= kSlots ? kSlots : (g < 2 ? 2 : g);
}

// acc[r] = sum over the slots in MASK of a(p,s) * x[col(p,s) * K + r] (slot
// order, as ell_row_dot); x points at this lane's first right-hand side.
// The row's values and columns are loaded first, then the gathers go out in
// groups of gather_group() slots.
template <typename T, typename V, int K, int R, unsigned MASK>
__device__ __forceinline__ void ell_row_dot_b(const V *__restrict__ offv, const int *__restrict__ offc,
                                              const T *x, const EllRow &er, T (&acc)[R])
{
    V a[kSlots];
    int ci[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            const i64 e = er.base + (i64)s * er.stride;
            a[s] = ld_stream(offv + e);
            ci[s] = ld_stream(offc + e);
        }
    }
    sched_fence();
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = (T)0;
    constexpr int G = gather_group<T, R>();
#pragma unroll
    for (int s0 = 0; s0 < kSlots; s0 += G) {
        Pack<T, R> xv[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            if (s < kSlots && (MASK & (1u << s))) xv[u] = ldp<T, R>(x + (i64)ci[s] * K);
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            if (s < kSlots && (MASK & (1u << s))) {
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] = madd(to_t<T>(a[s]), xv[u].v[r], acc[r]);
            }
        }
    }
}

// As ell_row_dot_b over MASK, with accE[r] the sum over the slots of EMASK
// alone (equal to ell_row_dot_b over EMASK bit for bit).
template <typename T, typename V, int K, int R, unsigned MASK, unsigned EMASK>
__device__ __forceinline__ void ell_row_dot_b2(const V *__restrict__ offv, const int *__restrict__ offc,
                                               const T *x, const EllRow &er, T (&acc)[R], T (&accE)[R])
{
    V a[kSlots];
    int ci[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (MASK & (1u << s)) {
            const i64 e = er.base + (i64)s * er.stride;
            a[s] = ld_stream(offv + e);
            ci[s] = ld_stream(offc + e);
        }
    }
    sched_fence();
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = accE[r] = (T)0;
    constexpr int G = gather_group<T, R>();
#pragma unroll
    for (int s0 = 0; s0 < kSlots; s0 += G) {
        Pack<T, R> xv[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            if (s < kSlots && (MASK & (1u << s))) xv[u] = ldp<T, R>(x + (i64)ci[s] * K);
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            if (s < kSlots && (MASK & (1u << s))) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[r] = madd(to_t<T>(a[s]), xv[u].v[r], acc[r]);
                    if (EMASK & (1u << s)) accE[r] = madd(to_t<T>(a[s]), xv[u].v[r], accE[r]);
                }
            }
        }
    }
}

}  // namespace hpgmx
