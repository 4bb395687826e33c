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

template <typename T, typename V> __device__ __forceinline__ T to_t(V v) { return (T)v; }
template <> __device__ __forceinline__ float to_t<float, __half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float to_t<float, bf16>(bf16 v) { return __bfloat162float(v); }

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// sum over the slots in MASK of a(p,s) * x[col(p,s)] (slot order).
template <typename T, typename V, unsigned MASK>
__device__ __forceinline__ T ell_row_dot(const V *__restrict__ offv, const int *__restrict__ offc,
                                         const T *x, const EllRow &er)
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
    T xv[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (MASK & (1u << s)) xv[s] = x[ci[s]];
    sched_fence();
    T acc = (T)0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (MASK & (1u << s)) acc += to_t<T>(a[s]) * xv[s];
    return acc;
}

constexpr unsigned kAllSlots = (1u << kSlots) - 1u;

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

// Remapping switch (HPGMX_XCD_REMAP=0 turns it off for layout studies).
int xcd_remap_enabled();

}  // namespace hpgmx
