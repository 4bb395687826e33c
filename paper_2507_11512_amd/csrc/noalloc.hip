// The adjoint stencil correlation without device allocation
// (hpgmx_stencil_grad_noalloc), for callers that cannot allocate device
// memory: code under stream capture, serving loops, harnesses that forbid
// hipMalloc.
//
// Its only scratch memory is the per-workgroup partial sums of the 27
// correlations, kept in a file-scope device array of fixed size (`scratch`,
// kNoAllocBlocks x 27 doubles = 216 KiB).  Every GPU the library runs on
// holds its own copy of the array until the process ends; the host never
// uses the array's name as an address (in host code it is only a stand-in):
// when the first handle on a device is created, with that device current,
// hipGetSymbolAddress gives the device address of that device's copy, and
// only that address is passed to kernels.  All calls on one GPU share the
// array, so two calls that overlap on one GPU (different streams, or host
// threads) race; calls on one stream are ordered and safe.  The array needs
// no clearing: each call writes every partial sum it reads.
#include "ell_device.hpp"

#include <mutex>
#include <stdexcept>

namespace hpgmx {

constexpr int kNoAllocBlocks = kMaxRedBlocks;  // workgroups of the reduction
constexpr int kNoAllocSums = 27;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocBlocks * kNoAllocSums];

namespace {
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};
}  // namespace

// Looks up this device's copy of `scratch` once (the device must be current).
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = (double *)ptr;
    return hipSuccess;
}

size_t noalloc_scratch_bytes() { return sizeof(double) * kNoAllocBlocks * kNoAllocSums; }

// acc[t] = sum over grid points I of lam_I * x_{I + d_t} (neighbour inside
// the grid), in the natural order I = i + nx (j + ny k): the same sums as
// k_stencil_corr, without permuting lam and x to the colour-blocked order
// (which would need two staging vectors).
__global__ __launch_bounds__(kBlock) void k_stencil_corr_nat(int nx, int ny, int nz, const double *__restrict__ lam,
                                                             const double *__restrict__ x, double *partials)
{
    double acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.0;
    const i64 N = (i64)nx * ny * nz, plane = (i64)nx * ny;
    const i64 stride = (i64)gridDim.x * kBlock;
    for (i64 I = (i64)blockIdx.x * kBlock + threadIdx.x; I < N; I += stride) {
        const int i = (int)(I % nx), j = (int)((I / nx) % ny), k = (int)(I / plane);
        const double l = lam[I];
        double xv[27];
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int di = t % 3 - 1, dj = (t / 3) % 3 - 1, dk = t / 9 - 1;
            const bool in = i + di >= 0 && i + di < nx && j + dj >= 0 && j + dj < ny && k + dk >= 0 && k + dk < nz;
            xv[t] = in ? x[I + di + (i64)nx * dj + plane * dk] : 0.0;
        }
        sched_fence();
#pragma unroll
        for (int t = 0; t < 27; ++t) acc[t] += l * xv[t];
    }
    store_partials_g<27, 1, 1>(acc, 27, partials);
}

// out[t] = sum of the nb partial sums of correlation t, in workgroup order.
__global__ __launch_bounds__(64) void k_corr_sum(const double *__restrict__ partials, int nb, double *out)
{
    const int t = threadIdx.x;
    if (t >= kNoAllocSums) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partials[(i64)t * kMaxRedBlocks + b];
    out[t] = s;
}

void launch_stencil_correlation_noalloc(int device, const Geom &g, const double *lam, const double *x, double *out27,
                                        hipStream_t s)
{
    double *part = (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
    if (!part) throw std::runtime_error("device scratch of the no-allocation gradient is not set up");
    const int nb = red_blocks(g.N);
    hipLaunchKernelGGL(k_stencil_corr_nat, dim3(nb), dim3(kBlock), 0, s, g.nx, g.ny, g.nz, lam, x, part);
    HPGMX_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_corr_sum, dim3(1), dim3(64), 0, s, (const double *)part, nb, out27);
    HPGMX_LAUNCH_CHECK();
}

}  // namespace hpgmx
