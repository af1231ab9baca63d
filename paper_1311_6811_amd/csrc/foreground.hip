// Learned foreground colour model for frames after the first (Eq. 1-2 use a
// uniform foreground density, as nothing is known of the foreground's colours
// at the first frame, Sec. 2.2.2). Three launches:
//   fg_zero_kernel     bin counts to 0
//   fg_hist_kernel     per workgroup an LDS histogram of the foreground pixels
//                      (mask != 0, or log(2*SLM) > 0 of the previous frame)
//                      of one view, added to the global counts with integer
//                      atomics (order-independent)
//   fg_density_kernel  log density of one colour value per bin, Laplace-
//                      smoothed: log((c + 1) / ((N + 4096) * 4096)), in FP64
#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr int kBins = PSFS_FG_BINS;
constexpr int kPixPerBlock = 4096;                  // 16 per lane

__global__ __launch_bounds__(256) void fg_zero_kernel(uint32_t *counts)
{
    for (int b = static_cast<int>(threadIdx.x); b < kBins; b += 256) counts[b] = 0u;
}

// grid (ceil(max_npix / kPixPerBlock), views)
__global__ __launch_bounds__(256) void fg_hist_kernel(FgArgs a)
{
    __shared__ uint32_t h[kBins];
    for (int b = static_cast<int>(threadIdx.x); b < kBins; b += 256) h[b] = 0u;
    __syncthreads();
    const SlmView &sv = a.view[blockIdx.y];
    const uint8_t *mask = a.mask[blockIdx.y];
    const float *map = a.lmap ? a.lmap + sv.map_off : nullptr;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPixPerBlock + threadIdx.x;
#pragma unroll 4
    for (int r = 0; r < kPixPerBlock / 256; ++r) {
        const int64_t p = base + 256 * r;
        if (p >= sv.npix) break;
        const bool fg = mask ? mask[p] != 0 : map[p] > 0.0f;
        if (fg) {
            const uint8_t *I = sv.img + 3 * p;
            atomicAdd(&h[colour_bin(I[0], I[1], I[2])], 1u);
        }
    }
    __syncthreads();
    for (int b = static_cast<int>(threadIdx.x); b < kBins; b += 256)
        if (h[b]) atomicAdd(a.counts + b, h[b]);
}

__global__ __launch_bounds__(256) void fg_density_kernel(FgArgs a)
{
    __shared__ unsigned long long red[256];
    unsigned long long s = 0;
    for (int b = static_cast<int>(threadIdx.x); b < kBins; b += 256) s += a.counts[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double denom = (static_cast<double>(red[0]) + kBins) * kBins;
    for (int b = static_cast<int>(threadIdx.x); b < kBins; b += 256)
        a.logd[b] = static_cast<float>(log((static_cast<double>(a.counts[b]) + 1.0) / denom));
}

}  // namespace

hipError_t launch_foreground(const FgArgs &a, int64_t max_npix, hipStream_t s)
{
    hipLaunchKernelGGL(fg_zero_kernel, dim3(1), dim3(256), 0, s, a.counts);
    if (a.n > 0 && max_npix > 0) {
        const dim3 g(static_cast<unsigned>((max_npix + kPixPerBlock - 1) / kPixPerBlock), static_cast<unsigned>(a.n));
        hipLaunchKernelGGL(fg_hist_kernel, g, dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(fg_density_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace psfs
