// Voxel colouring (Sec. 3.1.1; the voxel projection and colour step of
// Sec. 3.3.3): the colour of every listed voxel (normally the surface list)
// from the views that see it. Three launches:
//   colour_clear_kernel   per (voxel, view): the depth-buffer entry of the
//                         voxel's pixel to "empty"
//   depth_kernel          per (voxel, view): project as the fusion does and
//                         keep the nearest voxel of every pixel with a 64-bit
//                         atomic minimum of (depth bits << 32 | list position)
//   colour_gather_kernel  per voxel, one lane per view: a view whose pixel the
//                         voxel holds contributes the pixel's RGB; the integer
//                         sums over the views are reduced across the lanes and
//                         the mean (0 if unseen) and the view count written
// Depths are positive FP32, whose bit patterns order like the values, so the
// minimum key is the nearest voxel and, on equal depth, the earlier one in the
// list. The sums are integers, so the result does not depend on the order in
// which they are added.
#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr unsigned long long kEmpty = ~0ull;

// Pixel offset (within the view's buffer) and depth of list entry q in view g,
// or false when the view does not see it. Same FP32 arithmetic as the
// fusion's checked path, so both pick the same pixel.
__device__ __forceinline__ bool locate(const ColourArgs &a, const ViewGeom &g, int64_t vox, uint32_t &pix,
                                       float &depth)
{
    if (vox < 0 || vox >= a.nvox) return false;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    const int k = static_cast<int>(vox / plane);
    const int64_t rem = vox - static_cast<int64_t>(k) * plane;
    const int j = static_cast<int>(rem / a.nx), i = static_cast<int>(rem - static_cast<int64_t>(j) * a.nx);
    const float X = a.ox + a.h * (static_cast<float>(i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(j) + 0.5f);
    const float Z = a.oz + a.h * (static_cast<float>(k) + 0.5f);
    const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
    const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
    const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
    const float c = fmaf(g.P[10], Z, cx);
    const float r = __builtin_amdgcn_rcpf(c);
    const int x = static_cast<int>(floorf(fmaf(g.P[2], Z, ax) * r));
    const int y = static_cast<int>(floorf(fmaf(g.P[6], Z, bx) * r));
    if (!(c > 0.0f) || static_cast<uint32_t>(x) >= static_cast<uint32_t>(g.W) ||
        static_cast<uint32_t>(y) >= static_cast<uint32_t>(g.H))
        return false;
    pix = static_cast<uint32_t>(y) * static_cast<uint32_t>(g.W) + static_cast<uint32_t>(x);
    depth = c;
    return true;
}

// grid (ceil(nlist / 256), views): the depth-buffer entries the list can
// reach to "empty" (only those are read later)
__global__ __launch_bounds__(256) void colour_clear_kernel(ColourArgs a)
{
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= a.nlist) return;
    const ViewGeom &g = a.view[blockIdx.y];
    uint32_t pix;
    float depth;
    if (locate(a, g, a.list[q], pix, depth)) a.zbuf[g.map_off + pix] = kEmpty;
}

// grid (ceil(nlist / 256), views)
__global__ __launch_bounds__(256) void depth_kernel(ColourArgs a)
{
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= a.nlist) return;
    const ViewGeom &g = a.view[blockIdx.y];
    uint32_t pix;
    float depth;
    if (!locate(a, g, a.list[q], pix, depth)) return;
    const unsigned long long key =
        (static_cast<unsigned long long>(__float_as_uint(depth)) << 32) | static_cast<unsigned long long>(q);
    atomicMin(a.zbuf + g.map_off + pix, key);
}

// grid (ceil(nlist / kGatherVoxels)), block 256: lane group of 16 = one
// voxel, lane l of the group = view l (idle for l >= n). The sums over the
// group are integer butterflies within aligned 16-lane groups of the wave.
constexpr int kGatherLanes = 16;                    // one lane per possible view
constexpr int kGatherVoxels = 256 / kGatherLanes;   // voxels per workgroup
static_assert(kGatherLanes >= kMaxViews, "a lane for every view");

__global__ __launch_bounds__(256) void colour_gather_kernel(ColourArgs a)
{
    const int v = static_cast<int>(threadIdx.x) % kGatherLanes;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kGatherVoxels + static_cast<int>(threadIdx.x) / kGatherLanes;
    uint32_t r = 0, gr = 0, b = 0, seen = 0;
    if (q < a.nlist && v < a.n) {
        const ViewGeom &g = a.view[v];
        uint32_t pix;
        float depth;
        if (locate(a, g, a.list[q], pix, depth)) {
            const unsigned long long key =
                (static_cast<unsigned long long>(__float_as_uint(depth)) << 32) | static_cast<unsigned long long>(q);
            if (a.zbuf[g.map_off + pix] == key) {
                const uint8_t *p = a.img[v] + 3 * static_cast<int64_t>(pix);
                r = p[0];
                gr = p[1];
                b = p[2];
                seen = 1;
            }
        }
    }
#pragma unroll
    for (int d = kGatherLanes / 2; d >= 1; d >>= 1) {
        r += __shfl_xor(r, d, 64);
        gr += __shfl_xor(gr, d, 64);
        b += __shfl_xor(b, d, 64);
        seen += __shfl_xor(seen, d, 64);
    }
    if (v == 0 && q < a.nlist) {
        const float n = static_cast<float>(seen);
        a.colour[3 * q] = seen > 0 ? static_cast<float>(r) / n : 0.0f;
        a.colour[3 * q + 1] = seen > 0 ? static_cast<float>(gr) / n : 0.0f;
        a.colour[3 * q + 2] = seen > 0 ? static_cast<float>(b) / n : 0.0f;
        a.views[q] = static_cast<int32_t>(seen);
    }
}

}  // namespace

hipError_t launch_colour(const ColourArgs &a, hipStream_t s)
{
    if (a.nlist <= 0) return hipSuccess;
    const unsigned qb = static_cast<unsigned>((a.nlist + 255) / 256);
    if (a.n > 0) {
        hipLaunchKernelGGL(colour_clear_kernel, dim3(qb, static_cast<unsigned>(a.n)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(depth_kernel, dim3(qb, static_cast<unsigned>(a.n)), dim3(256), 0, s, a);
    }
    const unsigned gb = static_cast<unsigned>((a.nlist + kGatherVoxels - 1) / kGatherVoxels);
    hipLaunchKernelGGL(colour_gather_kernel, dim3(gb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace psfs
