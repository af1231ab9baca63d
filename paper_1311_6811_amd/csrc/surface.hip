// The step after the posterior (Sec. 2.2.2, last paragraph; Sec. 3.3.3 steps
// d and e): smoothing of the occupancy probabilities, thresholding, and removal
// of the voxels inside the body, leaving the surface voxels as a compact list.
//   smooth_surface_kernel  3x3x3 mean over the in-grid neighbours, threshold
//                          and surface flag in one traversal (the paper
//                          merges smoothing with voxel generation to save a
//                          round trip through memory); a surface voxel is
//                          occupied with an unoccupied or out-of-grid face
//                          neighbour
//   surface_count          per block of kSurfBlock consecutive voxels, the
//                          number of surface flags
//   surface_write          the flagged voxels' linear indices at their place
//                          in the ascending list (block offset = sum of the
//                          earlier blocks' counts)
// The paper keeps inner-voxel removal on the CPU; here it is a deterministic
// two-kernel stream compaction over a flag grid.
#include "psfs_internal.h"

namespace psfs {
namespace {

constexpr int kBX = 32, kBY = 8, kBZ = 4;          // tile of output voxels
constexpr int kSurfBlock = 4096;                    // voxels per compaction block (16 per lane)

// Smoothing, threshold and the surface test in one pass over a tile of
// kBX x kBY x kBZ output voxels. The surface test needs the occupancy of the
// face neighbours, hence the smoothed value one voxel beyond the tile, hence
// the posterior two voxels beyond it. The 3x3x3 sum is separable and taken in
// one fixed order (x, then y, then z), so a voxel's smoothed value has the
// same bits whether it is a tile's output or another tile's halo. Cells
// outside the grid hold posterior 0 and occupancy 0, so "a face neighbour
// with occupancy 0" covers both an unoccupied and an out-of-grid neighbour.
constexpr int kPX = kBX + 4, kPY = kBY + 4, kPZ = kBZ + 4;   // posterior, halo 2
constexpr int kSX = kBX + 2, kSY = kBY + 2, kSZ = kBZ + 2;   // smoothed, halo 1

__global__ __launch_bounds__(256) void smooth_surface_kernel(SurfArgs a)
{
    __shared__ float P[kPZ][kPY][kPX];
    __shared__ float SX[kPZ][kPY][kSX];             // sums over x
    __shared__ float SXY[kPZ][kSY][kSX];            // sums over x and y
    __shared__ uint8_t OCC[kSZ][kSY][kSX];
    const int nbx = (a.nx + kBX - 1) / kBX, nby = (a.ny + kBY - 1) / kBY;
    const int b = static_cast<int>(blockIdx.x);
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ox = bx * kBX, oy = by * kBY, oz = bz * kBZ;          // first output voxel
    const int tid = static_cast<int>(threadIdx.x);
    // all loads of the halo block first, then the LDS stores (one wait)
    constexpr int kPN = kPX * kPY * kPZ, kPIter = (kPN + 255) / 256;
    float pv[kPIter];
#pragma unroll
    for (int r = 0; r < kPIter; ++r) {
        const int e = tid + 256 * r;
        const int hx = e % kPX, hy = (e / kPX) % kPY, hz = e / (kPX * kPY);
        const int gx = ox - 2 + hx, gy = oy - 2 + hy, gz = oz - 2 + hz;
        const bool in = e < kPN && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz;
        pv[r] = in ? a.post[(static_cast<int64_t>(gz) * a.ny + gy) * a.nx + gx] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kPIter; ++r) {
        const int e = tid + 256 * r;
        if (e < kPN) (&P[0][0][0])[e] = pv[r];
    }
    __syncthreads();
    // separable sums, each pass a fixed number of unrolled rounds so that a
    // thread's LDS reads of all its elements are in flight together
    constexpr int kN1 = kSX * kPY * kPZ, kN2 = kSX * kSY * kPZ, kN3 = kSX * kSY * kSZ;
#pragma unroll
    for (int r = 0; r < (kN1 + 255) / 256; ++r) {
        const int e = tid + 256 * r;
        if (e < kN1) {
            const int sx = e % kSX, hy = (e / kSX) % kPY, hz = e / (kSX * kPY);
            SX[hz][hy][sx] = (P[hz][hy][sx] + P[hz][hy][sx + 1]) + P[hz][hy][sx + 2];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (kN2 + 255) / 256; ++r) {
        const int e = tid + 256 * r;
        if (e < kN2) {
            const int sx = e % kSX, sy = (e / kSX) % kSY, hz = e / (kSX * kSY);
            SXY[hz][sy][sx] = (SX[hz][sy][sx] + SX[hz][sy + 1][sx]) + SX[hz][sy + 2][sx];
        }
    }
    __syncthreads();
    // smoothed value and occupancy of the tile plus one voxel around it; the
    // smoothed values go where the posterior was (no longer read)
    float(*M)[kSY][kSX] = reinterpret_cast<float(*)[kSY][kSX]>(&P[0][0][0]);
    static_assert(kN3 <= kPX * kPY * kPZ, "smoothed block fits the posterior block");
#pragma unroll
    for (int r = 0; r < (kN3 + 255) / 256; ++r) {
        const int e = tid + 256 * r;
        if (e < kN3) {
            const int sx = e % kSX, sy = (e / kSX) % kSY, sz = e / (kSX * kSY);
            const int gx = ox - 1 + sx, gy = oy - 1 + sy, gz = oz - 1 + sz;
            uint8_t o = 0;
            if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz) {
                const int c = ((gx > 0) + 1 + (gx + 1 < a.nx)) * ((gy > 0) + 1 + (gy + 1 < a.ny)) *
                              ((gz > 0) + 1 + (gz + 1 < a.nz));
                const float m =
                    ((SXY[sz][sy][sx] + SXY[sz + 1][sy][sx]) + SXY[sz + 2][sy][sx]) / static_cast<float>(c);
                o = m > a.tau ? 1 : 0;
                M[sz][sy][sx] = m;
            }
            OCC[sz][sy][sx] = o;
        }
    }
    __syncthreads();
    const int lx = tid % kBX, ly = tid / kBX;
    const int gx = ox + lx, gy = oy + ly;
    if (gx >= a.nx || gy >= a.ny) return;
#pragma unroll
    for (int z = 0; z < kBZ; ++z) {
        const int gz = oz + z;
        if (gz >= a.nz) break;
        const int64_t idx = (static_cast<int64_t>(gz) * a.ny + gy) * a.nx + gx;
        const int sx = lx + 1, sy = ly + 1, sz = z + 1;
        const uint8_t o = OCC[sz][sy][sx];
        const bool surf = o && !(OCC[sz][sy][sx - 1] && OCC[sz][sy][sx + 1] && OCC[sz][sy - 1][sx] &&
                                 OCC[sz][sy + 1][sx] && OCC[sz - 1][sy][sx] && OCC[sz + 1][sy][sx]);
        if (a.smoothed) a.smoothed[idx] = M[sz][sy][sx];
        a.occ[idx] = o;
        a.flags[idx] = surf ? 1 : 0;
    }
}

// Lane l of a compaction block owns its 16 consecutive voxels
// base + 16 l .. base + 16 l + 15 (one 16-byte load of flags).
__device__ __forceinline__ uint32_t lane_flags(const SurfArgs &a, int64_t base)
{
    const int64_t v = base + 16 * static_cast<int64_t>(threadIdx.x);
    uint32_t bits = 0;
    if (v + 16 <= a.nvox) {
        const uint4 w = *reinterpret_cast<const uint4 *>(a.flags + v);
        const uint32_t word[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if ((word[q >> 2] >> (8 * (q & 3))) & 0xffu) bits |= 1u << q;
    } else {
        for (int q = 0; q < 16 && v + q < a.nvox; ++q)
            if (a.flags[v + q]) bits |= 1u << q;
    }
    return bits;
}

// Inclusive sum over the block's 256 lanes in lane order (wave scans + the
// totals of the waves before).
__device__ __forceinline__ int block_inclusive_scan(int x, int *wave_tot)
{
    const int lane = static_cast<int>(threadIdx.x & 63), w = static_cast<int>(threadIdx.x >> 6);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wave_tot[w] = x;
    __syncthreads();
    for (int q = 0; q < w; ++q) x += wave_tot[q];
    return x;
}

__global__ __launch_bounds__(256) void surface_count_kernel(SurfArgs a)
{
    __shared__ int wave_tot[4];
    const int c = __popc(lane_flags(a, static_cast<int64_t>(blockIdx.x) * kSurfBlock));
    const int incl = block_inclusive_scan(c, wave_tot);
    if (threadIdx.x == 255) a.counts[blockIdx.x] = incl;
}

__global__ __launch_bounds__(256) void surface_write_kernel(SurfArgs a)
{
    __shared__ int64_t red[256];
    __shared__ int wave_tot[4];
    const int b = static_cast<int>(blockIdx.x);
    // exclusive prefix of the block counts (and, in block 0, the total)
    int64_t s = 0, tot = 0;
    for (int q = static_cast<int>(threadIdx.x); q < a.nblocks; q += 256) {
        if (q < b) s += a.counts[q];
        tot += a.counts[q];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const int64_t block_off = red[0];
    __syncthreads();
    if (b == 0) {
        red[threadIdx.x] = tot;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.count = red[0];
    }
    const int64_t base = static_cast<int64_t>(b) * kSurfBlock;
    uint32_t bits = lane_flags(a, base);
    const int c = __popc(bits);
    int64_t pos = block_off + (block_inclusive_scan(c, wave_tot) - c);
    const int64_t v0 = base + 16 * static_cast<int64_t>(threadIdx.x);
    while (bits) {
        const int q = __ffs(bits) - 1;
        bits &= bits - 1;
        if (pos < a.capacity) a.out[pos] = static_cast<int32_t>(v0 + q);
        ++pos;
    }
}

__global__ void zero_count_kernel(int64_t *count)
{
    if (threadIdx.x == 0) *count = 0;
}

}  // namespace

int64_t surface_blocks(int64_t nvox) { return (nvox + kSurfBlock - 1) / kSurfBlock; }

hipError_t launch_surface(const SurfArgs &a, hipStream_t s)
{
    if (a.nvox == 0) {
        hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, a.count);
        return hipGetLastError();
    }
    const int64_t tiles = static_cast<int64_t>((a.nx + kBX - 1) / kBX) * ((a.ny + kBY - 1) / kBY) *
                          ((a.nz + kBZ - 1) / kBZ);
    hipLaunchKernelGGL(smooth_surface_kernel, dim3(static_cast<unsigned>(tiles)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(surface_count_kernel, dim3(static_cast<unsigned>(a.nblocks)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(surface_write_kernel, dim3(static_cast<unsigned>(a.nblocks)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace psfs
