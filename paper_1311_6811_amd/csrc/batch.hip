// Batched occupancy pass over many frames of uneven shape (grid size, view
// count, image size), as two persistent launches that pull work items from
// device counters:
//   batch_slm_kernel   items = 1024-pixel chunks of every view of every frame
//                      (Eq. 1-2 into one likelihood-map arena)
//   batch_fuse_kernel  items = voxel bricks of every frame (Eq. 3-9 + threshold),
//                      frames in decreasing cost order (longest first)
// A workgroup pops kGroup consecutive items per atomic, finds the owning
// view/frame by binary search in the device descriptor table, and runs the
// same per-pixel and per-column code as the single-frame kernels, so a batched
// frame is bit-identical to the same frame reconstructed alone. Every
// workgroup leaves its loop when the counter passes the item count.
#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr int kChunkPixels = 1024;      // 256 lanes x 4 pixels
constexpr int kGroup = 4;               // items popped per atomic

__device__ __forceinline__ int find_view(const BatchView *views, int nviews, int64_t chunk)
{
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].chunk0 <= chunk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_frame(const BatchFrame *frames, int nframes, int64_t brick)
{
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (frames[mid].brick0 <= brick) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pops the next kGroup items for the whole workgroup (uniform result).
__device__ __forceinline__ int64_t pop(unsigned long long *counter)
{
    __shared__ unsigned long long item;
    if (threadIdx.x == 0) item = atomicAdd(counter, static_cast<unsigned long long>(kGroup));
    __syncthreads();
    const int64_t r = static_cast<int64_t>(item);
    __syncthreads();
    return r;
}

__device__ __forceinline__ void slm_quad(const BatchView &bv, float *lmap, float k0, int64_t p0)
{
    if (p0 >= bv.npix) return;
    float *out = lmap + bv.g.map_off + p0;
    if (p0 + 4 <= bv.npix) {
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(bv.img + 3 * p0);
        const uint32_t w0 = __builtin_nontemporal_load(iw + 0);
        const uint32_t w1 = __builtin_nontemporal_load(iw + 1);
        const uint32_t w2 = __builtin_nontemporal_load(iw + 2);
        const f32x4 *mp = reinterpret_cast<const f32x4 *>(bv.mean + 3 * p0);
        const f32x4 *vp = reinterpret_cast<const f32x4 *>(bv.var + 3 * p0);
        const f32x4 m0 = __builtin_nontemporal_load(mp + 0);
        const f32x4 m1 = __builtin_nontemporal_load(mp + 1);
        const f32x4 m2 = __builtin_nontemporal_load(mp + 2);
        const f32x4 v0 = __builtin_nontemporal_load(vp + 0);
        const f32x4 v1 = __builtin_nontemporal_load(vp + 1);
        const f32x4 v2 = __builtin_nontemporal_load(vp + 2);
        f32x4 r;
        r.x = log2slm(byte_of(w0, 0), byte_of(w0, 1), byte_of(w0, 2), m0.x, m0.y, m0.z, v0.x, v0.y, v0.z, k0);
        r.y = log2slm(byte_of(w0, 3), byte_of(w1, 0), byte_of(w1, 1), m0.w, m1.x, m1.y, v0.w, v1.x, v1.y, k0);
        r.z = log2slm(byte_of(w1, 2), byte_of(w1, 3), byte_of(w2, 0), m1.z, m1.w, m2.x, v1.z, v1.w, v2.x, k0);
        r.w = log2slm(byte_of(w2, 1), byte_of(w2, 2), byte_of(w2, 3), m2.y, m2.z, m2.w, v2.y, v2.z, v2.w, k0);
        *reinterpret_cast<f32x4 *>(out) = r;
    } else {
        for (int64_t p = p0; p < bv.npix; ++p) {
            const uint8_t *I = bv.img + 3 * p;
            const float *m = bv.mean + 3 * p, *v = bv.var + 3 * p;
            out[p - p0] = log2slm(I[0], I[1], I[2], m[0], m[1], m[2], v[0], v[1], v[2], k0);
        }
    }
}

__global__ __launch_bounds__(256) void batch_slm_kernel(BatchArgs a)
{
    for (;;) {
        const int64_t c0 = pop(a.counters + 0);
        if (c0 >= a.nchunks) break;
        const int64_t c1 = c0 + kGroup < a.nchunks ? c0 + kGroup : a.nchunks;
        for (int64_t c = c0; c < c1; ++c) {
            const int v = __builtin_amdgcn_readfirstlane(find_view(a.views, a.nviews, c));
            const BatchView &bv = a.views[v];
            slm_quad(bv, a.lmap, a.k0, (c - bv.chunk0) * kChunkPixels + static_cast<int64_t>(threadIdx.x) * 4);
        }
    }
}

template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void batch_fuse_kernel(BatchArgs a)
{
    for (;;) {
        const int64_t b0 = pop(a.counters + 1);
        if (b0 >= a.nbricks) break;
        const int64_t b1 = b0 + kGroup < a.nbricks ? b0 + kGroup : a.nbricks;
        for (int64_t b = b0; b < b1; ++b) {
            const int f = __builtin_amdgcn_readfirstlane(find_frame(a.frames, a.nframes, b));
            const BatchFrame &fr = a.frames[f];
            const int64_t lb = b - fr.brick0;
            const int ntx = (fr.grid.nx + TX - 1) / TX, nty = (fr.grid.ny + TY - 1) / TY;
            const int64_t ntile = static_cast<int64_t>(ntx) * nty;
            const int64_t zc = lb / ntile;
            const int t = static_cast<int>(lb - zc * ntile);
            const int tyi = t / ntx, txi = t - tyi * ntx;
            const int i = txi * TX + static_cast<int>(threadIdx.x % TX);
            const int j = tyi * TY + static_cast<int>(threadIdx.x / TX);
            const BatchView *views = a.views + fr.view0;
            fuse_column<TX, KZ, SAMPLING>([&](int v) -> const ViewGeom & { return views[v].g; }, fr.n, a.lmap, fr.grid,
                                      i, j, static_cast<int>(zc) * KZ, a.L0, a.tau, fr.post, fr.occ);
        }
    }
}

__global__ void batch_reset_kernel(unsigned long long *counters)
{
    if (threadIdx.x < 2) counters[threadIdx.x] = 0ull;
}

template <int S>
hipError_t launch_batch_fuse_s(const BatchArgs &a, int tile, int grid, hipStream_t s)
{
    const TileCfg &c = tile_cfg(tile);
    const dim3 g(static_cast<unsigned>(grid)), b(c.tx * c.ty);
    switch (tile) {
    case 0: hipLaunchKernelGGL((batch_fuse_kernel<8, 32, 4, S>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((batch_fuse_kernel<8, 32, 8, S>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_fuse_kernel<8, 16, 4, S>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((batch_fuse_kernel<8, 32, 2, S>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((batch_fuse_kernel<32, 8, 4, S>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((batch_fuse_kernel<16, 16, 4, S>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int64_t batch_chunk_pixels() { return kChunkPixels; }

int64_t batch_bricks(int nx, int ny, int nz, int tile)
{
    const TileCfg &c = tile_cfg(tile);
    return static_cast<int64_t>((nx + c.tx - 1) / c.tx) * ((ny + c.ty - 1) / c.ty) * ((nz + c.kz - 1) / c.kz);
}

namespace {
template <int S>
int occupancy_s(int tile)
{
    const TileCfg &c = tile_cfg(tile);
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    const int bs = c.tx * c.ty;
    switch (tile) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<8, 32, 4, S>, bs, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<8, 32, 8, S>, bs, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<8, 16, 4, S>, bs, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<8, 32, 2, S>, bs, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<32, 8, 4, S>, bs, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_fuse_kernel<16, 16, 4, S>, bs, 0); break;
    default: break;
    }
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}
}  // namespace

int batch_fuse_occupancy(int tile, int sampling)
{
    return sampling == PSFS_BILINEAR ? occupancy_s<PSFS_BILINEAR>(tile) : occupancy_s<PSFS_NEAREST>(tile);
}

hipError_t launch_batch(const BatchArgs &a, int tile, int sampling, int slm_grid, int fuse_grid, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, a.counters);
    if (a.nchunks > 0) hipLaunchKernelGGL(batch_slm_kernel, dim3(static_cast<unsigned>(slm_grid)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nbricks == 0) return hipSuccess;
    return sampling == PSFS_BILINEAR ? launch_batch_fuse_s<PSFS_BILINEAR>(a, tile, fuse_grid, s)
                                     : launch_batch_fuse_s<PSFS_NEAREST>(a, tile, fuse_grid, s);
}

}  // namespace psfs
