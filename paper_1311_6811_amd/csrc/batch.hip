// Batched occupancy pass over many frames of uneven shape (grid size, view
// count, image size), as two persistent launches:
//   batch_slm_kernel   items = 1024-pixel chunks of every view of every frame
//                      (Eq. 1-2 into one likelihood-map arena)
//   batch_fuse_kernel  items = voxel bricks of every frame (Eq. 3-9 +
//                      threshold), frames in decreasing cost order (longest
//                      first)
// Workgroups pop kGroup consecutive items per atomic from device counters.
// The bricks are cut into one contiguous slice per XCD; the workgroups of an
// XCD pop their own slice first (a band of z-slabs of the same frames, so the
// XCD's L2 holds the matching band of map rows), then help with the other
// slices. A workgroup finds the owning view/frame of an item by binary search
// in the device descriptor table and runs the same per-pixel and per-column
// code as the single-frame kernels, so a batched frame is bit-identical to the
// same frame reconstructed alone. Every workgroup leaves when the counters it
// pops from have passed their ends.
#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr int kChunkPixels = 4 * kWavePixels;   // one per wave of a workgroup
constexpr int kGroup = 4;               // items popped per atomic
constexpr int kChunkCounter = 0;        // counters[0]: likelihood chunks popped
constexpr int kBrickCounter0 = 1;       // counters[1 + x]: bricks popped from slice x
constexpr int kCounters = kBrickCounter0 + kNumXcd;

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

__global__ __launch_bounds__(256) void batch_slm_kernel(BatchArgs a)
{
    __shared__ SlmStage stage[4];
    const int wave = static_cast<int>(threadIdx.x >> 6);
    for (;;) {
        const int64_t c0 = pop(a.counters + kChunkCounter);
        if (c0 >= a.nchunks) break;
        const int64_t c1 = c0 + kGroup < a.nchunks ? c0 + kGroup : a.nchunks;
        for (int64_t c = c0; c < c1; ++c) {
            const int v = __builtin_amdgcn_readfirstlane(find_view(a.views, a.nviews, c));
            const BatchView &bv = a.views[v];
            const int64_t p0 = (c - bv.chunk0) * kChunkPixels + wave * kWavePixels;
            float *out = a.lmap + bv.g.map_off;
            if (p0 + kWavePixels <= bv.npix)
                slm_wave(bv.img, bv.mean, bv.var, out, p0, a.k0, stage[wave], nullptr);
            else if (p0 < bv.npix)
                slm_wave_tail(bv.img, bv.mean, bv.var, out, p0, bv.npix, a.k0, nullptr);
        }
    }
}

template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void batch_fuse_kernel(BatchArgs a)
{
    // workgroups are dispatched to the XCDs in turn
    const int home = static_cast<int>(blockIdx.x % kNumXcd);
    for (int q = 0; q < kNumXcd; ++q) {
        const int slice = (home + q) % kNumXcd;
        const int64_t lo = a.nbricks * slice / kNumXcd, hi = a.nbricks * (slice + 1) / kNumXcd;
        for (;;) {
            const int64_t b0 = lo + pop(a.counters + kBrickCounter0 + slice);
            if (b0 >= hi) break;
            const int64_t b1 = b0 + kGroup < hi ? b0 + kGroup : hi;
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
                fuse_column<TX, KZ, SAMPLING>([&](int v) -> const ViewGeom & { return views[v].g; }, fr.n, a.lmap,
                                              fr.grid, i, j, static_cast<int>(zc) * KZ, a.L0, a.tau, fr.post, fr.occ);
            }
        }
    }
}

__global__ void batch_reset_kernel(unsigned long long *counters)
{
    if (threadIdx.x < kCounters) counters[threadIdx.x] = 0ull;
}

// ---- staged batch ------------------------------------------------------------
// The frames form a few groups (contiguous in table order, about equal cost);
// launch s runs the likelihood chunks of group s beside the fusion bricks of
// group s-1 (whose maps launch s-1 wrote), so the HBM-bound likelihood stream
// and the gather-bound fusion share the GPU for most of the batch. A
// workgroup alternates between the two kinds of work, popping kGroup items
// at a time from the launch's own counters, and leaves when both are used
// up. Within a frame the bricks run octant by octant, so a slice of
// consecutive bricks is a compact block of the grid; a workgroup finds the
// frame of its first brick by binary search and steps forward from there.
constexpr int kStageCounters = 1 + kNumXcd;     // chunk counter, then one per XCD slice of bricks
static_assert((kBatchMaxStages + 1) * kStageCounters * sizeof(unsigned long long) <= kBatchCounterBytes,
              "counters of every staged launch");

template <int TX, int TY, int KZ, int SAMPLING>
__device__ __forceinline__ void batch_brick(const BatchArgs &a, const BatchFrame &fr, int64_t lb)
{
    const uint32_t ntx = static_cast<uint32_t>((fr.grid.nx + TX - 1) / TX), nty = static_cast<uint32_t>((fr.grid.ny + TY - 1) / TY);
    const uint32_t nzc = static_cast<uint32_t>((fr.grid.nz + KZ - 1) / KZ);
    uint32_t txi, tyi, zc;
    octant_tile(static_cast<uint32_t>(lb), ntx, nty, nzc, txi, tyi, zc);
    const int i = static_cast<int>(txi) * TX + static_cast<int>(threadIdx.x % TX);
    const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x / TX);
    const BatchView *views = a.views + fr.view0;
    fuse_column<TX, KZ, SAMPLING>([&](int v) -> const ViewGeom & { return views[v].g; }, fr.n, a.lmap, fr.grid, i, j,
                                  static_cast<int>(zc) * KZ, a.L0, a.tau, fr.post, fr.occ);
}

template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void batch_stage_kernel(BatchArgs a, int stage)
{
    static_assert(TX * TY == 256, "four waves: one likelihood chunk of kWavePixels per wave");
    __shared__ SlmStage st[4];
    unsigned long long *cnt = a.counters + stage * kStageCounters;
    const int wave = static_cast<int>(threadIdx.x >> 6);
    const bool has_l = stage < a.nstages, has_f = stage >= 1;
    const int64_t c_lo = has_l ? a.stage_chunk[stage] : 0, c_hi = has_l ? a.stage_chunk[stage + 1] : 0;
    const int64_t b_lo = has_f ? a.stage_brick[stage - 1] : 0, b_hi = has_f ? a.stage_brick[stage] : 0;
    const int home = static_cast<int>(blockIdx.x % kNumXcd);       // workgroups go to the XCDs in turn
    bool ldone = c_lo >= c_hi, fdone = b_lo >= b_hi;
    int q = 0;                                                      // fusion slice offset from home
    while (!ldone || !fdone) {
        if (!ldone) {
            const int64_t c0 = c_lo + pop(cnt);
            if (c0 >= c_hi) {
                ldone = true;
            } else {
                const int64_t c1 = c0 + kGroup < c_hi ? c0 + kGroup : c_hi;
                int v = __builtin_amdgcn_readfirstlane(find_view(a.views, a.nviews, c0));
                for (int64_t c = c0; c < c1; ++c) {
                    while (v + 1 < a.nviews && a.views[v + 1].chunk0 <= c) ++v;
                    const BatchView &bv = a.views[v];
                    const int64_t p0 = (c - bv.chunk0) * kChunkPixels + wave * kWavePixels;
                    float *out = a.lmap + bv.g.map_off;
                    if (p0 + kWavePixels <= bv.npix)
                        slm_wave(bv.img, bv.mean, bv.var, out, p0, a.k0, st[wave], nullptr);
                    else if (p0 < bv.npix)
                        slm_wave_tail(bv.img, bv.mean, bv.var, out, p0, bv.npix, a.k0, nullptr);
                }
            }
        }
        while (!fdone) {
            const int slice = (home + q) % kNumXcd;
            const int64_t n = b_hi - b_lo;
            const int64_t lo = b_lo + n * slice / kNumXcd, hi = b_lo + n * (slice + 1) / kNumXcd;
            const int64_t b0 = lo + pop(cnt + 1 + slice);
            if (b0 >= hi) {
                if (++q == kNumXcd) fdone = true;
                continue;                                           // try the next slice
            }
            const int64_t b1 = b0 + kGroup < hi ? b0 + kGroup : hi;
            int f = __builtin_amdgcn_readfirstlane(find_frame(a.frames, a.nframes, b0));
            for (int64_t b = b0; b < b1; ++b) {
                while (f + 1 < a.nframes && a.frames[f + 1].brick0 <= b) ++f;
                const BatchFrame &fr = a.frames[f];
                batch_brick<TX, TY, KZ, SAMPLING>(a, fr, b - fr.brick0);
            }
            break;                                                  // one fusion group per turn
        }
    }
}

__global__ void batch_stage_reset_kernel(unsigned long long *counters)
{
    if (threadIdx.x < (kBatchMaxStages + 1) * kStageCounters) counters[threadIdx.x] = 0ull;
}

template <int S>
hipError_t launch_stage_s(const BatchArgs &a, int tile, int grid, int stage, hipStream_t s)
{
    const dim3 g(static_cast<unsigned>(grid)), b(256);
    switch (tile) {
    case 0: hipLaunchKernelGGL((batch_stage_kernel<8, 32, 4, S>), g, b, 0, s, a, stage); break;
    case 1: hipLaunchKernelGGL((batch_stage_kernel<8, 32, 8, S>), g, b, 0, s, a, stage); break;
    case 3: hipLaunchKernelGGL((batch_stage_kernel<8, 32, 2, S>), g, b, 0, s, a, stage); break;
    case 4: hipLaunchKernelGGL((batch_stage_kernel<32, 8, 4, S>), g, b, 0, s, a, stage); break;
    case 5: hipLaunchKernelGGL((batch_stage_kernel<16, 16, 4, S>), g, b, 0, s, a, stage); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S>
int stage_occupancy_s(int tile)
{
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (tile) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_stage_kernel<8, 32, 4, S>, 256, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_stage_kernel<8, 32, 8, S>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_stage_kernel<8, 32, 2, S>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_stage_kernel<32, 8, 4, S>, 256, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_stage_kernel<16, 16, 4, S>, 256, 0); break;
    default: break;
    }
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
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

bool batch_staged_tile(int tile) { return tile != 2; }

int batch_stage_occupancy(int tile, int sampling)
{
    return sampling == PSFS_BILINEAR ? stage_occupancy_s<PSFS_BILINEAR>(tile) : stage_occupancy_s<PSFS_NEAREST>(tile);
}

hipError_t launch_batch_staged(const BatchArgs &a, int tile, int sampling, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(batch_stage_reset_kernel, dim3(1), dim3(64), 0, s, a.counters);
    hipError_t e = hipGetLastError();
    for (int st = 0; st <= a.nstages && e == hipSuccess; ++st)
        e = sampling == PSFS_BILINEAR ? launch_stage_s<PSFS_BILINEAR>(a, tile, grid, st, s)
                                      : launch_stage_s<PSFS_NEAREST>(a, tile, grid, st, s);
    return e;
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
