// Batched occupancy pass over many frames of uneven shape (grid size, view
// count, image size). The frames (in the table's order) go through a chain of
// launches like the frame-sequence step: launch i computes the likelihood
// maps (Eq. 1-2) of frame i beside the fusion (Eq. 3-9 + threshold) of frame
// i-1, whose maps launch i-1 wrote into the batch's map arena; the first
// launch has no fusion part and the last no likelihood part. Each launch
// reads its frames' descriptors from the device table, so a graph of the
// chain stays valid when the frames' pointers change (the table is uploaded
// before each run). Inside a launch the workgroups come in rounds of kNumXcd
// (one per XCD): the likelihood rounds first, then the fusion rounds, whose
// bricks run octant by octant with one contiguous range per XCD, as in the
// single-frame pipelined kernel. Tiles of 128 lanes run each frame's two
// parts as separate launches instead. Per-pixel and per-column code is that
// of the single-frame kernels, so a batched frame is bit-identical to the
// same frame reconstructed alone.
#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

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

// Likelihood workgroup sb of frame fl: 4 x kWavePixels pixels of one view.
__device__ __forceinline__ void batch_slm_block(const BatchArgs &a, int fl, int sb, int per_view, SlmStage *st)
{
    const BatchFrame &fr = a.frames[fl];
    if (sb >= fr.n * per_view) return;
    const int v = sb / per_view;
    const BatchView &bv = a.views[fr.view0 + v];
    const int wave = static_cast<int>(threadIdx.x >> 6);
    const int64_t p0 = (static_cast<int64_t>(sb - v * per_view) * 4 + wave) * kWavePixels;
    float *out = a.lmap + bv.g.map_off;
    if (p0 + kWavePixels <= bv.npix)
        slm_wave(bv.img, bv.mean, bv.var, out, p0, a.k0, st[wave], nullptr);
    else if (p0 < bv.npix)
        slm_wave_tail(bv.img, bv.mean, bv.var, out, p0, bv.npix, a.k0, nullptr);
}

// Likelihood of frame fl (p.slm_rounds rounds) beside the fusion of frame ff
// (p.fuse_rounds rounds); either part may be empty.
template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void batch_pipe_kernel(BatchArgs a, int fl, int ff, PipeArgs p)
{
    static_assert(TX * TY == 256, "four waves per workgroup");
    __shared__ SlmStage st[4];
    const int round = static_cast<int>(blockIdx.x) / kNumXcd, x = static_cast<int>(blockIdx.x) % kNumXcd;
    if (round < p.slm_rounds) {
        batch_slm_block(a, fl, round * kNumXcd + x, p.slm_per_view, st);
    } else {
        const int64_t tile = static_cast<int64_t>(x) * p.fuse_rounds + (round - p.slm_rounds);
        if (tile >= p.fuse_tiles) return;
        batch_brick<TX, TY, KZ, SAMPLING>(a, a.frames[ff], tile);
    }
}

// The separate launches of the 128-lane tile: a frame's likelihood, then its fusion.
__global__ __launch_bounds__(256) void batch_slm_kernel(BatchArgs a, int fl, int per_view)
{
    __shared__ SlmStage st[4];
    batch_slm_block(a, fl, static_cast<int>(blockIdx.x), per_view, st);
}

template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void batch_fuse_kernel(BatchArgs a, int ff, int64_t tiles)
{
    const int64_t tile = xcd_remap(blockIdx.x, tiles);
    batch_brick<TX, TY, KZ, SAMPLING>(a, a.frames[ff], tile);
}

template <int TX, int TY, int KZ, int S>
hipError_t launch_pipe_t(const BatchArgs &a, int fl, int ff, const PipeArgs &p, hipStream_t s)
{
    const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((batch_pipe_kernel<TX, TY, KZ, S>), dim3(static_cast<unsigned>(blocks)), dim3(TX * TY), 0, s, a,
                       fl, ff, p);
    return hipGetLastError();
}

template <int S>
hipError_t launch_pipe_s(const BatchArgs &a, int tile, int fl, int ff, const PipeArgs &p, hipStream_t s)
{
    switch (tile) {
    case 0: return launch_pipe_t<8, 32, 4, S>(a, fl, ff, p, s);
    case 1: return launch_pipe_t<8, 32, 8, S>(a, fl, ff, p, s);
    case 3: return launch_pipe_t<8, 32, 2, S>(a, fl, ff, p, s);
    case 4: return launch_pipe_t<32, 8, 4, S>(a, fl, ff, p, s);
    case 5: return launch_pipe_t<16, 16, 4, S>(a, fl, ff, p, s);
    case 6: return launch_pipe_t<16, 16, 8, S>(a, fl, ff, p, s);
    default: return hipErrorInvalidValue;
    }
}

template <int S>
hipError_t launch_fuse_s(const BatchArgs &a, int ff, int64_t tiles, hipStream_t s)
{
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL((batch_fuse_kernel<8, 16, 4, S>), dim3(static_cast<unsigned>(tiles)), dim3(128), 0, s, a, ff, tiles);
    return hipGetLastError();
}

}  // namespace

int64_t batch_slm_blocks_per_view(int64_t max_npix) { return (max_npix + 4 * kWavePixels - 1) / (4 * kWavePixels); }

int64_t batch_bricks(int nx, int ny, int nz, int tile)
{
    const TileCfg &c = tile_cfg(tile);
    return static_cast<int64_t>((nx + c.tx - 1) / c.tx) * ((ny + c.ty - 1) / c.ty) * ((nz + c.kz - 1) / c.kz);
}

bool batch_pipelined_tile(int tile) { return tile_cfg(tile).tx * tile_cfg(tile).ty == 256; }

hipError_t launch_batch_step(const BatchArgs &a, int tile, int sampling, int fl, int64_t slm_per_view, int nviews_l,
                             int ff, int64_t fuse_tiles, hipStream_t s)
{
    const int64_t slm_blocks = fl >= 0 ? slm_per_view * nviews_l : 0;
    if (!batch_pipelined_tile(tile)) {
        hipError_t e = hipSuccess;
        if (slm_blocks > 0) {
            hipLaunchKernelGGL(batch_slm_kernel, dim3(static_cast<unsigned>(slm_blocks)), dim3(256), 0, s, a, fl,
                               static_cast<int>(slm_per_view));
            e = hipGetLastError();
        }
        if (e != hipSuccess || ff < 0) return e;
        return sampling == PSFS_BILINEAR ? launch_fuse_s<PSFS_BILINEAR>(a, ff, fuse_tiles, s)
                                         : launch_fuse_s<PSFS_NEAREST>(a, ff, fuse_tiles, s);
    }
    PipeArgs p{};
    p.slm_per_view = static_cast<int32_t>(fl >= 0 ? slm_per_view : 0);
    p.slm_rounds = static_cast<int32_t>((slm_blocks + kNumXcd - 1) / kNumXcd);
    p.fuse_tiles = ff >= 0 ? fuse_tiles : 0;
    p.fuse_rounds = static_cast<int32_t>((p.fuse_tiles + kNumXcd - 1) / kNumXcd);
    return sampling == PSFS_BILINEAR ? launch_pipe_s<PSFS_BILINEAR>(a, tile, fl, ff, p, s)
                                     : launch_pipe_s<PSFS_NEAREST>(a, tile, fl, ff, p, s);
}

}  // namespace psfs
