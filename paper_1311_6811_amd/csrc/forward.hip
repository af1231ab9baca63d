// Forward kernels of the occupancy pass for gfx950:
//   slm_kernel        Eq. 1-2, per-pixel log(2*SLM) map of every view
//   fuse_kernel       Eq. 3-9, projection + gather + log-domain fusion +
//                     posterior + threshold (nearest or bilinear sampling)
//   threshold_kernel  Sec. 2.2.2 thresholding of an existing posterior
//
// Log-domain form used throughout: with P(O)=1/2 the occluder sum of Eq. 5-9
// gives P(S_k|V=1) = SLM_k and P(S_k|V=0) = 1/2, so each view that sees a voxel
// adds log(2*SLM_k) to the logit of Eq. 3. With SLM = u/(u+N) (Eq. 1-2, equal
// pixel priors), log(2*SLM) = log 2 - softplus(log N - log u).
#include "kernels_common.h"

namespace psfs {

namespace {

using namespace dev;

// A workgroup converts 4 x kWavePixels consecutive pixels of one view
// (grid.y = view); wave w takes the w-th quarter.
__global__ __launch_bounds__(256) void slm_kernel(SlmArgs a)
{
    __shared__ SlmStage stage[4];
    const SlmView &sv = a.view[blockIdx.y];
    const int wave = static_cast<int>(threadIdx.x >> 6);
    const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * 4 + wave) * kWavePixels;
    float *out = a.lmap + sv.map_off;
    if (p0 + kWavePixels <= sv.npix)
        slm_wave(sv.img, sv.mean, sv.var, out, p0, a.k0, stage[wave], a.fg, InputCheck{a.check, 1u << blockIdx.y});
    else if (p0 < sv.npix)
        slm_wave_tail(sv.img, sv.mean, sv.var, out, p0, sv.npix, a.k0, a.fg, InputCheck{a.check, 1u << blockIdx.y});
}

// Lane layout: a workgroup covers a TX x TY tile of voxel columns (x fastest,
// 64-lane waves are TX x (64/TX) slabs, one voxel thick in z) and KZ
// consecutive z-slices; each lane owns one column segment of KZ voxels.
// Logical tile b enumerates (x tile, y tile, z slab) with x fastest.
template <int TX, int TY, int KZ, int SAMPLING>
__device__ __forceinline__ void fuse_tile(const FuseArgs &a, int64_t b)
{
    // tile counts are below nx*ny*nz < 2^31: 32-bit arithmetic
    const uint32_t ntx = static_cast<uint32_t>((a.nx + TX - 1) / TX), nty = static_cast<uint32_t>((a.ny + TY - 1) / TY);
    const uint32_t nzc = static_cast<uint32_t>((a.nz + KZ - 1) / KZ);
    uint32_t txi, tyi, zc;
    octant_tile(static_cast<uint32_t>(b), ntx, nty, nzc, txi, tyi, zc);
    const int i = static_cast<int>(txi) * TX + static_cast<int>(threadIdx.x % TX);
    const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x / TX);
    const int k0 = static_cast<int>(zc) * KZ;
    const GridDesc gd{a.nx, a.ny, a.nz, a.ox, a.oy, a.oz, a.h};
    fuse_column<TX, KZ, SAMPLING>([&](int v) -> const ViewGeom & { return a.view[v]; }, a.n, a.lmap, gd, i, j, k0,
                              a.L0, a.tau, a.post, a.occ);
}

template <int TX, int TY, int KZ>
__host__ __device__ int64_t tile_count_of(const FuseArgs &a)
{
    return static_cast<int64_t>((a.nx + TX - 1) / TX) * ((a.ny + TY - 1) / TY) * ((a.nz + KZ - 1) / KZ);
}

template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void fuse_kernel(FuseArgs a)
{
    fuse_tile<TX, TY, KZ, SAMPLING>(a, xcd_remap(blockIdx.x, tile_count_of<TX, TY, KZ>(a)));
}

// Likelihood maps of the next frame (Eq. 1-2, SlmArgs) and fusion of the
// current frame (Eq. 3-9, FuseArgs, maps written by an earlier launch) in one
// launch; the two parts share no data. Workgroups come in rounds of kNumXcd
// consecutive ones, which the dispatcher places one per XCD: first the
// likelihood rounds (kNumXcd workgroups of 4 x kWavePixels pixels each), then
// the fusion rounds (kNumXcd tiles each). The likelihood workgroups are short
// and HBM-bound; fusion tiles take the slots they free while the stream is
// still running, so the gather- and arithmetic-bound fusion overlaps the
// stream. (Measured at 128^3 x 8 views: this order beat interleaving the two
// kinds of rounds 1:1, 1:2 and 1:4, and both beat two launches by ~15 %.) The
// fusion tiles of one XCD form one contiguous range, as in fuse_kernel.
template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void pipe_kernel(SlmArgs s, FuseArgs f, PipeArgs p)
{
    static_assert(TX * TY == 256, "four waves per workgroup");
    __shared__ SlmStage stage[4];
    const int round = static_cast<int>(blockIdx.x) / kNumXcd, x = static_cast<int>(blockIdx.x) % kNumXcd;
    if (round < p.slm_rounds) {
        const int sr = round;
        const int sb = sr * kNumXcd + x;
        if (sb >= s.n * p.slm_per_view) return;
        const int v = sb / p.slm_per_view;
        const SlmView &sv = s.view[v];
        const int wave = static_cast<int>(threadIdx.x >> 6);
        const int64_t p0 = (static_cast<int64_t>(sb - v * p.slm_per_view) * 4 + wave) * kWavePixels;
        float *out = s.lmap + sv.map_off;
        if (p0 + kWavePixels <= sv.npix)
            slm_wave(sv.img, sv.mean, sv.var, out, p0, s.k0, stage[wave], s.fg, InputCheck{s.check, 1u << v});
        else if (p0 < sv.npix)
            slm_wave_tail(sv.img, sv.mean, sv.var, out, p0, sv.npix, s.k0, s.fg, InputCheck{s.check, 1u << v});
    } else {
        const int fr = round - p.slm_rounds;
        const int64_t tile = static_cast<int64_t>(x) * p.fuse_rounds + fr;
        if (tile >= p.fuse_tiles) return;
        fuse_tile<TX, TY, KZ, SAMPLING>(f, tile);
    }
}

// Two frames of one rig per launch, laid out as pipe_kernel: likelihood rounds
// (pair maps of the next two frames, the background read once for both), then
// fusion rounds (both posteriors of the current pair from one projection and
// one 8-byte gather per voxel-view).
template <int TX, int TY, int KZ>
__global__ __launch_bounds__(TX * TY) void pipe_pair_kernel(SlmArgs s, PairImages ib, FuseArgs f, PipeArgs p,
                                                            float *post_b, uint8_t *occ_b)
{
    static_assert(TX * TY == 256, "four waves per workgroup");
    __shared__ SlmStage stage[4];
    const int round = static_cast<int>(blockIdx.x) / kNumXcd, x = static_cast<int>(blockIdx.x) % kNumXcd;
    if (round < p.slm_rounds) {
        const int sb = round * kNumXcd + x;
        if (sb >= s.n * p.slm_per_view) return;
        const int v = sb / p.slm_per_view;
        const SlmView &sv = s.view[v];
        const int wave = static_cast<int>(threadIdx.x >> 6);
        const int64_t p0 = (static_cast<int64_t>(sb - v * p.slm_per_view) * 4 + wave) * kWavePixels;
        float *out2 = s.lmap + 2 * sv.map_off;
        if (p0 + kWavePixels <= sv.npix)
            slm_wave_pair(sv.img, ib.img[v], sv.mean, sv.var, out2, p0, s.k0, stage[wave], s.fg,
                          InputCheck{s.check, 1u << v});
        else if (p0 < sv.npix)
            slm_wave_pair_tail(sv.img, ib.img[v], sv.mean, sv.var, out2, p0, sv.npix, s.k0, s.fg,
                               InputCheck{s.check, 1u << v});
    } else {
        const int64_t tile = static_cast<int64_t>(x) * p.fuse_rounds + (round - p.slm_rounds);
        if (tile >= p.fuse_tiles) return;
        const uint32_t ntx = static_cast<uint32_t>((f.nx + TX - 1) / TX), nty = static_cast<uint32_t>((f.ny + TY - 1) / TY);
        const uint32_t nzc = static_cast<uint32_t>((f.nz + KZ - 1) / KZ);
        uint32_t txi, tyi, zc;
        octant_tile(static_cast<uint32_t>(tile), ntx, nty, nzc, txi, tyi, zc);
        const int i = static_cast<int>(txi) * TX + static_cast<int>(threadIdx.x % TX);
        const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x / TX);
        const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
        fuse_column_pair<TX, KZ>([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, i, j,
                                 static_cast<int>(zc) * KZ, f.L0, f.tau, f.post, f.occ, post_b, occ_b);
    }
}

// Four frames of one rig per launch, laid out as pipe_pair_kernel with quad
// maps: the background is read once for four frames' likelihoods, and one
// projection and one 16-byte gather per voxel-view serve four posteriors.
// Launched with 32x8-lane tiles of 4 voxels per lane: a wave covers 32x2
// columns, so each frame's u8 occupancy goes out in 32-byte row pieces
// (16x16 tiles wrote 16-byte pieces, which cost 11.5 MB of partial-line
// writes per launch at 128^3 x 8 views) and its 16-byte gathers land on
// fewer map rows than the 8x8 columns of the 8x32 tile (per launch at that
// size: 32x8 51.7, 16x16 52.5, 16x16x2 53.1, 8x32 56.2 us).
template <int TX, int TY, int KZ>
__global__ __launch_bounds__(TX * TY) void pipe_quad_kernel(SlmArgs s, QuadImages qi, FuseArgs f, PipeArgs p,
                                                            QuadOut qo)
{
    static_assert(TX * TY == 256, "four waves per workgroup");
    __shared__ SlmStage stage[4];
    const int round = static_cast<int>(blockIdx.x) / kNumXcd, x = static_cast<int>(blockIdx.x) % kNumXcd;
    if (round < p.slm_rounds) {
        const int sb = round * kNumXcd + x;
        if (sb >= s.n * p.slm_per_view) return;
        const int v = sb / p.slm_per_view;
        const SlmView &sv = s.view[v];
        const int wave = static_cast<int>(threadIdx.x >> 6);
        const int64_t p0 = (static_cast<int64_t>(sb - v * p.slm_per_view) * 4 + wave) * kWavePixels;
        float *out4 = s.lmap + 4 * sv.map_off;
        const uint8_t *const img[4] = {sv.img, qi.img[0][v], qi.img[1][v], qi.img[2][v]};
        if (p0 + kWavePixels <= sv.npix)
            slm_wave_quad(img, sv.mean, sv.var, out4, p0, s.k0, stage[wave], s.fg, InputCheck{s.check, 1u << v});
        else if (p0 < sv.npix)
            slm_wave_quad_tail(img, sv.mean, sv.var, out4, p0, sv.npix, s.k0, s.fg, InputCheck{s.check, 1u << v});
    } else {
        const int64_t tile = static_cast<int64_t>(x) * p.fuse_rounds + (round - p.slm_rounds);
        if (tile >= p.fuse_tiles) return;
        const uint32_t ntx = static_cast<uint32_t>((f.nx + TX - 1) / TX), nty = static_cast<uint32_t>((f.ny + TY - 1) / TY);
        const uint32_t nzc = static_cast<uint32_t>((f.nz + KZ - 1) / KZ);
        uint32_t txi, tyi, zc;
        octant_tile(static_cast<uint32_t>(tile), ntx, nty, nzc, txi, tyi, zc);
        const int i = static_cast<int>(txi) * TX + static_cast<int>(threadIdx.x % TX);
        const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x / TX);
        const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
        float *const post[4] = {f.post, qo.post[0], qo.post[1], qo.post[2]};
        uint8_t *const occ[4] = {f.occ, qo.occ[0], qo.occ[1], qo.occ[2]};
        fuse_column_quad<TX, KZ>([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, i, j,
                                 static_cast<int>(zc) * KZ, f.L0, f.tau, post, occ,
                                 reinterpret_cast<float *>(&stage[threadIdx.x >> 6]));
    }
}

__global__ __launch_bounds__(256) void threshold_kernel(const float *post, int64_t n, float tau, uint8_t *occ)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        occ[i] = post[i] > tau ? 1 : 0;
}

constexpr TileCfg kTiles[] = {
    {8, 32, 4}, {8, 32, 8}, {8, 16, 4}, {8, 32, 2}, {32, 8, 4}, {16, 16, 4},
};

template <int TX, int TY, int KZ, int S>
hipError_t launch_pipe_t(const SlmArgs &sa, const FuseArgs &fa, int64_t max_npix, hipStream_t s)
{
    PipeArgs p{};
    const int64_t per_view = sa.n > 0 ? (max_npix + 4 * kWavePixels - 1) / (4 * kWavePixels) : 0;
    const int64_t slm_blocks = per_view * sa.n;
    const int64_t tiles = fa.post ? tile_count_of<TX, TY, KZ>(fa) : 0;
    p.slm_per_view = static_cast<int32_t>(per_view);
    p.slm_rounds = static_cast<int32_t>((slm_blocks + kNumXcd - 1) / kNumXcd);
    p.fuse_rounds = static_cast<int32_t>((tiles + kNumXcd - 1) / kNumXcd);
    p.fuse_tiles = tiles;
    const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((pipe_kernel<TX, TY, KZ, S>), dim3(static_cast<unsigned>(blocks)), dim3(TX * TY), 0, s, sa, fa, p);
    return hipGetLastError();
}

template <int S>
hipError_t launch_pipe_s(const SlmArgs &sa, const FuseArgs &fa, int tile, int64_t max_npix, hipStream_t s)
{
    switch (tile) {
    case 1: return launch_pipe_t<8, 32, 8, S>(sa, fa, max_npix, s);
    case 3: return launch_pipe_t<8, 32, 2, S>(sa, fa, max_npix, s);
    case 4: return launch_pipe_t<32, 8, 4, S>(sa, fa, max_npix, s);
    case 5: return launch_pipe_t<16, 16, 4, S>(sa, fa, max_npix, s);
    default: return launch_pipe_t<8, 32, 4, S>(sa, fa, max_npix, s);    // tile 0; tile 2 has 128 lanes
    }
}

template <int S>
hipError_t launch_fuse_s(const FuseArgs &a, int tile, hipStream_t s)
{
    const TileCfg &c = kTiles[tile];
    const int64_t nb = static_cast<int64_t>((a.nx + c.tx - 1) / c.tx) * ((a.ny + c.ty - 1) / c.ty) *
                       ((a.nz + c.kz - 1) / c.kz);
    const dim3 grid(static_cast<unsigned>(nb)), block(c.tx * c.ty);
    switch (tile) {
    case 0: hipLaunchKernelGGL((fuse_kernel<8, 32, 4, S>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((fuse_kernel<8, 32, 8, S>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((fuse_kernel<8, 16, 4, S>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((fuse_kernel<8, 32, 2, S>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((fuse_kernel<32, 8, 4, S>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((fuse_kernel<16, 16, 4, S>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int tile_count() { return static_cast<int>(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileCfg &tile_cfg(int tile) { return kTiles[tile]; }
int default_tile() { return 0; }

hipError_t launch_slm(const SlmArgs &a, int64_t max_npix, hipStream_t s)
{
    const int64_t per_block = 4 * kWavePixels;
    const dim3 grid(static_cast<unsigned>((max_npix + per_block - 1) / per_block), static_cast<unsigned>(a.n));
    hipLaunchKernelGGL(slm_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs &a, int tile, int sampling, hipStream_t s)
{
    return sampling == PSFS_BILINEAR ? launch_fuse_s<PSFS_BILINEAR>(a, tile, s)
                                     : launch_fuse_s<PSFS_NEAREST>(a, tile, s);
}

hipError_t launch_pipeline(const SlmArgs &sa, const FuseArgs &fa, int tile, int sampling, int64_t max_npix,
                           hipStream_t s)
{
    return sampling == PSFS_BILINEAR ? launch_pipe_s<PSFS_BILINEAR>(sa, fa, tile, max_npix, s)
                                     : launch_pipe_s<PSFS_NEAREST>(sa, fa, tile, max_npix, s);
}

hipError_t launch_pipeline_pair(const SlmArgs &sa, const PairImages &ib, const FuseArgs &fa, float *post_b,
                                uint8_t *occ_b, int64_t max_npix, hipStream_t s)
{
    PipeArgs p{};
    const int64_t per_view = sa.n > 0 ? (max_npix + 4 * kWavePixels - 1) / (4 * kWavePixels) : 0;
    const int64_t slm_blocks = per_view * sa.n;
    const int64_t tiles = fa.post ? tile_count_of<8, 32, 4>(fa) : 0;
    p.slm_per_view = static_cast<int32_t>(per_view);
    p.slm_rounds = static_cast<int32_t>((slm_blocks + kNumXcd - 1) / kNumXcd);
    p.fuse_rounds = static_cast<int32_t>((tiles + kNumXcd - 1) / kNumXcd);
    p.fuse_tiles = tiles;
    const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((pipe_pair_kernel<8, 32, 4>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, sa, ib, fa, p,
                       post_b, occ_b);
    return hipGetLastError();
}

hipError_t launch_pipeline_quad(const SlmArgs &sa, const QuadImages &qi, const FuseArgs &fa, const QuadOut &qo,
                                int64_t max_npix, hipStream_t s)
{
    PipeArgs p{};
    const int64_t per_view = sa.n > 0 ? (max_npix + 4 * kWavePixels - 1) / (4 * kWavePixels) : 0;
    const int64_t slm_blocks = per_view * sa.n;
    const int64_t tiles = fa.post ? tile_count_of<32, 8, 4>(fa) : 0;
    p.slm_per_view = static_cast<int32_t>(per_view);
    p.slm_rounds = static_cast<int32_t>((slm_blocks + kNumXcd - 1) / kNumXcd);
    p.fuse_rounds = static_cast<int32_t>((tiles + kNumXcd - 1) / kNumXcd);
    p.fuse_tiles = tiles;
    const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((pipe_quad_kernel<32, 8, 4>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, sa, qi, fa, p,
                       qo);
    return hipGetLastError();
}

hipError_t launch_threshold(const float *post, int64_t n, float tau, uint8_t *occ, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(threshold_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, post, n, tau, occ);
    return hipGetLastError();
}

}  // namespace psfs
