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

constexpr int kSlmQuads = 2;            // pixel quads per lane in slm_kernel

struct Quad {
    uint32_t w[3];
    f32x4 m[3], v[3];
};

__device__ __forceinline__ void load_quad(const SlmView &sv, int64_t p0, Quad &q)
{
    const uint32_t *iw = reinterpret_cast<const uint32_t *>(sv.img + 3 * p0);
    const f32x4 *mp = reinterpret_cast<const f32x4 *>(sv.mean + 3 * p0);
    const f32x4 *vp = reinterpret_cast<const f32x4 *>(sv.var + 3 * p0);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q.w[r] = __builtin_nontemporal_load(iw + r);
        q.m[r] = __builtin_nontemporal_load(mp + r);
        q.v[r] = __builtin_nontemporal_load(vp + r);
    }
}

__device__ __forceinline__ f32x4 quad_log2slm(const Quad &q, float k0)
{
    f32x4 r;
    r.x = log2slm(byte_of(q.w[0], 0), byte_of(q.w[0], 1), byte_of(q.w[0], 2), q.m[0].x, q.m[0].y, q.m[0].z,
                  q.v[0].x, q.v[0].y, q.v[0].z, k0);
    r.y = log2slm(byte_of(q.w[0], 3), byte_of(q.w[1], 0), byte_of(q.w[1], 1), q.m[0].w, q.m[1].x, q.m[1].y,
                  q.v[0].w, q.v[1].x, q.v[1].y, k0);
    r.z = log2slm(byte_of(q.w[1], 2), byte_of(q.w[1], 3), byte_of(q.w[2], 0), q.m[1].z, q.m[1].w, q.m[2].x,
                  q.v[1].z, q.v[1].w, q.v[2].x, k0);
    r.w = log2slm(byte_of(q.w[2], 1), byte_of(q.w[2], 2), byte_of(q.w[2], 3), q.m[2].y, q.m[2].z, q.m[2].w,
                  q.v[2].y, q.v[2].z, q.v[2].w, k0);
    return r;
}

__device__ __forceinline__ void tail_pixels(const SlmView &sv, float *lmap, float k0, int64_t p0)
{
    for (int64_t p = p0; p < sv.npix; ++p) {
        const uint8_t *I = sv.img + 3 * p;
        const float *m = sv.mean + 3 * p, *v = sv.var + 3 * p;
        lmap[sv.map_off + p] = log2slm(I[0], I[1], I[2], m[0], m[1], m[2], v[0], v[1], v[2], k0);
    }
}

// A lane converts kSlmQuads groups of 4 consecutive pixels, kSlmQuads*256*4
// pixels apart within the workgroup's span; each group is 12 image bytes
// (3 dwords) and 12 floats each of mean and variance (3 x 16 B), naturally
// aligned. All loads are issued before any arithmetic.
__global__ __launch_bounds__(256) void slm_kernel(SlmArgs a)
{
    const SlmView sv = a.view[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (256 * 4 * kSlmQuads) + threadIdx.x * 4;
    Quad q[kSlmQuads];
    bool full[kSlmQuads];
#pragma unroll
    for (int t = 0; t < kSlmQuads; ++t) {
        const int64_t p0 = base + t * 1024;
        full[t] = p0 + 4 <= sv.npix;
        if (full[t]) load_quad(sv, p0, q[t]);
    }
#pragma unroll
    for (int t = 0; t < kSlmQuads; ++t) {
        const int64_t p0 = base + t * 1024;
        if (full[t])
            *reinterpret_cast<f32x4 *>(a.lmap + sv.map_off + p0) = quad_log2slm(q[t], a.k0);
        else if (p0 < sv.npix)
            tail_pixels(sv, a.lmap, a.k0, p0);
    }
}

// Lane layout: a workgroup covers a TX x TY tile of voxel columns (x fastest,
// 64-lane waves are TX x (64/TX) slabs, one voxel thick in z) and KZ
// consecutive z-slices; each lane owns one column segment of KZ voxels.
template <int TX, int TY, int KZ, int SAMPLING>
__global__ __launch_bounds__(TX * TY) void fuse_kernel(FuseArgs a)
{
    const int ntx = (a.nx + TX - 1) / TX, nty = (a.ny + TY - 1) / TY;
    const int64_t ntile = static_cast<int64_t>(ntx) * nty;
    const int64_t nb = ntile * ((a.nz + KZ - 1) / KZ);
    const int64_t b = xcd_remap(blockIdx.x, nb);
    const int64_t zc = b / ntile;
    const int t = static_cast<int>(b - zc * ntile);
    const int tyi = t / ntx, txi = t - tyi * ntx;
    const int i = txi * TX + static_cast<int>(threadIdx.x % TX);
    const int j = tyi * TY + static_cast<int>(threadIdx.x / TX);
    const int k0 = static_cast<int>(zc) * KZ;
    const GridDesc gd{a.nx, a.ny, a.nz, a.ox, a.oy, a.oz, a.h};
    fuse_column<TX, KZ, SAMPLING>([&](int v) -> const ViewGeom & { return a.view[v]; }, a.n, a.lmap, gd, i, j, k0,
                              a.L0, a.tau, a.post, a.occ);
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
    const int64_t per_block = 256 * 4 * kSlmQuads;
    const dim3 grid(static_cast<unsigned>((max_npix + per_block - 1) / per_block), static_cast<unsigned>(a.n));
    hipLaunchKernelGGL(slm_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs &a, int tile, int sampling, hipStream_t s)
{
    return sampling == PSFS_BILINEAR ? launch_fuse_s<PSFS_BILINEAR>(a, tile, s)
                                     : launch_fuse_s<PSFS_NEAREST>(a, tile, s);
}

hipError_t launch_threshold(const float *post, int64_t n, float tau, uint8_t *occ, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(threshold_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, post, n, tau, occ);
    return hipGetLastError();
}

}  // namespace psfs
