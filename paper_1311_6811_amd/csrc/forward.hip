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

// One lane converts 4 consecutive pixels: 12 image bytes (3 dwords) and 12
// floats each of mean and variance (3 x 16 B), all naturally aligned.
__global__ __launch_bounds__(256) void slm_kernel(SlmArgs a)
{
    const SlmView sv = a.view[blockIdx.y];
    const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 4;
    if (p0 >= sv.npix) return;
    float *out = a.lmap + sv.map_off + p0;
    if (p0 + 4 <= sv.npix) {
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(sv.img + 3 * p0);
        const uint32_t w0 = __builtin_nontemporal_load(iw + 0);
        const uint32_t w1 = __builtin_nontemporal_load(iw + 1);
        const uint32_t w2 = __builtin_nontemporal_load(iw + 2);
        const f32x4 *mp = reinterpret_cast<const f32x4 *>(sv.mean + 3 * p0);
        const f32x4 *vp = reinterpret_cast<const f32x4 *>(sv.var + 3 * p0);
        const f32x4 m0 = __builtin_nontemporal_load(mp + 0);
        const f32x4 m1 = __builtin_nontemporal_load(mp + 1);
        const f32x4 m2 = __builtin_nontemporal_load(mp + 2);
        const f32x4 v0 = __builtin_nontemporal_load(vp + 0);
        const f32x4 v1 = __builtin_nontemporal_load(vp + 1);
        const f32x4 v2 = __builtin_nontemporal_load(vp + 2);
        f32x4 r;
        r.x = log2slm(byte_of(w0, 0), byte_of(w0, 1), byte_of(w0, 2), m0.x, m0.y, m0.z, v0.x, v0.y, v0.z, a.k0);
        r.y = log2slm(byte_of(w0, 3), byte_of(w1, 0), byte_of(w1, 1), m0.w, m1.x, m1.y, v0.w, v1.x, v1.y, a.k0);
        r.z = log2slm(byte_of(w1, 2), byte_of(w1, 3), byte_of(w2, 0), m1.z, m1.w, m2.x, v1.z, v1.w, v2.x, a.k0);
        r.w = log2slm(byte_of(w2, 1), byte_of(w2, 2), byte_of(w2, 3), m2.y, m2.z, m2.w, v2.y, v2.z, v2.w, a.k0);
        *reinterpret_cast<f32x4 *>(out) = r;
    } else {
        for (int64_t p = p0; p < sv.npix; ++p) {
            const uint8_t *I = sv.img + 3 * p;
            const float *m = sv.mean + 3 * p, *v = sv.var + 3 * p;
            out[p - p0] = log2slm(I[0], I[1], I[2], m[0], m[1], m[2], v[0], v[1], v[2], a.k0);
        }
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
    fuse_column<KZ, SAMPLING>([&](int v) -> const ViewGeom & { return a.view[v]; }, a.n, a.lmap, gd, i, j, k0,
                              a.L0, a.tau, a.post, a.occ);
}

__global__ __launch_bounds__(256) void threshold_kernel(const float *post, int64_t n, float tau, uint8_t *occ)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        occ[i] = post[i] > tau ? 1 : 0;
}

constexpr TileCfg kTiles[] = {
    {32, 8, 4}, {32, 8, 2}, {32, 8, 8}, {16, 16, 4}, {64, 4, 4}, {64, 4, 2},
};

template <int S>
hipError_t launch_fuse_s(const FuseArgs &a, int tile, hipStream_t s)
{
    const TileCfg &c = kTiles[tile];
    const int64_t nb = static_cast<int64_t>((a.nx + c.tx - 1) / c.tx) * ((a.ny + c.ty - 1) / c.ty) *
                       ((a.nz + c.kz - 1) / c.kz);
    const dim3 grid(static_cast<unsigned>(nb)), block(c.tx * c.ty);
    switch (tile) {
    case 0: hipLaunchKernelGGL((fuse_kernel<32, 8, 4, S>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((fuse_kernel<32, 8, 2, S>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((fuse_kernel<32, 8, 8, S>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((fuse_kernel<16, 16, 4, S>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((fuse_kernel<64, 4, 4, S>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((fuse_kernel<64, 4, 2, S>), grid, block, 0, s, a); break;
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
    const int64_t quads = (max_npix + 3) / 4;
    const dim3 grid(static_cast<unsigned>((quads + 255) / 256), static_cast<unsigned>(a.n));
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
