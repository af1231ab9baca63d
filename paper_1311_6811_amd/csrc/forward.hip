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
// one 8-byte gather per voxel-view). Launched with 32x8-lane tiles of 4 voxels
// per lane, 2x2 columns per 4-lane group and the outputs regrouped into
// non-temporal row pieces, as the four-frame step (33.6 against 35.4-36.1 us
// per launch at 128^3 x 8 views for the 8x32 tile with per-voxel stores).
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
        const int pos = quad_lane_pos(static_cast<int>(threadIdx.x & 63));
        const int i = static_cast<int>(txi) * TX + (pos % TX);
        const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x >> 6) * (64 / TX) + pos / TX;
        const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
        fuse_column_pair<TX, KZ>([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, i, j,
                                 static_cast<int>(zc) * KZ, f.L0, f.tau, f.post, f.occ, post_b, occ_b,
                                 reinterpret_cast<float *>(&stage[threadIdx.x >> 6]));
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
// size: 32x8 51.7, 16x16 52.5, 16x16x2 53.1, 8x32 56.2 us). Inside a wave the
// lanes hold the 32x2 columns in groups of 2x2 (quad_lane_pos).
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
        const int pos = quad_lane_pos(static_cast<int>(threadIdx.x & 63));
        const int i = static_cast<int>(txi) * TX + (pos % TX);
        const int j = static_cast<int>(tyi) * TY + static_cast<int>(threadIdx.x >> 6) * (64 / TX) + pos / TX;
        const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
        float *const post[4] = {f.post, qo.post[0], qo.post[1], qo.post[2]};
        uint8_t *const occ[4] = {f.occ, qo.occ[0], qo.occ[1], qo.occ[2]};
        fuse_column_quad<TX, KZ>([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, i, j,
                                 static_cast<int>(zc) * KZ, f.L0, f.tau, post, occ,
                                 reinterpret_cast<float *>(&stage[threadIdx.x >> 6]));
    }
}

// ---- one-frame nearest fusion from pixel boxes staged in LDS ----------------
// A workgroup of kSBThreads lanes fuses a kSBX x kSBY x kSBZ block of voxels
// (lane t: column (t % 16, (t / 16) % 16), voxels kSBKZ (t / 256) ..
// kSBKZ (t / 256) + kSBKZ - 1 of the block's slices). Per view, the voxel
// centres of the block project into the hull of its 8 projected corner
// centres (the depth is affine and positive at every corner, so on the block
// the projection is continuous and maps the box into that hull); the pixel
// box around the hull, widened by a bound on the FP32 rounding of the
// per-voxel projection, holds every pixel a voxel-view of the block reads.
// The boxes of all views are copied into one LDS arena in view order by
// direct-to-LDS 4-byte buffer loads (one wave instruction per 64 consecutive
// box entries; pixels outside the image read as 0), so that a workgroup waits
// once for all its loads; the voxel-views then read LDS. Views whose box does
// not fit in what is left of the arena, or whose corners are not clearly in
// front of the camera, are gathered directly; views whose box misses the
// image are skipped (every voxel-view of them adds 0). Same per-voxel
// projection arithmetic, pixel rule and view order as fuse_column: the
// posteriors are bit-identical.
constexpr int kSBX = 16, kSBY = 16, kSBZ = 8;
constexpr int kSBThreads = 512;
constexpr int kSBKZ = kSBX * kSBY * kSBZ / kSBThreads;
constexpr int kSArena = 8192;                       // staged floats per workgroup: 32 KB
static_assert(kSBKZ * (kSBThreads / (kSBX * kSBY)) == kSBZ, "lanes cover the block");

struct SBox {
    int x0, y0, w, area;
    int mode;                                       // 0: misses the image, 1: stageable, 2: direct gathers
};

// Voxel centre coordinate, as every fusion path computes it.
__device__ __forceinline__ float voxel_centre(float o, float h, int i)
{
    return o + h * (static_cast<float>(i) + 0.5f);
}

// Pixel boxes of every view for the block with first voxel (i_lo, j_lo, k_lo)
// (phantom voxels past the grid edge included, so that every lane's voxel
// lies in the hull). Lanes 8v .. 8v+7 of the first two waves take the corners
// of view v in FP64 from the FP32 centres the voxel lanes use; lane 8v writes
// boxes[v]. The FP32 evaluation of floor's argument for a voxel (three
// roundings in each of the numerator and the depth, a reciprocal of 1 ulp and
// a product) is within 1.8e-7 (S_u + |u| S_c) / c + 1.8e-7 |u| of the exact
// value, with S the sum of the absolute terms of a row: over the block S is
// largest and c smallest at a corner. The box is widened by 2^-6 px plus five
// times that bound.
template <class Views>
__device__ __forceinline__ void block_boxes(const Views &views, int n, const GridDesc &a, int i_lo, int j_lo,
                                            int k_lo, SBox *boxes)
{
    const int t = static_cast<int>(threadIdx.x);
    if (t >= 8 * kMaxViews) return;                 // whole waves: the shuffles need every lane
    const int v = (t >> 3) < n ? (t >> 3) : 0;
    const int corner = t & 7;
    const ViewGeom &g = views(v);
    const double X = voxel_centre(a.ox, a.h, i_lo + ((corner & 1) ? kSBX - 1 : 0));
    const double Y = voxel_centre(a.oy, a.h, j_lo + ((corner & 2) ? kSBY - 1 : 0));
    const double Z = voxel_centre(a.oz, a.h, k_lo + ((corner & 4) ? kSBZ - 1 : 0));
    double row[3], sum[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double t0 = static_cast<double>(g.P[4 * q]) * X, t1 = static_cast<double>(g.P[4 * q + 1]) * Y;
        const double t2 = static_cast<double>(g.P[4 * q + 2]) * Z, t3 = static_cast<double>(g.P[4 * q + 3]);
        row[q] = (t0 + t1) + (t2 + t3);
        sum[q] = (fabs(t0) + fabs(t1)) + (fabs(t2) + fabs(t3));
    }
    const double c = row[2];
    // NaN fails every comparison below; the 2^20 limits keep the conversions exact
    bool ok = c > 1e-4 * sum[2] && sum[2] < 1e30;
    const double u = ok ? row[0] / c : 0.0, w = ok ? row[1] / c : 0.0;
    ok = ok && fabs(u) < 1048576.0 && fabs(w) < 1048576.0;
    double umin = u, umax = u, wmin = w, wmax = w, cmin = ok ? c : -1.0;
    double su = sum[0], sw = sum[1], sc = sum[2], au = fabs(u), aw = fabs(w);
#pragma unroll
    for (int m = 1; m <= 4; m <<= 1) {
        umin = fmin(umin, __shfl_xor(umin, m, 64));
        umax = fmax(umax, __shfl_xor(umax, m, 64));
        wmin = fmin(wmin, __shfl_xor(wmin, m, 64));
        wmax = fmax(wmax, __shfl_xor(wmax, m, 64));
        cmin = fmin(cmin, __shfl_xor(cmin, m, 64));
        su = fmax(su, __shfl_xor(su, m, 64));
        sw = fmax(sw, __shfl_xor(sw, m, 64));
        sc = fmax(sc, __shfl_xor(sc, m, 64));
        au = fmax(au, __shfl_xor(au, m, 64));
        aw = fmax(aw, __shfl_xor(aw, m, 64));
    }
    if ((t >> 3) >= n || corner != 0) return;
    SBox b{0, 0, 0, 0, 2};
    if (cmin > 0.0) {
        const double mu = 0.015625 + 9e-7 * ((su + au * sc) / cmin + au);
        const double mw = 0.015625 + 9e-7 * ((sw + aw * sc) / cmin + aw);
        if (mu < 0.25 && mw < 0.25) {
            const int x0 = static_cast<int>(floor(umin - mu)), x1 = static_cast<int>(floor(umax + mu));
            const int y0 = static_cast<int>(floor(wmin - mw)), y1 = static_cast<int>(floor(wmax + mw));
            const int bw = x1 - x0 + 1, bh = y1 - y0 + 1;
            if (x1 < 0 || x0 >= g.W || y1 < 0 || y0 >= g.H)
                b.mode = 0;
            else if (bw <= kSArena && bh <= kSArena && bw * bh <= kSArena)
                b = SBox{x0, y0, bw, bw * bh, 1};
        }
    }
    boxes[v] = b;
}

__device__ __forceinline__ SBox read_sbox(const SBox *boxes, int v)
{
    SBox b;
    b.x0 = __builtin_amdgcn_readfirstlane(boxes[v].x0);
    b.y0 = __builtin_amdgcn_readfirstlane(boxes[v].y0);
    b.w = __builtin_amdgcn_readfirstlane(boxes[v].w);
    b.area = __builtin_amdgcn_readfirstlane(boxes[v].area);
    b.mode = __builtin_amdgcn_readfirstlane(boxes[v].mode);
    return b;
}

template <class Views>
__device__ __forceinline__ void fuse_block(const Views &views, int n, const float *lmap, const GridDesc &a,
                                           uint32_t bi, uint32_t bj, uint32_t bk, float L0, float tau, float *post,
                                           uint8_t *occ, float *arena, SBox *boxes)
{
    const int t = static_cast<int>(threadIdx.x);
    const int wave = t >> 6, lane = t & 63;
    const int i_lo = static_cast<int>(bi) * kSBX, j_lo = static_cast<int>(bj) * kSBY, k_lo = static_cast<int>(bk) * kSBZ;
    const int i = i_lo + (t % kSBX), j = j_lo + (t / kSBX) % kSBY, k0 = k_lo + kSBKZ * (t / (kSBX * kSBY));
    block_boxes(views, n, a, i_lo, j_lo, k_lo, boxes);
    const float X = voxel_centre(a.ox, a.h, i), Y = voxel_centre(a.oy, a.h, j);
    float Z[kSBKZ], L[kSBKZ];
#pragma unroll
    for (int kk = 0; kk < kSBKZ; ++kk) {
        Z[kk] = voxel_centre(a.oz, a.h, k0 + kk);
        L[kk] = L0;
    }
    __syncthreads();                                // boxes visible

    // Stage every view's box that fits in what is left of the arena, in view
    // order (each wave derives the same offsets); box entry e = r w + c is
    // pixel (x0 + c, y0 + r); pixels outside the image get an offset past the
    // end of the map, which loads 0.
    int off = 0;
    for (int v = 0; v < n; ++v) {
        const SBox b = read_sbox(boxes, v);
        if (b.mode != 1 || off + b.area > kSArena) continue;
        const ViewGeom &g = views(v);
        const uint32_t W = static_cast<uint32_t>(g.W), H = static_cast<uint32_t>(g.H);
        const __amdgpu_buffer_rsrc_t rs = map_rsrc(lmap + g.map_off, W * H * 4u);
        const float inv_w = 1.0f / static_cast<float>(b.w);
        for (int q = wave; q * 64 < b.area; q += kSBThreads / 64) {
            const int e = q * 64 + lane;
            if (e < b.area) {
                // (e + 1/2) / w is at least 1/(2w) from an integer and e < 2^22: exact row
                const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_w);
                const int c = e - r * b.w;
                const uint32_t x = static_cast<uint32_t>(b.x0 + c), y = static_cast<uint32_t>(b.y0 + r);
                const uint32_t o = (x < W && y < H) ? (__umul24(y, W) + x) * 4u : 0xFFFFFFFFu;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(arena + off + q * 64),
                                                         4, o, 0, 0, 0);
            }
        }
        off += b.area;
    }
    __syncthreads();                                // every wave's loads have landed

    off = 0;
    for (int v = 0; v < n; ++v) {
        const SBox b = read_sbox(boxes, v);
        if (b.mode == 0) continue;
        const ViewGeom &g = views(v);
        const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
        const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
        const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
        if (b.mode == 1 && off + b.area <= kSArena) {
            // box entry of pixel (x, y): (y - y0) w + (x - x0), exact in FP32
            // (integers below 2^24); the clamp only keeps the reads in the box
            const float *sb = arena + off;
            const float wf = static_cast<float>(b.w);
            const float od = static_cast<float>(b.y0) * wf + static_cast<float>(b.x0);
            const float emax = static_cast<float>(b.area - 1);
#pragma unroll
            for (int kk = 0; kk < kSBKZ; ++kk) {
                const float r = __builtin_amdgcn_rcpf(fmaf(g.P[10], Z[kk], cx));
                const float x = floorf(fmaf(g.P[2], Z[kk], ax) * r);
                const float y = floorf(fmaf(g.P[6], Z[kk], bx) * r);
                const float ef = __builtin_amdgcn_fmed3f(fmaf(y, wf, x - od), 0.0f, emax);
                L[kk] += sb[static_cast<int>(ef)];
            }
            off += b.area;
        } else {
            const uint32_t W = static_cast<uint32_t>(g.W), H = static_cast<uint32_t>(g.H);
            const __amdgpu_buffer_rsrc_t rs = map_rsrc(lmap + g.map_off, W * H * 4u);
            float val[kSBKZ];
#pragma unroll
            for (int kk = 0; kk < kSBKZ; ++kk) {
                const float c = fmaf(g.P[10], Z[kk], cx);
                const float r = __builtin_amdgcn_rcpf(c);
                const int x = static_cast<int>(floorf(fmaf(g.P[2], Z[kk], ax) * r));
                const int y = static_cast<int>(floorf(fmaf(g.P[6], Z[kk], bx) * r));
                const bool ok = c > 0.0f && static_cast<uint32_t>(x) < W && static_cast<uint32_t>(y) < H;
                val[kk] = map_load(rs, ok ? (__umul24(static_cast<uint32_t>(y), W) + static_cast<uint32_t>(x)) * 4u
                                          : 0xFFFFFFFFu);
            }
#pragma unroll
            for (int kk = 0; kk < kSBKZ; ++kk) L[kk] += val[kk];
        }
    }
    if (i >= a.nx || j >= a.ny) return;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    int64_t idx = (static_cast<int64_t>(k0) * a.ny + j) * a.nx + i;
#pragma unroll
    for (int kk = 0; kk < kSBKZ; ++kk, idx += plane) {
        if (k0 + kk < a.nz) {
            const float p = sigmoid_fast(L[kk]);
            post[idx] = p;
            if (occ) occ[idx] = p > tau ? 1 : 0;
        }
    }
}

template <class T>
__host__ __device__ int64_t block_count(const T &a)
{
    return static_cast<int64_t>((a.nx + kSBX - 1) / kSBX) * ((a.ny + kSBY - 1) / kSBY) * ((a.nz + kSBZ - 1) / kSBZ);
}

// One-frame nearest fusion, one voxel block per workgroup; the blocks of one
// XCD form one contiguous octant-ordered range.
__global__ __launch_bounds__(kSBThreads) void fuse_block_kernel(FuseArgs f)
{
    __shared__ float arena[kSArena];
    __shared__ SBox boxes[kMaxViews];
    const int64_t nb = block_count(f);
    const uint32_t b = static_cast<uint32_t>(xcd_remap(blockIdx.x, nb));
    const uint32_t nbx = static_cast<uint32_t>((f.nx + kSBX - 1) / kSBX), nby = static_cast<uint32_t>((f.ny + kSBY - 1) / kSBY);
    const uint32_t nbz = static_cast<uint32_t>((f.nz + kSBZ - 1) / kSBZ);
    uint32_t bi, bj, bk;
    octant_tile(b, nbx, nby, nbz, bi, bj, bk);
    const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
    fuse_block([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, bi, bj, bk, f.L0, f.tau,
               f.post, f.occ, arena, boxes);
}

// Likelihood maps of the next frame and block-staged fusion of the current
// one in one launch, laid out as pipe_kernel with kSBThreads-lane workgroups:
// likelihood rounds first (kSBThreads / 64 waves of kWavePixels pixels per
// workgroup), then fusion rounds (one voxel block each; the blocks of one XCD
// form one contiguous octant-ordered range). The two roles share one LDS
// allocation, so both run four workgroups (32 waves) per CU.
__global__ __launch_bounds__(kSBThreads) void pipe_block_kernel(SlmArgs s, FuseArgs f, PipeArgs p)
{
    constexpr size_t kStageBytes = (kSBThreads / 64) * sizeof(SlmStage);
    constexpr size_t kArenaBytes = kSArena * sizeof(float);
    __shared__ __align__(16) unsigned char lds[kStageBytes > kArenaBytes ? kStageBytes : kArenaBytes];
    __shared__ SBox boxes[kMaxViews];
    const int round = static_cast<int>(blockIdx.x) / kNumXcd, x = static_cast<int>(blockIdx.x) % kNumXcd;
    if (round < p.slm_rounds) {
        const int sb = round * kNumXcd + x;
        if (sb >= s.n * p.slm_per_view) return;
        const int v = sb / p.slm_per_view;
        const SlmView &sv = s.view[v];
        const int wave = static_cast<int>(threadIdx.x >> 6);
        const int64_t p0 = (static_cast<int64_t>(sb - v * p.slm_per_view) * (kSBThreads / 64) + wave) * kWavePixels;
        float *out = s.lmap + sv.map_off;
        SlmStage *stage = reinterpret_cast<SlmStage *>(lds);
        if (p0 + kWavePixels <= sv.npix)
            slm_wave(sv.img, sv.mean, sv.var, out, p0, s.k0, stage[wave], s.fg, InputCheck{s.check, 1u << v});
        else if (p0 < sv.npix)
            slm_wave_tail(sv.img, sv.mean, sv.var, out, p0, sv.npix, s.k0, s.fg, InputCheck{s.check, 1u << v});
    } else {
        const int64_t blk = static_cast<int64_t>(x) * p.fuse_rounds + (round - p.slm_rounds);
        if (blk >= p.fuse_tiles) return;
        const uint32_t nbx = static_cast<uint32_t>((f.nx + kSBX - 1) / kSBX), nby = static_cast<uint32_t>((f.ny + kSBY - 1) / kSBY);
        const uint32_t nbz = static_cast<uint32_t>((f.nz + kSBZ - 1) / kSBZ);
        uint32_t bi, bj, bk;
        octant_tile(static_cast<uint32_t>(blk), nbx, nby, nbz, bi, bj, bk);
        const GridDesc gd{f.nx, f.ny, f.nz, f.ox, f.oy, f.oz, f.h};
        fuse_block([&](int v) -> const ViewGeom & { return f.view[v]; }, f.n, f.lmap, gd, bi, bj, bk, f.L0, f.tau,
                   f.post, f.occ, reinterpret_cast<float *>(lds), boxes);
    }
}

__global__ __launch_bounds__(256) void threshold_kernel(const float *post, int64_t n, float tau, uint8_t *occ)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        occ[i] = post[i] > tau ? 1 : 0;
}

// Tile kBlockTile is the kSBX x kSBY x kSBZ voxel block: the one-frame
// nearest paths fuse it from pixel boxes staged in LDS (fuse_block_kernel),
// bilinear sampling with 16 x 16 columns of 8 voxels.
constexpr TileCfg kTiles[] = {
    {8, 32, 4}, {8, 32, 8}, {8, 16, 4}, {8, 32, 2}, {32, 8, 4}, {16, 16, 4}, {kSBX, kSBY, kSBZ},
};
constexpr int kBlockTile = 6;

hipError_t launch_fuse_block(const FuseArgs &a, hipStream_t s)
{
    const int64_t nb = block_count(a);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(fuse_block_kernel, dim3(static_cast<unsigned>(nb)), dim3(kSBThreads), 0, s, a);
    return hipGetLastError();
}

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
    if (S == PSFS_NEAREST && tile == kBlockTile) {
        PipeArgs p{};
        const int64_t per_wg = (kSBThreads / 64) * kWavePixels;
        const int64_t per_view = sa.n > 0 ? (max_npix + per_wg - 1) / per_wg : 0;
        const int64_t tiles = fa.post ? block_count(fa) : 0;
        p.slm_per_view = static_cast<int32_t>(per_view);
        p.slm_rounds = static_cast<int32_t>((per_view * sa.n + kNumXcd - 1) / kNumXcd);
        p.fuse_rounds = static_cast<int32_t>((tiles + kNumXcd - 1) / kNumXcd);
        p.fuse_tiles = tiles;
        const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL(pipe_block_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kSBThreads), 0, s, sa, fa, p);
        return hipGetLastError();
    }
    switch (tile) {
    case 6: return launch_pipe_t<16, 16, 8, S>(sa, fa, max_npix, s);
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
    if (S == PSFS_NEAREST && tile == kBlockTile) return launch_fuse_block(a, s);
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
    case 6: hipLaunchKernelGGL((fuse_kernel<16, 16, 8, S>), grid, block, 0, s, a); break;
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
    const int64_t tiles = fa.post ? tile_count_of<32, 8, 4>(fa) : 0;
    p.slm_per_view = static_cast<int32_t>(per_view);
    p.slm_rounds = static_cast<int32_t>((slm_blocks + kNumXcd - 1) / kNumXcd);
    p.fuse_rounds = static_cast<int32_t>((tiles + kNumXcd - 1) / kNumXcd);
    p.fuse_tiles = tiles;
    const int64_t blocks = static_cast<int64_t>(p.slm_rounds + p.fuse_rounds) * kNumXcd;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((pipe_pair_kernel<32, 8, 4>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, sa, ib, fa, p,
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
