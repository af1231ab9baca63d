// Differentiable variant of the occupancy pass for gfx950.
//
// Forward: every view's log(2*SLM) map (Eq. 1-2) is sampled bilinearly at the
// projected voxel centre and summed into the logit of Eq. 3-9's posterior,
// L = logit(prior) + sum_k l~_k; the loss is the mean binary cross-entropy
// with logits, softplus(L) - y*L, over a box of voxels.
//
// Backward (hand-written adjoint, projections recomputed, not stored):
//   g_v = dLoss/dL_v = grad_loss * (sigmoid(L_v) - y_v) / |region|
//   adjoint map:  Abar_k[tap] += g_v * w_tap         (w = bilinear weights)
//   camera:       dLoss/dP_k = sum_v g_v * (dl~/du du/dP + dl~/dv dv/dP), with
//                 u = a/c, v = b/c, (a,b,c) = P [X;1]:
//                 du/dP_row0 = X~/c, dv/dP_row1 = X~/c, d(u,v)/dP_row2 = -(u,v) X~/c
//   pixel chain:  dlog(2*SLM)/dd = -sigmoid(d) with d = log N - log u, and
//                 dd/dmu_c = (I_c - mu_c)/v_c,
//                 dd/dv_c = (I_c - mu_c)^2/(2 v_c^2) - 1/(2 v_c).
// Reductions of the loss and of the camera gradients run in a fixed order
// (per lane, a fixed wavefront butterfly, waves in order, workgroups in order
// in FP64). The adjoint maps are accumulated in fixed point: every term
// g_v * w satisfies |g_v * w| <= G = |grad_loss| / |region|, so it is rounded
// to a multiple of 2^-E with 2^E * G <= 2^19; a workgroup's terms for one
// pixel (at most 2048) then fit in int32 in LDS (integer LDS atomics, much
// faster than FP32 ones on this GPU) and the global sums fit in int64 (at most
// 2^31 terms). Integer sums do not depend on order, so all outputs are
// reproducible bit for bit; the rounding error per term is <= 2^-20 G.
#include <algorithm>

#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kBoxCap = 4096;           // floats of one view's pixel box staged in LDS
constexpr int kStageIters = kBoxCap / kBlock;

struct Coords {
    int i, j, kb;                       // lane column, first slice of the workgroup
    int bi, bj;                         // first column of the workgroup
};

__device__ __forceinline__ bool in_region(const DiffArgs &a, int i, int j, int k)
{
    return i >= a.sub[0] && i < a.sub[1] && j >= a.sub[2] && j < a.sub[3] && k >= a.sub[4] && k < a.sub[5];
}

__device__ __forceinline__ float softplusf(float x)
{
    return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// Exponent E of the adjoint fixed point (see the file comment); 0 when G is
// 0 or not finite (every term is then 0 or the input invalid).
// Two's-complement int32 as the uint64 addend of a signed int64 sum.
__device__ __forceinline__ unsigned long long widen(int q)
{
    return static_cast<unsigned long long>(static_cast<long long>(q));
}

__device__ __forceinline__ int adjoint_exponent(float grad_loss, float inv_count)
{
    const float G = fabsf(grad_loss) * inv_count;
    if (!(G > 0.0f) || !isfinite(G)) return 0;
    int e;
    frexpf(G, &e);                      // G < 2^e
    return 19 - e;
}

// Projection rows of view v at an FP64 voxel column (X, Y), from the camera
// matrix widened on the host (kernel arguments: scalar operands of the FMAs).
__device__ __forceinline__ Proj64 proj64_view(const DiffArgs &a, int v, double X, double Y)
{
    const double *P = a.Pd[v];
    Proj64 p;
    p.ax = fma(P[0], X, fma(P[1], Y, P[3]));
    p.bx = fma(P[4], X, fma(P[5], Y, P[7]));
    p.cx = fma(P[8], X, fma(P[9], Y, P[11]));
    p.pz0 = P[2];
    p.pz1 = P[6];
    p.pz2 = P[10];
    return p;
}

// 1/c in FP64: the hardware reciprocal (relative error ~5e-8 on this GPU)
// refined by one Newton step (~2e-15; a projected coordinate of ~1000 px is
// then placed to ~1e-12 px).
__device__ __forceinline__ double rcp64(double c)
{
    const double r = __builtin_amdgcn_rcp(c);
    return fma(r, fma(-c, r, 1.0), r);
}

// One view's projection of a voxel centre, in FP64 (see the forward kernel).
struct Tap4 {
    float fx, fy;
    double x0, y0;
    float u, v, rc;
};

// Projection of a voxel centre known to lie in front of the camera (depth
// c > 0): a voxel of a workgroup whose pixel box is valid, since the depth is
// affine in the position and positive at every corner of the voxel box.
__device__ __forceinline__ void project64_front(const Proj64 &p, double Zd, Tap4 &t)
{
    const double c = fma(p.pz2, Zd, p.cx);
    const double r = rcp64(c);
    const double u = fma(p.pz0, Zd, p.ax) * r;
    const double w = fma(p.pz1, Zd, p.bx) * r;
    t.x0 = floor(u);
    t.y0 = floor(w);
    t.fx = static_cast<float>(u - t.x0);
    t.fy = static_cast<float>(w - t.y0);
    t.u = static_cast<float>(u);
    t.v = static_cast<float>(w);
    t.rc = static_cast<float>(r);
}

// The same for any voxel centre: false when it is not in front.
__device__ __forceinline__ bool project64(const Proj64 &p, double Zd, Tap4 &t)
{
    if (!(fma(p.pz2, Zd, p.cx) > 0.0)) return false;
    project64_front(p, Zd, t);
    return true;
}

// Pixel box [x0, x0+w) x [y0, y0+h) holding both bilinear taps in x and y of
// every voxel centre of the workgroup's voxel box, for every view: the
// projection maps the box into the hull of its 8 projected corners (all in
// front of the camera), widened by 1e-6 px for the lanes' own FP64 rounding.
// Lanes 8v..8v+7 project the corners of view v; the box is stored in LDS.
// ok = 0 when a corner is not in front or the box exceeds kBoxCap floats.
struct PixBox {
    int x0, y0, w, h, ok;
};

// Workgroup of either pass = 16 x 16 voxel columns x kFZ slices, a lane one
// column and its kFZ voxels. Its views' pixel boxes hold ~0.7 pixels per
// voxel at 128^3 x 8 views of 640x480 (~0.9 for 8 x 8 x 16 or 8 x 8 x 32
// blocks), and the per-view work (box, barriers, projection rows) is shared
// by 2048 voxels. The forward's waves are 16 x 4 columns (lane t: column
// (t % 16, t / 16)); the backward's are 8 x 8 columns (wave w, lane l: column
// (8 (w & 1) + l % 8, 8 (w >> 1) + l / 8)), so that fewer of its lanes lie on
// one viewing ray of a ring camera, where they would add into the same
// pixels of the adjoint box (same-address LDS atomics).
constexpr int kFX = 16, kFY = 16, kFZ = 8;

template <bool SQUARE_WAVES>
__device__ __forceinline__ Coords block_coords(int nx, int ny, int nz)
{
    const int ntx = (nx + kFX - 1) / kFX, nty = (ny + kFY - 1) / kFY;
    const int64_t ntile = static_cast<int64_t>(ntx) * nty;
    const int64_t nb = ntile * ((nz + kFZ - 1) / kFZ);
    const int64_t b = xcd_remap(blockIdx.x, nb);
    const int64_t zc = b / ntile;
    const int t = static_cast<int>(b - zc * ntile);
    const int tyi = t / ntx, txi = t - tyi * ntx;
    const int w = static_cast<int>(threadIdx.x >> 6), l = static_cast<int>(threadIdx.x & 63);
    Coords c;
    c.bi = txi * kFX;
    c.bj = tyi * kFY;
    if (SQUARE_WAVES) {
        c.i = c.bi + 8 * (w & 1) + (l & 7);
        c.j = c.bj + 8 * (w >> 1) + (l >> 3);
    } else {
        c.i = c.bi + static_cast<int>(threadIdx.x % kFX);
        c.j = c.bj + static_cast<int>(threadIdx.x / kFX);
    }
    c.kb = static_cast<int>(zc) * kFZ;
    return c;
}

template <int EX, int EY, int EZ>
__device__ __forceinline__ void compute_boxes(const DiffArgs &a, const Coords &q, PixBox *boxes)
{
    for (int t0 = 0; t0 < 8 * a.n; t0 += kBlock) {
        const int t = t0 + static_cast<int>(threadIdx.x);
        const int v = t < 8 * a.n ? t >> 3 : 0;
        const int corner = t & 7;
        const ViewGeom &g = a.view[v];
        const double X = static_cast<double>(a.ox) + static_cast<double>(a.h) * ((corner & 1 ? q.bi + EX - 1 : q.bi) + 0.5);
        const double Y = static_cast<double>(a.oy) + static_cast<double>(a.h) * ((corner & 2 ? q.bj + EY - 1 : q.bj) + 0.5);
        const double Z = static_cast<double>(a.oz) + static_cast<double>(a.h) * ((corner & 4 ? q.kb + EZ - 1 : q.kb) + 0.5);
        const Proj64 p = proj64_view(a, v, X, Y);
        const double c = fma(p.pz2, Z, p.cx);
        double ok = c > 0.0 ? 1.0 : 0.0;
        const double u = fma(p.pz0, Z, p.ax) / c, w = fma(p.pz1, Z, p.bx) / c;
        double umin = u, umax = u, wmin = w, wmax = w;
#pragma unroll
        for (int m = 1; m <= 4; m <<= 1) {
            umin = fmin(umin, __shfl_xor(umin, m, 64));
            umax = fmax(umax, __shfl_xor(umax, m, 64));
            wmin = fmin(wmin, __shfl_xor(wmin, m, 64));
            wmax = fmax(wmax, __shfl_xor(wmax, m, 64));
            ok = fmin(ok, __shfl_xor(ok, m, 64));
        }
        if (t < 8 * a.n && corner == 0) {
            PixBox b{0, 0, 0, 0, 0};
            // NaN or huge coordinates fail these range tests
            if (ok > 0.5 && umin > -1e6 && umax < 1e6 && wmin > -1e6 && wmax < 1e6) {
                b.x0 = static_cast<int>(floor(umin - 1e-6));
                b.y0 = static_cast<int>(floor(wmin - 1e-6));
                b.w = static_cast<int>(floor(umax + 1e-6)) + 2 - b.x0;
                b.h = static_cast<int>(floor(wmax + 1e-6)) + 2 - b.y0;
                // sides are checked before the product so it cannot overflow
                b.ok = (b.w > 0 && b.h > 0 && b.w <= kBoxCap && b.h <= kBoxCap && b.w * b.h <= kBoxCap) ? 1 : 0;
            }
            boxes[v] = b;
        }
    }
}

__device__ __forceinline__ PixBox read_box(const PixBox *boxes, int v)
{
    PixBox b;
    b.x0 = __builtin_amdgcn_readfirstlane(boxes[v].x0);
    b.y0 = __builtin_amdgcn_readfirstlane(boxes[v].y0);
    b.w = __builtin_amdgcn_readfirstlane(boxes[v].w);
    b.h = __builtin_amdgcn_readfirstlane(boxes[v].h);
    b.ok = __builtin_amdgcn_readfirstlane(boxes[v].ok);
    return b;
}

// Element e of a box, row-major: r = e / w without an integer division
// ((e + 1/2) / w is at least 1/(2w) away from an integer for e < 2^22).
__device__ __forceinline__ void box_rc(int e, int w, float inv_w, int &r, int &c)
{
    r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_w);
    c = e - r * w;
}

// Copies a view's map over the box into LDS; pixels outside the image read as
// 0. All loads of a lane are issued before its LDS stores. NP passes of the
// workgroup cover boxes of up to NP * kBlock pixels.
template <int NP>
__device__ __forceinline__ void stage_box_n(float *lds, const PixBox &b, const float *map, int W, int H)
{
    const int area = b.w * b.h;
    const float inv_w = 1.0f / static_cast<float>(b.w);
    float vals[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        const int e = static_cast<int>(threadIdx.x) + t * kBlock;
        vals[t] = 0.0f;
        if (e < area) {
            int r, c;
            box_rc(e, b.w, inv_w, r, c);
            const int x = b.x0 + c, y = b.y0 + r;
            if (x >= 0 && x < W && y >= 0 && y < H) vals[t] = map[static_cast<int64_t>(y) * W + x];
        }
    }
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        const int e = static_cast<int>(threadIdx.x) + t * kBlock;
        if (e < area) lds[e] = vals[t];
    }
}

// stage_box_n with as few passes as the (workgroup-uniform) box needs: most
// boxes of the 8x8-column workgroups hold under 1024 pixels.
__device__ __forceinline__ void stage_box(float *lds, const PixBox &b, const float *map, int W, int H)
{
    const int area = b.w * b.h;
    if (area <= 4 * kBlock)
        stage_box_n<4>(lds, b, map, W, H);
    else if (area <= 8 * kBlock)
        stage_box_n<8>(lds, b, map, W, H);
    else
        stage_box_n<kStageIters>(lds, b, map, W, H);
}

__global__ __launch_bounds__(kBlock) void diff_fwd_kernel(DiffArgs a)
{
    __shared__ float lmap_box[kBoxCap];
    __shared__ PixBox boxes[kMaxViews];
    const Coords q = block_coords<false>(a.nx, a.ny, a.nz);
    compute_boxes<kFX, kFY, kFZ>(a, q, boxes);
    const double Xd = static_cast<double>(a.ox) + static_cast<double>(a.h) * (q.i + 0.5);
    const double Yd = static_cast<double>(a.oy) + static_cast<double>(a.h) * (q.j + 0.5);
    float L[kFZ];
#pragma unroll
    for (int kk = 0; kk < kFZ; ++kk) L[kk] = a.L0;
    __syncthreads();

    for (int v = 0; v < a.n; ++v) {
        const ViewGeom &g = a.view[v];
        const float *map = a.lmap + g.map_off;
        const Proj64 p = proj64_view(a, v, Xd, Yd);
        const PixBox box = read_box(boxes, v);
        if (box.ok) {
            __syncthreads();                // the previous view's reads are done
            stage_box(lmap_box, box, map, g.W, g.H);
            __syncthreads();
            // box element of tap (x0, y0): (y0 - box.y0) w + (x0 - box.x0),
            // exact in FP64 (integers far below 2^53)
            const double wd = static_cast<double>(box.w);
            const double od = static_cast<double>(box.y0) * wd + static_cast<double>(box.x0);
            const int emax = box.w * box.h - box.w - 2;
            // every voxel centre of the workgroup is in front of the camera and
            // has both taps in the box (taps outside the image read the 0s the
            // staging wrote there); the clamp only keeps the reads in the box
#pragma unroll
            for (int kk = 0; kk < kFZ; ++kk) {
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.kb + kk + 0.5);
                Tap4 t;
                project64_front(p, Zd, t);
                const int e = min(max(static_cast<int>(fma(t.y0, wd, t.x0 - od)), 0), emax);
                const float *s = lmap_box + e;
                const float top = fmaf(t.fx, s[1] - s[0], s[0]);
                const float bot = fmaf(t.fx, s[box.w + 1] - s[box.w], s[box.w]);
                L[kk] += fmaf(t.fy, bot - top, top);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < kFZ; ++kk) {
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.kb + kk + 0.5);
                Tap4 t;
                if (!project64(p, Zd, t)) continue;
                L[kk] += bilinear_sample(map, g.W, g.H, t.x0, t.y0, t.fx, t.fy);
            }
        }
    }

    double part = 0.0;
    if (q.i < a.nx && q.j < a.ny) {
#pragma unroll
        for (int kk = 0; kk < kFZ; ++kk) {
            const int k = q.kb + kk;
            if (k >= a.nz) continue;
            const int64_t idx = (static_cast<int64_t>(k) * a.ny + q.j) * a.nx + q.i;
            a.logits[idx] = L[kk];
            if (in_region(a, q.i, q.j, k)) {
                const float y = static_cast<float>(a.labels[idx]);
                part += static_cast<double>(softplusf(L[kk]) - y * L[kk]);
            }
        }
    }
    part = wave_sum(part);
    __shared__ double wsum[kWaves];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += wsum[w];
        a.loss_part[blockIdx.x] = s;
    }
}

// loss = inv_count * sum of the workgroup partials, in a fixed order: thread
// t adds partials t + 256 q (eight loads in flight at a time), then the
// wave butterfly of wave_sum, then the four waves in order.
__global__ __launch_bounds__(256) void loss_finalize_kernel(const double *part, int64_t nparts, float inv_count, float *loss)
{
    __shared__ double wsum[4];
    double s = 0.0;
    for (int64_t b0 = 0; b0 < nparts; b0 += 8 * 256) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t b = b0 + threadIdx.x + 256 * q;
            v[q] = b < nparts ? part[b] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) s += v[q];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *loss = static_cast<float>(((wsum[0] + wsum[1]) + (wsum[2] + wsum[3])) * static_cast<double>(inv_count));
}

__global__ __launch_bounds__(256) void zero_kernel(float *p, int64_t n4)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride)
        reinterpret_cast<f32x4 *>(p)[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

__global__ __launch_bounds__(kBlock) void diff_bwd_kernel(DiffArgs a)
{
    __shared__ __align__(16) float lmap_box[kBoxCap];
    __shared__ int adj_box[kBoxCap];
    __shared__ float cam[kWaves][kMaxViews * 12];
    __shared__ PixBox boxes[kMaxViews];
    const Coords q = block_coords<true>(a.nx, a.ny, a.nz);
    const float X = a.ox + a.h * (static_cast<float>(q.i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(q.j) + 0.5f);
    const double Xd = static_cast<double>(a.ox) + static_cast<double>(a.h) * (q.i + 0.5);
    const double Yd = static_cast<double>(a.oy) + static_cast<double>(a.h) * (q.j + 0.5);
    const float gl = *a.grad_loss;
    const float qscale = ldexpf(1.0f, adjoint_exponent(gl, a.inv_count));

    float gv[kFZ];
    bool any = false;
#pragma unroll
    for (int kk = 0; kk < kFZ; ++kk) {
        const int k = q.kb + kk;
        gv[kk] = 0.0f;
        if (q.i < a.nx && q.j < a.ny && k < a.nz && in_region(a, q.i, q.j, k)) {
            const int64_t idx = (static_cast<int64_t>(k) * a.ny + q.j) * a.nx + q.i;
            gv[kk] = gl * (sigmoidf_stable(a.logits[idx]) - static_cast<float>(a.labels[idx])) * a.inv_count;
            any = any || gv[kk] != 0.0f;
        }
    }
    // a workgroup with no voxel in the loss region contributes nothing
    const bool block_any = __syncthreads_or(any ? 1 : 0) != 0;
    if (block_any) compute_boxes<kFX, kFY, kFZ>(a, q, boxes);
    // the adjoint box starts at zero once; each view's flush clears the
    // entries it reads, and a view scatters only inside its own box
    for (int e = threadIdx.x; e < kBoxCap; e += kBlock) adj_box[e] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    for (int v = 0; v < a.n; ++v) {
        const ViewGeom &g = a.view[v];
        const float *map = a.lmap + g.map_off;
        unsigned long long *adj = reinterpret_cast<unsigned long long *>(a.adj) + g.map_off;
        const Proj64 p = proj64_view(a, v, Xd, Yd);
        PixBox box{0, 0, 0, 0, 0};
        if (block_any) box = read_box(boxes, v);
        if (box.ok) {
            __syncthreads();                // the previous view's flush is done
            stage_box(lmap_box, box, map, g.W, g.H);
            __syncthreads();
        }
        float su = 0.0f, suz = 0.0f, sv = 0.0f, svz = 0.0f, sc = 0.0f, scz = 0.0f;
        if (box.ok) {
            const double wd = static_cast<double>(box.w);
            const double od = static_cast<double>(box.y0) * wd + static_cast<double>(box.x0);
            const int emax = box.w * box.h - box.w - 2;
            // as in the forward kernel: no per-voxel depth or range tests. A
            // voxel whose taps all fall outside the image reads four 0s, adds
            // 0 to the camera sums and scatters only into box pixels outside
            // the image, which the flush skips: the same as skipping it.
#pragma unroll
            for (int kk = 0; kk < kFZ; ++kk) {
                if (gv[kk] == 0.0f) continue;
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.kb + kk + 0.5);
                Tap4 t;
                project64_front(p, Zd, t);
                const float fx = t.fx, fy = t.fy, gk = gv[kk];
                const int q00 = static_cast<int>(rintf(gk * (1.0f - fx) * (1.0f - fy) * qscale));
                const int q10 = static_cast<int>(rintf(gk * fx * (1.0f - fy) * qscale));
                const int q01 = static_cast<int>(rintf(gk * (1.0f - fx) * fy * qscale));
                const int q11 = static_cast<int>(rintf(gk * fx * fy * qscale));
                const int e = min(max(static_cast<int>(fma(t.y0, wd, t.x0 - od)), 0), emax);
                const float l00 = lmap_box[e], l10 = lmap_box[e + 1], l01 = lmap_box[e + box.w], l11 = lmap_box[e + box.w + 1];
                atomicAdd(&adj_box[e], q00);
                atomicAdd(&adj_box[e + 1], q10);
                atomicAdd(&adj_box[e + box.w], q01);
                atomicAdd(&adj_box[e + box.w + 1], q11);
                const float dldu = (1.0f - fy) * (l10 - l00) + fy * (l11 - l01);
                const float dldv = (1.0f - fx) * (l01 - l00) + fx * (l11 - l10);
                const float gu = gk * dldu * t.rc, gw = gk * dldv * t.rc;
                const float gc = -(gu * t.u + gw * t.v);
                const float Z = static_cast<float>(Zd);
                su += gu; suz = fmaf(gu, Z, suz);
                sv += gw; svz = fmaf(gw, Z, svz);
                sc += gc; scz = fmaf(gc, Z, scz);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < kFZ; ++kk) {
                if (gv[kk] == 0.0f) continue;
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.kb + kk + 0.5);
                Tap4 t;
                if (!project64(p, Zd, t)) continue;
                if (!(t.x0 >= -1.0 && t.x0 < g.W && t.y0 >= -1.0 && t.y0 < g.H)) continue;
                const int ix = static_cast<int>(t.x0), iy = static_cast<int>(t.y0);
                const bool xin0 = ix >= 0, xin1 = ix + 1 < g.W, yin0 = iy >= 0, yin1 = iy + 1 < g.H;
                const float fx = t.fx, fy = t.fy, gk = gv[kk];
                const int q00 = static_cast<int>(rintf(gk * (1.0f - fx) * (1.0f - fy) * qscale));
                const int q10 = static_cast<int>(rintf(gk * fx * (1.0f - fy) * qscale));
                const int q01 = static_cast<int>(rintf(gk * (1.0f - fx) * fy * qscale));
                const int q11 = static_cast<int>(rintf(gk * fx * fy * qscale));
                const int64_t base = static_cast<int64_t>(iy) * g.W + ix;
                float l00 = 0.0f, l10 = 0.0f, l01 = 0.0f, l11 = 0.0f;
                if (xin0 && yin0) { l00 = map[base]; atomicAdd(adj + base, widen(q00)); }
                if (xin1 && yin0) { l10 = map[base + 1]; atomicAdd(adj + base + 1, widen(q10)); }
                if (xin0 && yin1) { l01 = map[base + g.W]; atomicAdd(adj + base + g.W, widen(q01)); }
                if (xin1 && yin1) { l11 = map[base + g.W + 1]; atomicAdd(adj + base + g.W + 1, widen(q11)); }
                const float dldu = (1.0f - fy) * (l10 - l00) + fy * (l11 - l01);
                const float dldv = (1.0f - fx) * (l01 - l00) + fx * (l11 - l10);
                const float gu = gk * dldu * t.rc, gw = gk * dldv * t.rc;
                const float gc = -(gu * t.u + gw * t.v);
                const float Z = static_cast<float>(Zd);
                su += gu; suz = fmaf(gu, Z, suz);
                sv += gw; svz = fmaf(gw, Z, svz);
                sc += gc; scz = fmaf(gc, Z, scz);
            }
        }
        if (box.ok) {
            __syncthreads();                // every scatter into the box is done
            const int area = box.w * box.h;
            const float inv_w = 1.0f / static_cast<float>(box.w);
            for (int e = threadIdx.x; e < area; e += kBlock) {
                int r, c;
                box_rc(e, box.w, inv_w, r, c);
                const int x = box.x0 + c, y = box.y0 + r;
                const int val = adj_box[e];
                adj_box[e] = 0;
                if (x >= 0 && x < g.W && y >= 0 && y < g.H && val != 0)
                    atomicAdd(adj + static_cast<int64_t>(y) * g.W + x, widen(val));
            }
        }
        // dLoss/dP row r = sum over the lane's voxels of g_r * (X, Y, Z, 1)
        if (block_any) {
            const float vals[12] = {X * su, Y * su, suz, su, X * sv, Y * sv, svz, sv, X * sc, Y * sc, scz, sc};
            // Wave sums of the 12 entries through LDS, in a fixed order: the
            // wave writes its 12 x 64 values, lane 4e + m adds lanes
            // 16m .. 16m+15 of entry e, then a quad butterfly. The staged box
            // is free here (every wave has passed the view's scatter barrier,
            // and the next view stages after a barrier): each wave uses its
            // own 768 floats of it.
            float *red = lmap_box + wave * (12 * 64);
#pragma unroll
            for (int e = 0; e < 12; ++e) red[e * 64 + lane] = vals[e];
            wave_lds_sync();
            float s = 0.0f;
            if (lane < 48) {
                const f32x4 *src = reinterpret_cast<const f32x4 *>(red + (lane >> 2) * 64 + (lane & 3) * 16);
                const f32x4 r0 = src[0], r1 = src[1], r2 = src[2], r3 = src[3];
                s = (((r0.x + r0.y) + (r0.z + r0.w)) + ((r1.x + r1.y) + (r1.z + r1.w))) +
                    (((r2.x + r2.y) + (r2.z + r2.w)) + ((r3.x + r3.y) + (r3.z + r3.w)));
            }
            s += dpp<0xb1>(s);
            s += dpp<0x4e>(s);
            if (lane < 48 && (lane & 3) == 0) cam[wave][v * 12 + (lane >> 2)] = s;
            wave_lds_sync();
        } else if (lane < 12) {
            cam[wave][v * 12 + lane] = 0.0f;
        }
    }
    __syncthreads();
    const int ne = a.n * 12;
    for (int e = threadIdx.x; e < ne; e += kBlock) {
        float s = 0.0f;
        for (int w = 0; w < kWaves; ++w) s += cam[w][e];
        a.cam_part[static_cast<int64_t>(blockIdx.x) * ne + e] = s;
    }
}

// The 12 camera-gradient entries of view v: gP[12v + e] = sum over the
// backward workgroups b of cam_part[b][12v + e], in FP64 and a fixed order
// (thread t adds b = t, t + 256, ...; then wave butterflies; then the four
// waves in order). Run by one 256-lane workgroup per view of the pixel chain,
// which follows the backward kernel on the stream.
__device__ __forceinline__ void camera_gradient(const ChainArgs &a, int v)
{
    __shared__ double wsum[kWaves][12];
    const int ne = a.n * 12;
    double acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = 0.0;
    for (int64_t b = threadIdx.x; b < a.cam_parts; b += 256) {
        const float *row = a.cam_part + b * ne + v * 12;
#pragma unroll
        for (int e = 0; e < 12; ++e) acc[e] += static_cast<double>(row[e]);
    }
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        const double w = wave_sum(acc[e]);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6][e] = w;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double sum = 0.0;
        for (int w = 0; w < kWaves; ++w) sum += wsum[w][threadIdx.x];
        a.gP[v * 12 + threadIdx.x] = static_cast<float>(sum);
    }
}

// dLoss/dmu_c and dLoss/dvar_c of one pixel from its adjoint A (the
// reciprocal of each variance once, refined to about half an ulp).
__device__ __forceinline__ void chain_pixel(float A, float i0, float i1, float i2, const float m[3], const float v[3],
                                            float k0, float gm[3], float gvv[3])
{
    const float I[3] = {i0, i1, i2};
    float t[3], rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        rv[c] = recip(v[c]);
        t[c] = (I[c] - m[c]) * rv[c];
    }
    const float q = fmaf(I[0] - m[0], t[0], fmaf(I[1] - m[1], t[1], (I[2] - m[2]) * t[2]));   // sum d_c^2 / v_c
    const float half_logdet = (0.5f * kLn2) * (__builtin_amdgcn_logf(v[0] * v[1]) + __builtin_amdgcn_logf(v[2]));
    const float d = (k0 - half_logdet) - 0.5f * q;
    const float s = -A * sigmoid_fast(d);           // dLoss/dd
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        gm[c] = s * t[c];
        gvv[c] = s * (0.5f * t[c] * t[c] - 0.5f * rv[c]);
    }
}

typedef long long i64x2 __attribute__((ext_vector_type(2)));

// The chain for the pixels [p0, p0 + 256) of one view (p0 a multiple of 4,
// all inside the view): each load instruction of the wave reads one
// contiguous span, the lanes regroup the inputs per pixel quad through LDS
// (as the likelihood pass does) and regroup the gradients back so that each
// store instruction writes one contiguous span.
__device__ __forceinline__ void chain_wave(const ChainView &cv, const long long *adj, double unit, float k0,
                                           int64_t p0, SlmStage &st)
{
    const int lane = static_cast<int>(threadIdx.x & 63);
    const f32x4 *mp = reinterpret_cast<const f32x4 *>(cv.mean + 3 * p0);
    const f32x4 *vp = reinterpret_cast<const f32x4 *>(cv.var + 3 * p0);
    const uint32_t *ip = reinterpret_cast<const uint32_t *>(cv.img + 3 * p0);
    const i64x2 *ap = reinterpret_cast<const i64x2 *>(adj + p0 + 4 * lane);
    f32x4 m[3], v[3];
    uint32_t w[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        m[r] = __builtin_nontemporal_load(mp + lane + 64 * r);
        v[r] = __builtin_nontemporal_load(vp + lane + 64 * r);
        w[r] = __builtin_nontemporal_load(ip + lane + 64 * r);
    }
    const i64x2 a01 = __builtin_nontemporal_load(ap), a23 = __builtin_nontemporal_load(ap + 1);
    const float A[4] = {static_cast<float>(static_cast<double>(a01.x) * unit), static_cast<float>(static_cast<double>(a01.y) * unit),
                        static_cast<float>(static_cast<double>(a23.x) * unit), static_cast<float>(static_cast<double>(a23.y) * unit)};
    f32x4 qm[3], qv[3];
    uint32_t qw[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = m[r];
        st.w[lane + 64 * r] = w[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        qm[r] = st.f[3 * lane + r];
        qw[r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) st.f[lane + 64 * r] = v[r];
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) qv[r] = st.f[3 * lane + r];
    wave_lds_sync();
    float mm[12], vv[12], gm[12], gvv[12];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        mm[4 * r] = qm[r].x; mm[4 * r + 1] = qm[r].y; mm[4 * r + 2] = qm[r].z; mm[4 * r + 3] = qm[r].w;
        vv[4 * r] = qv[r].x; vv[4 * r + 1] = qv[r].y; vv[4 * r + 2] = qv[r].z; vv[4 * r + 3] = qv[r].w;
    }
#pragma unroll
    for (int px = 0; px < 4; ++px) {
        const int b = 3 * px;
        chain_pixel(A[px], byte_of(qw[b / 4], b % 4), byte_of(qw[(b + 1) / 4], (b + 1) % 4),
                    byte_of(qw[(b + 2) / 4], (b + 2) % 4), mm + b, vv + b, k0, gm + b, gvv + b);
    }
    f32x4 *gmo = reinterpret_cast<f32x4 *>(cv.gmean + 3 * p0);
    f32x4 *gvo = reinterpret_cast<f32x4 *>(cv.gvar + 3 * p0);
#pragma unroll
    for (int r = 0; r < 3; ++r) st.f[3 * lane + r] = f32x4{gm[4 * r], gm[4 * r + 1], gm[4 * r + 2], gm[4 * r + 3]};
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) gmo[lane + 64 * r] = st.f[lane + 64 * r];
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) st.f[3 * lane + r] = f32x4{gvv[4 * r], gvv[4 * r + 1], gvv[4 * r + 2], gvv[4 * r + 3]};
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) gvo[lane + 64 * r] = st.f[lane + 64 * r];
}

__global__ __launch_bounds__(256) void pixel_chain_kernel(ChainArgs a)
{
    __shared__ SlmStage st[4];
    if (blockIdx.x == 0) camera_gradient(a, static_cast<int>(blockIdx.y));
    const ChainView cv = a.view[blockIdx.y];
    const int wave = static_cast<int>(threadIdx.x >> 6);
    const int64_t pw = (static_cast<int64_t>(blockIdx.x) * 4 + wave) * 256;   // the wave's first pixel
    if (pw >= cv.npix) return;
    const long long *adj = reinterpret_cast<const long long *>(a.adj) + cv.map_off;
    const double unit = ldexp(1.0, -adjoint_exponent(*a.grad_loss, a.inv_count));
    if (pw + 256 <= cv.npix) {
        chain_wave(cv, adj, unit, a.k0, pw, st[wave]);
        return;
    }
    // the view's last, partial span: lane by lane
    const int64_t p0 = pw + 4 * static_cast<int64_t>(threadIdx.x & 63);
    if (p0 >= cv.npix) return;
    for (int64_t p = p0; p < cv.npix && p < p0 + 4; ++p) {
        const uint8_t *I = cv.img + 3 * p;
        const float A = static_cast<float>(static_cast<double>(adj[p]) * unit);
        chain_pixel(A, I[0], I[1], I[2], cv.mean + 3 * p, cv.var + 3 * p, a.k0, cv.gmean + 3 * p, cv.gvar + 3 * p);
    }
}

}  // namespace

int64_t diff_fwd_blocks(int nx, int ny, int nz)
{
    return static_cast<int64_t>((nx + kFX - 1) / kFX) * ((ny + kFY - 1) / kFY) * ((nz + kFZ - 1) / kFZ);
}
int64_t diff_bwd_blocks(int nx, int ny, int nz) { return diff_fwd_blocks(nx, ny, nz); }

hipError_t launch_diff_forward(const DiffArgs &a, float *loss, hipStream_t s)
{
    const int64_t nb = diff_fwd_blocks(a.nx, a.ny, a.nz);
    if (nb > 0) hipLaunchKernelGGL(diff_fwd_kernel, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(loss_finalize_kernel, dim3(1), dim3(256), 0, s, a.loss_part, nb, a.inv_count, loss);
    return hipGetLastError();
}

hipError_t launch_diff_backward(const DiffArgs &a, const ChainArgs &c, int64_t map_floats, int64_t max_npix,
                                float *gP, hipStream_t s)
{
    if (map_floats > 0) {
        const int64_t n4 = map_floats / 4;
        const int64_t blocks = std::min<int64_t>((n4 + 1023) / 1024, 4096);
        hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a.adj, n4);
    }
    const int64_t nb = diff_bwd_blocks(a.nx, a.ny, a.nz);
    if (nb > 0 && a.n > 0) hipLaunchKernelGGL(diff_bwd_kernel, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, a);
    if (a.n > 0) {
        // the pixel chain also sums the camera-gradient partials (camera_gradient)
        ChainArgs ca = c;
        ca.cam_part = a.cam_part;
        ca.cam_parts = nb > 0 ? nb : 0;
        ca.gP = gP;
        const int64_t quads = (max_npix + 3) / 4;
        hipLaunchKernelGGL(pixel_chain_kernel, dim3(static_cast<unsigned>((quads + 255) / 256), static_cast<unsigned>(c.n)),
                           dim3(256), 0, s, ca);
    }
    return hipGetLastError();
}

}  // namespace psfs
