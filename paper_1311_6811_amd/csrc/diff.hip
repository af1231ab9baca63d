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
// (per-lane, wavefront shuffle tree, waves in order, workgroups in order in
// FP64), so those two outputs are reproducible bit for bit. The adjoint maps
// are accumulated with FP32 atomics, so the background gradients may differ
// in the last bits between runs.
#include <algorithm>

#include "kernels_common.h"

namespace psfs {
namespace {

using namespace dev;

constexpr int kTX = 32, kTY = 8;        // workgroup = 32 x 8 voxel columns, 4 waves
constexpr int kBlock = kTX * kTY;
constexpr int kWaves = kBlock / 64;
constexpr int kFwdKZ = 4;
constexpr int kBwdKZ = 4;

struct Coords {
    int i, j, k0;
};

template <int KZ>
__device__ __forceinline__ Coords block_coords(int nx, int ny, int nz)
{
    const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY;
    const int64_t ntile = static_cast<int64_t>(ntx) * nty;
    const int64_t nb = ntile * ((nz + KZ - 1) / KZ);
    const int64_t b = xcd_remap(blockIdx.x, nb);
    const int64_t zc = b / ntile;
    const int t = static_cast<int>(b - zc * ntile);
    const int tyi = t / ntx, txi = t - tyi * ntx;
    return Coords{txi * kTX + static_cast<int>(threadIdx.x % kTX), tyi * kTY + static_cast<int>(threadIdx.x / kTX),
                  static_cast<int>(zc) * KZ};
}

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

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// One view's projection of a voxel centre, in FP64 (see the forward kernel).
struct Tap4 {
    float fx, fy;
    double x0, y0;
    float u, v, rc;
};

__device__ __forceinline__ bool project64(const Proj64 &p, double Zd, Tap4 &t)
{
    const double c = fma(p.pz2, Zd, p.cx);
    if (!(c > 0.0)) return false;
    const double r = 1.0 / c;
    const double u = fma(p.pz0, Zd, p.ax) * r;
    const double w = fma(p.pz1, Zd, p.bx) * r;
    t.x0 = floor(u);
    t.y0 = floor(w);
    t.fx = static_cast<float>(u - t.x0);
    t.fy = static_cast<float>(w - t.y0);
    t.u = static_cast<float>(u);
    t.v = static_cast<float>(w);
    t.rc = static_cast<float>(r);
    return true;
}

__global__ __launch_bounds__(kBlock) void diff_fwd_kernel(DiffArgs a)
{
    const Coords q = block_coords<kFwdKZ>(a.nx, a.ny, a.nz);
    const double Xd = static_cast<double>(a.ox) + static_cast<double>(a.h) * (q.i + 0.5);
    const double Yd = static_cast<double>(a.oy) + static_cast<double>(a.h) * (q.j + 0.5);
    float L[kFwdKZ];
#pragma unroll
    for (int kk = 0; kk < kFwdKZ; ++kk) L[kk] = a.L0;

    for (int v = 0; v < a.n; ++v) {
        const ViewGeom &g = a.view[v];
        const float *map = a.lmap + g.map_off;
        const Proj64 p = proj64_column(g, Xd, Yd);
#pragma unroll
        for (int kk = 0; kk < kFwdKZ; ++kk) {
            const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.k0 + kk + 0.5);
            Tap4 t;
            if (project64(p, Zd, t)) L[kk] += bilinear_sample(map, g.W, g.H, t.x0, t.y0, t.fx, t.fy);
        }
    }

    double part = 0.0;
    if (q.i < a.nx && q.j < a.ny) {
#pragma unroll
        for (int kk = 0; kk < kFwdKZ; ++kk) {
            const int k = q.k0 + kk;
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

// loss = inv_count * sum of the workgroup partials (one workgroup, fixed order).
__global__ __launch_bounds__(256) void loss_finalize_kernel(const double *part, int64_t nparts, float inv_count, float *loss)
{
    __shared__ double buf[256];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nparts; b += 256) s += part[b];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = static_cast<float>(buf[0] * static_cast<double>(inv_count));
}

__global__ __launch_bounds__(256) void zero_kernel(float *p, int64_t n4)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride)
        reinterpret_cast<f32x4 *>(p)[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

__global__ __launch_bounds__(kBlock) void diff_bwd_kernel(DiffArgs a)
{
    const Coords q = block_coords<kBwdKZ>(a.nx, a.ny, a.nz);
    const float X = a.ox + a.h * (static_cast<float>(q.i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(q.j) + 0.5f);
    const double Xd = static_cast<double>(a.ox) + static_cast<double>(a.h) * (q.i + 0.5);
    const double Yd = static_cast<double>(a.oy) + static_cast<double>(a.h) * (q.j + 0.5);
    const float gl = *a.grad_loss;

    float gv[kBwdKZ];
#pragma unroll
    for (int kk = 0; kk < kBwdKZ; ++kk) {
        const int k = q.k0 + kk;
        gv[kk] = 0.0f;
        if (q.i < a.nx && q.j < a.ny && k < a.nz && in_region(a, q.i, q.j, k)) {
            const int64_t idx = (static_cast<int64_t>(k) * a.ny + q.j) * a.nx + q.i;
            gv[kk] = gl * (sigmoidf_stable(a.logits[idx]) - static_cast<float>(a.labels[idx])) * a.inv_count;
        }
    }

    __shared__ float cam[kWaves][kMaxViews * 12];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    for (int v = 0; v < a.n; ++v) {
        const ViewGeom &g = a.view[v];
        const float *map = a.lmap + g.map_off;
        float *adj = a.adj + g.map_off;
        const Proj64 p = proj64_column(g, Xd, Yd);
        float su = 0.0f, suz = 0.0f, sv = 0.0f, svz = 0.0f, sc = 0.0f, scz = 0.0f;
#pragma unroll
        for (int kk = 0; kk < kBwdKZ; ++kk) {
            if (gv[kk] == 0.0f) continue;
            const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (q.k0 + kk + 0.5);
            Tap4 t;
            if (!project64(p, Zd, t)) continue;
            if (!(t.x0 >= -1.0 && t.x0 < g.W && t.y0 >= -1.0 && t.y0 < g.H)) continue;
            const int ix = static_cast<int>(t.x0), iy = static_cast<int>(t.y0);
            const bool xin0 = ix >= 0, xin1 = ix + 1 < g.W, yin0 = iy >= 0, yin1 = iy + 1 < g.H;
            const int64_t base = static_cast<int64_t>(iy) * g.W + ix;
            const float fx = t.fx, fy = t.fy, gk = gv[kk];
            float l00 = 0.0f, l10 = 0.0f, l01 = 0.0f, l11 = 0.0f;
            if (xin0 && yin0) { l00 = map[base]; unsafeAtomicAdd(adj + base, gk * (1.0f - fx) * (1.0f - fy)); }
            if (xin1 && yin0) { l10 = map[base + 1]; unsafeAtomicAdd(adj + base + 1, gk * fx * (1.0f - fy)); }
            if (xin0 && yin1) { l01 = map[base + g.W]; unsafeAtomicAdd(adj + base + g.W, gk * (1.0f - fx) * fy); }
            if (xin1 && yin1) { l11 = map[base + g.W + 1]; unsafeAtomicAdd(adj + base + g.W + 1, gk * fx * fy); }
            const float dldu = (1.0f - fy) * (l10 - l00) + fy * (l11 - l01);
            const float dldv = (1.0f - fx) * (l01 - l00) + fx * (l11 - l10);
            const float gu = gk * dldu * t.rc, gw = gk * dldv * t.rc;
            const float gc = -(gu * t.u + gw * t.v);
            const float Z = static_cast<float>(Zd);
            su += gu; suz = fmaf(gu, Z, suz);
            sv += gw; svz = fmaf(gw, Z, svz);
            sc += gc; scz = fmaf(gc, Z, scz);
        }
        // dLoss/dP row r = sum over the lane's voxels of g_r * (X, Y, Z, 1)
        const float vals[12] = {X * su, Y * su, suz, su, X * sv, Y * sv, svz, sv, X * sc, Y * sc, scz, sc};
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const float r = wave_sum(vals[e]);
            if (lane == 0) cam[wave][v * 12 + e] = r;
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

// gP[e] = sum over workgroups of cam_part[b][e], FP64, fixed order. One workgroup per entry.
__global__ __launch_bounds__(256) void cam_finalize_kernel(const float *part, int64_t nparts, int ne, float *gP)
{
    __shared__ double buf[256];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nparts; b += 256) s += static_cast<double>(part[b * ne + e]);
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gP[e] = static_cast<float>(buf[0]);
}

__device__ __forceinline__ void chain_pixel(float A, float i0, float i1, float i2, const float m[3], const float v[3],
                                            float k0, float gm[3], float gvv[3])
{
    const float d = pixel_d(i0, i1, i2, m[0], m[1], m[2], v[0], v[1], v[2], k0);
    const float s = -A * sigmoidf_stable(d);        // dLoss/dd
    const float I[3] = {i0, i1, i2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float t = (I[c] - m[c]) / v[c];
        gm[c] = s * t;
        gvv[c] = s * (0.5f * t * t - 0.5f / v[c]);
    }
}

__global__ __launch_bounds__(256) void pixel_chain_kernel(ChainArgs a)
{
    const ChainView cv = a.view[blockIdx.y];
    const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 4;
    if (p0 >= cv.npix) return;
    const float *A = a.adj + cv.map_off + p0;
    if (p0 + 4 <= cv.npix) {
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(cv.img + 3 * p0);
        const uint32_t w[3] = {iw[0], iw[1], iw[2]};
        const f32x4 *mp = reinterpret_cast<const f32x4 *>(cv.mean + 3 * p0);
        const f32x4 *vp = reinterpret_cast<const f32x4 *>(cv.var + 3 * p0);
        const f32x4 A4 = *reinterpret_cast<const f32x4 *>(A);
        float m[12], v[12], gm[12], gvv[12];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const f32x4 mm = mp[r], vv = vp[r];
            m[4 * r] = mm.x; m[4 * r + 1] = mm.y; m[4 * r + 2] = mm.z; m[4 * r + 3] = mm.w;
            v[4 * r] = vv.x; v[4 * r + 1] = vv.y; v[4 * r + 2] = vv.z; v[4 * r + 3] = vv.w;
        }
        const float Av[4] = {A4.x, A4.y, A4.z, A4.w};
#pragma unroll
        for (int px = 0; px < 4; ++px) {
            const int b = 3 * px;
            chain_pixel(Av[px], byte_of(w[b / 4], b % 4), byte_of(w[(b + 1) / 4], (b + 1) % 4),
                        byte_of(w[(b + 2) / 4], (b + 2) % 4), m + b, v + b, a.k0, gm + b, gvv + b);
        }
        f32x4 *gmo = reinterpret_cast<f32x4 *>(cv.gmean + 3 * p0);
        f32x4 *gvo = reinterpret_cast<f32x4 *>(cv.gvar + 3 * p0);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            gmo[r] = f32x4{gm[4 * r], gm[4 * r + 1], gm[4 * r + 2], gm[4 * r + 3]};
            gvo[r] = f32x4{gvv[4 * r], gvv[4 * r + 1], gvv[4 * r + 2], gvv[4 * r + 3]};
        }
    } else {
        for (int64_t p = p0; p < cv.npix; ++p) {
            const uint8_t *I = cv.img + 3 * p;
            chain_pixel(A[p - p0], I[0], I[1], I[2], cv.mean + 3 * p, cv.var + 3 * p, a.k0, cv.gmean + 3 * p,
                        cv.gvar + 3 * p);
        }
    }
}

int64_t nblocks(int nx, int ny, int nz, int kz)
{
    return static_cast<int64_t>((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY) * ((nz + kz - 1) / kz);
}

}  // namespace

int64_t diff_fwd_blocks(int nx, int ny, int nz) { return nblocks(nx, ny, nz, kFwdKZ); }
int64_t diff_bwd_blocks(int nx, int ny, int nz) { return nblocks(nx, ny, nz, kBwdKZ); }

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
        const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 4096);
        hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a.adj, n4);
    }
    const int64_t nb = diff_bwd_blocks(a.nx, a.ny, a.nz);
    if (nb > 0 && a.n > 0) hipLaunchKernelGGL(diff_bwd_kernel, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, a);
    if (a.n > 0) {
        hipLaunchKernelGGL(cam_finalize_kernel, dim3(a.n * 12), dim3(256), 0, s, a.cam_part,
                           (nb > 0 ? nb : 0), a.n * 12, gP);
        const int64_t quads = (max_npix + 3) / 4;
        hipLaunchKernelGGL(pixel_chain_kernel, dim3(static_cast<unsigned>((quads + 255) / 256), static_cast<unsigned>(c.n)),
                           dim3(256), 0, s, c);
    }
    return hipGetLastError();
}

}  // namespace psfs
