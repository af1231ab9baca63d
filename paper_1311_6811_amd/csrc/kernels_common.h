// Device helpers shared by the forward and differentiable kernels.
#pragma once

#include "psfs_internal.h"

namespace psfs {
namespace dev {

constexpr float kLn2 = 0.693147180559945309f;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// d = log N(I | mu, var) - log u of one pixel (Eq. 1), with
// k0 = -1.5*log(2*pi) - log_u: d = k0 - 1/2 * (log(v0*v1*v2) + sum_c d_c^2/v_c).
__device__ __forceinline__ float pixel_d(float i0, float i1, float i2, float m0, float m1, float m2,
                                        float v0, float v1, float v2, float k0)
{
    const float d0 = i0 - m0, d1 = i1 - m1, d2 = i2 - m2;
    const float q = d0 * d0 / v0 + d1 * d1 / v1 + d2 * d2 / v2;
    const float half_logdet = 0.5f * (logf(v0 * v1) + logf(v2));
    return (k0 - half_logdet) - 0.5f * q;
}

// log(2*SLM) = log 2 - softplus(d), since SLM = u/(u+N) = sigmoid(-d) (Eq. 1-2
// with equal pixel priors).
__device__ __forceinline__ float log2slm(float i0, float i1, float i2, float m0, float m1, float m2,
                                         float v0, float v1, float v2, float k0)
{
    const float d = pixel_d(i0, i1, i2, m0, m1, m2, v0, v1, v2, k0);
    const float softplus = fmaxf(d, 0.0f) + log1pf(expf(-fabsf(d)));
    return kLn2 - softplus;
}

// sigmoid(x) without overflow for either sign.
__device__ __forceinline__ float sigmoidf_stable(float x)
{
    const float e = expf(-fabsf(x));
    return x >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
}

__device__ __forceinline__ float byte_of(uint32_t w, int b)
{
    return static_cast<float>((w >> (8 * b)) & 0xffu);
}

// Bilinear sample of a likelihood map at (x0 + fx, y0 + fy); taps outside the
// image count 0. x0, y0 are integral doubles (possibly far outside the image).
__device__ __forceinline__ float bilinear_sample(const float *map, int W, int H, double x0, double y0, float fx, float fy)
{
    if (!(x0 >= -1.0 && x0 < W && y0 >= -1.0 && y0 < H)) return 0.0f;
    const int ix = static_cast<int>(x0), iy = static_cast<int>(y0);
    const bool xin0 = ix >= 0, xin1 = ix + 1 < W, yin0 = iy >= 0, yin1 = iy + 1 < H;
    const int64_t base = static_cast<int64_t>(iy) * W + ix;
    const float l00 = (xin0 && yin0) ? map[base] : 0.0f;
    const float l10 = (xin1 && yin0) ? map[base + 1] : 0.0f;
    const float l01 = (xin0 && yin1) ? map[base + W] : 0.0f;
    const float l11 = (xin1 && yin1) ? map[base + W + 1] : 0.0f;
    const float top = fmaf(fx, l10 - l00, l00);
    const float bot = fmaf(fx, l11 - l01, l01);
    return fmaf(fy, bot - top, top);
}

// Workgroups are dispatched round-robin over the XCDs; give each XCD one
// contiguous range of logical blocks (z-slabs of the grid), so that its L2
// holds one band of rows of every likelihood map.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb)
{
    const int64_t per = nb / kNumXcd;
    if (bid >= per * kNumXcd) return bid;
    return (bid % kNumXcd) * per + bid / kNumXcd;
}

// Projection rows of one view evaluated in FP64 at an FP64 voxel centre:
// the z-independent part once per voxel column, then one FMA per row.
struct Proj64 {
    double ax, bx, cx, pz0, pz1, pz2;
};

__device__ __forceinline__ Proj64 proj64_column(const ViewGeom &g, double X, double Y)
{
    Proj64 p;
    p.ax = fma(static_cast<double>(g.P[0]), X, fma(static_cast<double>(g.P[1]), Y, static_cast<double>(g.P[3])));
    p.bx = fma(static_cast<double>(g.P[4]), X, fma(static_cast<double>(g.P[5]), Y, static_cast<double>(g.P[7])));
    p.cx = fma(static_cast<double>(g.P[8]), X, fma(static_cast<double>(g.P[9]), Y, static_cast<double>(g.P[11])));
    p.pz0 = g.P[2];
    p.pz1 = g.P[6];
    p.pz2 = g.P[10];
    return p;
}

// Eq. 3-9 for one lane's column segment of KZ voxels, (i, j, k0..k0+KZ-1):
// for every view in order k = 0..n-1, project the voxel centre, read the view's
// log(2*SLM) at the nearest pixel (or bilinearly) and add it to the logit;
// then posterior = sigmoid(logit) and occupancy = posterior > tau. The view
// order is fixed, so every lane layout and work decomposition produces the
// same bits. views(v) returns the ViewGeom of view v (P pre-offset by half of
// row 2 for nearest sampling).
template <int KZ, int SAMPLING, class Views>
__device__ __forceinline__ void fuse_column(const Views &views, int n, const float *lmap, const GridDesc &a, int i,
                                            int j, int k0, float L0, float tau, float *post, uint8_t *occ)
{
    const float X = a.ox + a.h * (static_cast<float>(i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(j) + 0.5f);
    float Z[KZ], L[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        Z[kk] = a.oz + a.h * (static_cast<float>(k0 + kk) + 0.5f);
        L[kk] = L0;
    }

    if (SAMPLING == PSFS_NEAREST) {
        for (int v = 0; v < n; ++v) {
            const ViewGeom &g = views(v);
            const float *map = lmap + g.map_off;
            const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
            const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
            const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float c = fmaf(g.P[10], Z[kk], cx);
                const float r = __builtin_amdgcn_rcpf(c);
                const int x = static_cast<int>(floorf(fmaf(g.P[2], Z[kk], ax) * r));
                const int y = static_cast<int>(floorf(fmaf(g.P[6], Z[kk], bx) * r));
                if (c > 0.0f && static_cast<unsigned>(x) < static_cast<unsigned>(g.W) &&
                    static_cast<unsigned>(y) < static_cast<unsigned>(g.H))
                    L[kk] += map[static_cast<int64_t>(y) * g.W + x];
            }
        }
    } else {
        // Bilinear weights turn a projection error du into an error
        // du * (l10 - l00) of the sample, and FP32 cannot place u closer than
        // ~3e-5 px at u ~ 640. The projection is therefore evaluated in FP64
        // (full rate on CDNA4, like unpacked FP32), from the FP64 voxel centre.
        const double Xd = static_cast<double>(a.ox) + static_cast<double>(a.h) * (i + 0.5);
        const double Yd = static_cast<double>(a.oy) + static_cast<double>(a.h) * (j + 0.5);
        for (int v = 0; v < n; ++v) {
            const ViewGeom &g = views(v);
            const float *map = lmap + g.map_off;
            const double ax = fma(static_cast<double>(g.P[0]), Xd, fma(static_cast<double>(g.P[1]), Yd, static_cast<double>(g.P[3])));
            const double bx = fma(static_cast<double>(g.P[4]), Xd, fma(static_cast<double>(g.P[5]), Yd, static_cast<double>(g.P[7])));
            const double cx = fma(static_cast<double>(g.P[8]), Xd, fma(static_cast<double>(g.P[9]), Yd, static_cast<double>(g.P[11])));
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (k0 + kk + 0.5);
                const double c = fma(static_cast<double>(g.P[10]), Zd, cx);
                if (!(c > 0.0)) continue;
                const double r = 1.0 / c;
                const double u = fma(static_cast<double>(g.P[2]), Zd, ax) * r;
                const double w = fma(static_cast<double>(g.P[6]), Zd, bx) * r;
                const double x0 = floor(u), y0 = floor(w);
                const float fx = static_cast<float>(u - x0), fy = static_cast<float>(w - y0);
                L[kk] += bilinear_sample(map, g.W, g.H, x0, y0, fx, fy);
            }
        }
    }

    if (i >= a.nx || j >= a.ny) return;
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        const int k = k0 + kk;
        if (k < a.nz) {
            const int64_t idx = (static_cast<int64_t>(k) * a.ny + j) * a.nx + i;
            const float p = 1.0f / (1.0f + expf(-L[kk]));
            post[idx] = p;
            if (occ) occ[idx] = p > tau ? 1 : 0;
        }
    }
}

}  // namespace dev
}  // namespace psfs
