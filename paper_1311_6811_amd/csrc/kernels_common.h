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

}  // namespace dev
}  // namespace psfs
