// Particle weights of the annealed particle filter (Sec. 2.3.1-2.3.2): for
// each particle and view, the outline points of the body model's ten
// cylinders are looked up in the view's edge map (Eq. 14) and their
// silhouette points in the silhouette map (Eq. 15); log w = -(sum over views
// of the two means of 1 - p) (Eq. 16); the weights w^beta are then
// normalised over the particles (Eq. 10).
//
// Sample points of a cylinder (A, B, rA, rB) seen from a camera centre C: 8
// cross-sections at t = (m + 1/2) / 8 with centre X = A + t (B - A) and radius
// r = rA + t (rB - rA); u = the unit component of X - C across the axis (its
// length rho), e = axis x u. Outline points: X - (r^2/rho) u +- r sqrt(1 -
// r^2/rho^2) e, where the viewing ray touches the cross-section circle;
// silhouette points: X and X +- (r/2) e. A point reads the map at its nearest
// pixel (the rule of Eq. 3-9) and counts p = 0 behind the camera, outside the
// image, or when the circle holds the camera centre (rho <= r).
//
// Layout: one workgroup per particle; each view gets wpv = 16 / n waves (1 to
// 16, so a workgroup holds at most 1024 threads) and their lanes share the 80
// (cylinder, cross-section) pairs, pair s going to wave s % wpv, lane s / wpv.
// Up to 8 views every lane has at most one pair: a lane's work is one chain of
// FP64 arithmetic and five map reads, and with only a few hundred particles
// per layer the kernel is bound by the latency of that chain, not by HBM or
// MFMA throughput, so the chain is kept short (one reciprocal per projected
// point, hardware reciprocal refined by Newton steps) and spread wide.
// The geometry runs in FP64: a pixel is the floor of a projected coordinate,
// so the projection's precision decides which pixel is read. Sums are reduced
// by a fixed butterfly and in a fixed order over waves and views, so every
// result is reproducible bit for bit.
#include <cmath>

#include "particles.h"

namespace psfs {
namespace {

constexpr int kPairs = kCylinders * kSections;     // 80 lane tasks per view
constexpr int kMaxWaves = 16;                      // waves per workgroup
constexpr int kNormThreads = 1024;

struct D3 {
    double x, y, z;
};

__device__ inline D3 add(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 sub3(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 scale(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// 1/c in FP64: hardware reciprocal and two Newton steps (about 1 ulp).
__device__ __forceinline__ double rcp64(double c)
{
    double r = __builtin_amdgcn_rcp(c);
    r = fma(r, fma(-c, r, 1.0), r);
    return fma(r, fma(-c, r, 1.0), r);
}

// Map value at the nearest pixel of world point q; 0 behind the camera or
// outside the image.
__device__ inline double map_at(const double (&P)[12], const float *map, int w, int h, D3 q)
{
    const double hz = P[8] * q.x + P[9] * q.y + P[10] * q.z + P[11];
    if (!(hz > 0.0)) return 0.0;
    const double rz = rcp64(hz);
    const double hx = P[0] * q.x + P[1] * q.y + P[2] * q.z + P[3];
    const double hy = P[4] * q.x + P[5] * q.y + P[6] * q.z + P[7];
    const double x = floor(hx * rz + 0.5);
    const double y = floor(hy * rz + 0.5);
    if (!(x >= 0.0 && x < static_cast<double>(w) && y >= 0.0 && y < static_cast<double>(h))) return 0.0;
    return static_cast<double>(map[static_cast<int64_t>(y) * w + static_cast<int64_t>(x)]);
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// grid (np), block 64 * wpv * max(n, 1) with wpv = waves per view
__global__ __launch_bounds__(1024) void particle_weights_kernel(PartArgs a, int wpv)
{
    __shared__ double part[kMaxWaves][2];
    __shared__ double tot[kPartViews];
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int view = wave / wpv, sub = wave % wpv;
    const int64_t p = blockIdx.x;
    if (view < a.n) {
        const PartView &v = a.view[view];
        double P[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) P[i] = static_cast<double>(v.P[i]);
        // camera centre C = -M^-1 p4 (M the left 3x3, p4 the last column):
        // M^-1 has the columns r1 x r2, r2 x r0, r0 x r1 over det M.
        const D3 r0{P[0], P[1], P[2]}, r1{P[4], P[5], P[6]}, r2{P[8], P[9], P[10]};
        const D3 c12 = cross(r1, r2), c20 = cross(r2, r0), c01 = cross(r0, r1);
        const double det = dot(r0, c12);
        const D3 C = scale(-1.0 / det, add(add(scale(P[3], c12), scale(P[7], c20)), scale(P[11], c01)));

        double se = 0.0, sr = 0.0;
        for (int s = sub + wpv * lane; s < kPairs; s += 64 * wpv) {
            const int c = s / kSections, m = s % kSections;
            const float4 *cp = reinterpret_cast<const float4 *>(a.cyl + (p * kCylinders + c) * kCylFloats);
            const float4 q0 = cp[0], q1 = cp[1];
            const D3 A{q0.x, q0.y, q0.z}, B{q0.w, q1.x, q1.y};
            const double rA = q1.z, rB = q1.w;
            const double t = (m + 0.5) / kSections;
            const D3 d = sub3(B, A);
            const D3 X = add(A, scale(t, d));
            const double r = rA + t * (rB - rA);
            const D3 ax = scale(rcp64(sqrt(dot(d, d))), d);
            D3 wv = sub3(X, C);
            wv = sub3(wv, scale(dot(wv, ax), ax));
            const double rho = sqrt(dot(wv, wv));
            if (!(rho > r)) {               // no outline: all five points read 0
                se += 2.0;
                sr += 3.0;
                continue;
            }
            const double irho = rcp64(rho);
            const D3 u = scale(irho, wv);
            const D3 e = cross(ax, u);
            const double q = r * irho;
            const D3 base = sub3(X, scale(r * q, u));
            const D3 side = scale(r * sqrt(1.0 - q * q), e);
            const D3 half = scale(0.5 * r, e);
            se += (1.0 - map_at(P, v.edge, v.w, v.h, sub3(base, side))) +
                  (1.0 - map_at(P, v.edge, v.w, v.h, add(base, side)));
            sr += (1.0 - map_at(P, v.sil, v.w, v.h, sub3(X, half))) + (1.0 - map_at(P, v.sil, v.w, v.h, X)) +
                  (1.0 - map_at(P, v.sil, v.w, v.h, add(X, half)));
        }
        se = wave_sum(se);
        sr = wave_sum(sr);
        if (lane == 0) {
            part[wave][0] = se;
            part[wave][1] = sr;
        }
    }
    __syncthreads();
    // thread k < n: the two means of view k (its waves' sums in wave order)
    const int k = static_cast<int>(threadIdx.x);
    if (k < a.n) {
        double se = 0.0, sr = 0.0;
        for (int j = 0; j < wpv; ++j) {
            se += part[k * wpv + j][0];
            sr += part[k * wpv + j][1];
        }
        const double me = se / (2.0 * kPairs), mr = sr / (3.0 * kPairs);
        if (a.terms) {
            a.terms[(p * a.n + k) * 2] = me;
            a.terms[(p * a.n + k) * 2 + 1] = mr;
        }
        tot[k] = me + mr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double total = 0.0;
        for (int j = 0; j < a.n; ++j) total += tot[j];
        a.logw[p] = -total;
    }
}

// One workgroup: max of beta * log w, then the sum of exp(beta * log w - max),
// each reduced per wave by a butterfly and over the waves in wave order (the
// same order in every thread), then every weight.
__global__ __launch_bounds__(kNormThreads) void particle_normalise_kernel(NormArgs a)
{
    __shared__ double red[2][kNormThreads / 64];
    const int t = static_cast<int>(threadIdx.x), lane = t & 63, wave = t >> 6;
    if (a.np <= kNormThreads) {
        // one particle per thread: its log weight is read once and its
        // exponential computed once, for the sum and for its weight
        const bool has = t < a.np;
        const double z = has ? a.beta * a.logw[t] : -INFINITY;
        double mx = z;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        if (lane == 0) red[0][wave] = mx;
        __syncthreads();
        double zmax = red[0][0];
        for (int k = 1; k < kNormThreads / 64; ++k) zmax = fmax(zmax, red[0][k]);
        const double e = has ? exp(z - zmax) : 0.0;
        const double sum = wave_sum(e);
        if (lane == 0) red[1][wave] = sum;
        __syncthreads();
        double total = 0.0;
        for (int k = 0; k < kNormThreads / 64; ++k) total += red[1][k];
        if (has) a.weights[t] = e / total;
        return;
    }
    double mx = -INFINITY;
    for (int64_t i = t; i < a.np; i += kNormThreads) mx = fmax(mx, a.beta * a.logw[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (lane == 0) red[0][wave] = mx;
    __syncthreads();
    double zmax = red[0][0];
    for (int k = 1; k < kNormThreads / 64; ++k) zmax = fmax(zmax, red[0][k]);
    double sum = 0.0;
    for (int64_t i = t; i < a.np; i += kNormThreads) sum += exp(a.beta * a.logw[i] - zmax);
    sum = wave_sum(sum);
    if (lane == 0) red[1][wave] = sum;
    __syncthreads();
    double total = 0.0;
    for (int k = 0; k < kNormThreads / 64; ++k) total += red[1][k];
    for (int64_t i = t; i < a.np; i += kNormThreads) a.weights[i] = exp(a.beta * a.logw[i] - zmax) / total;
}

}  // namespace

hipError_t launch_particle_weights(const PartArgs &a, hipStream_t s)
{
    if (a.np <= 0) return hipSuccess;
    const int views = a.n > 0 ? a.n : 1;
    const int wpv = kMaxWaves / views;
    hipLaunchKernelGGL(particle_weights_kernel, dim3(static_cast<uint32_t>(a.np)), dim3(64 * wpv * views), 0, s, a, wpv);
    return hipGetLastError();
}

hipError_t launch_particle_normalise(const NormArgs &a, hipStream_t s)
{
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(particle_normalise_kernel, dim3(1), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace psfs
