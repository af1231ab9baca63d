// Device helpers shared by the forward and differentiable kernels.
#pragma once

#include "psfs_internal.h"

namespace psfs {
namespace dev {

constexpr float kLn2 = 0.693147180559945309f;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// 1/v to about half an ulp: hardware reciprocal refined by one Newton step.
__device__ __forceinline__ float recip(float v)
{
    const float r = __builtin_amdgcn_rcpf(v);
    return fmaf(r, fmaf(-v, r, 1.0f), r);
}

// d = log N(I | mu, var) - log u of one pixel (Eq. 1), with
// k0 = -1.5*log(2*pi) - log_u: d = k0 - 1/2 * (log(v0*v1*v2) + sum_c d_c^2/v_c).
// The log-determinant uses the hardware log2 (about 1 ulp): its error enters
// log(2*SLM) at ~1e-6 absolute or less, below the FP32 rounding of d itself.
__device__ __forceinline__ float pixel_d(float i0, float i1, float i2, float m0, float m1, float m2,
                                        float v0, float v1, float v2, float k0)
{
    const float d0 = i0 - m0, d1 = i1 - m1, d2 = i2 - m2;
    const float q = fmaf(d0 * d0, recip(v0), fmaf(d1 * d1, recip(v1), d2 * d2 * recip(v2)));
    const float half_logdet = (0.5f * kLn2) * (__builtin_amdgcn_logf(v0 * v1) + __builtin_amdgcn_logf(v2));
    return (k0 - half_logdet) - 0.5f * q;
}

// log(2*SLM) = log 2 - softplus(d), since SLM = u/(u+N) = sigmoid(-d) (Eq. 1-2
// with equal pixel priors). softplus(d) = max(d,0) + log(1 + e^-|d|) with the
// hardware exp2/log2: 1 + e^-|d| lies in [1, 2], so the absolute error is a
// few 1e-8.
__device__ __forceinline__ float log2slm(float i0, float i1, float i2, float m0, float m1, float m2,
                                         float v0, float v1, float v2, float k0)
{
    constexpr float kLog2E = 1.44269504088896341f;
    const float d = pixel_d(i0, i1, i2, m0, m1, m2, v0, v1, v2, k0);
    const float e = __builtin_amdgcn_exp2f(-fabsf(d) * kLog2E);
    const float softplus = fmaxf(d, 0.0f) + kLn2 * __builtin_amdgcn_logf(1.0f + e);
    return kLn2 - softplus;
}

// 1 / (1 + e^-x) with the hardware exp2 and reciprocal (a few ulp; e^-x
// overflowing to +inf gives 0, as it should).
__device__ __forceinline__ float sigmoid_fast(float x)
{
    constexpr float kLog2E = 1.44269504088896341f;
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-x * kLog2E));
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

// ---- Eq. 1-2 over pixel quads ------------------------------------------------
// A quad is 4 consecutive pixels: 12 image bytes (3 words) and 12 floats each
// of mean and variance (3 x 16 B), interleaved RGB.
struct Quad {
    uint32_t w[3];
    f32x4 m[3], v[3];
};

__device__ __forceinline__ f32x4 quad_log2slm(const Quad &q, f32x4 k0)
{
    f32x4 r;
    r.x = log2slm(byte_of(q.w[0], 0), byte_of(q.w[0], 1), byte_of(q.w[0], 2), q.m[0].x, q.m[0].y, q.m[0].z,
                  q.v[0].x, q.v[0].y, q.v[0].z, k0.x);
    r.y = log2slm(byte_of(q.w[0], 3), byte_of(q.w[1], 0), byte_of(q.w[1], 1), q.m[0].w, q.m[1].x, q.m[1].y,
                  q.v[0].w, q.v[1].x, q.v[1].y, k0.y);
    r.z = log2slm(byte_of(q.w[1], 2), byte_of(q.w[1], 3), byte_of(q.w[2], 0), q.m[1].z, q.m[1].w, q.m[2].x,
                  q.v[1].z, q.v[1].w, q.v[2].x, k0.z);
    r.w = log2slm(byte_of(q.w[2], 1), byte_of(q.w[2], 2), byte_of(q.w[2], 3), q.m[2].y, q.m[2].z, q.m[2].w,
                  q.v[2].y, q.v[2].z, q.v[2].w, k0.w);
    return r;
}

// Colour bin of a pixel in the learned foreground model: 16 levels per
// channel, bin = (R >> 4) * 256 + (G >> 4) * 16 + (B >> 4).
__device__ __forceinline__ uint32_t colour_bin(uint32_t r, uint32_t g, uint32_t b)
{
    return ((r >> 4) << 8) | ((g >> 4) << 4) | (b >> 4);
}

__device__ __forceinline__ uint32_t byte_u(uint32_t w, int b) { return (w >> (8 * b)) & 0xffu; }

// Per-pixel constant of d for a quad: k0 with the uniform foreground density
// (k0 = -1.5 log 2pi - log u); with a learned model (fg = log density per
// colour bin), k0 - fg[bin] where k0 = -1.5 log 2pi.
__device__ __forceinline__ f32x4 quad_k0(const Quad &q, float k0, const float *fg)
{
    f32x4 k{k0, k0, k0, k0};
    if (fg) {
        k.x -= fg[colour_bin(byte_u(q.w[0], 0), byte_u(q.w[0], 1), byte_u(q.w[0], 2))];
        k.y -= fg[colour_bin(byte_u(q.w[0], 3), byte_u(q.w[1], 0), byte_u(q.w[1], 1))];
        k.z -= fg[colour_bin(byte_u(q.w[1], 2), byte_u(q.w[1], 3), byte_u(q.w[2], 0))];
        k.w -= fg[colour_bin(byte_u(q.w[2], 1), byte_u(q.w[2], 2), byte_u(q.w[2], 3))];
    }
    return k;
}

constexpr int kWavePixels = 256;        // pixels per wave in the likelihood kernels

// Optional input validation: Eq. 1 needs every background variance positive
// and finite and every mean finite. A value class test (one instruction per
// value) flags NaN, infinities, zeros and negative variances.
constexpr int kClassPosFinite = (1 << 7) | (1 << 8);            // +denormal, +normal
constexpr int kClassFinite = 0x1f8;                             // -normal .. +normal

__device__ __forceinline__ bool mean_invalid(float m) { return !__builtin_amdgcn_classf(m, kClassFinite); }
__device__ __forceinline__ bool var_invalid(float v) { return !__builtin_amdgcn_classf(v, kClassPosFinite); }

__device__ __forceinline__ bool vec_invalid(const f32x4 &m, const f32x4 &v)
{
    return mean_invalid(m.x) | mean_invalid(m.y) | mean_invalid(m.z) | mean_invalid(m.w) | var_invalid(v.x) |
           var_invalid(v.y) | var_invalid(v.z) | var_invalid(v.w);
}

// Where a wave reports an invalid background value: bit `bit` of *flags
// (view k -> bit k); flags == nullptr turns the check off.
struct InputCheck {
    uint32_t *flags;
    uint32_t bit;
};

// Called by all 64 lanes of a wave: one atomic OR when any lane saw a bad value.
__device__ __forceinline__ void report_wave(const InputCheck &chk, bool bad)
{
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(chk.flags, chk.bit);
}

// LDS of one wave in slm_wave: 192 16-byte vectors (means, then variances;
// slm_wave_quad uses all 256 to regroup its results) and 192 image words.
struct SlmStage {
    f32x4 f[4 * 64];
    uint32_t w[3 * 64];
};

// Orders this wave's LDS stores before its later LDS loads (lanes exchange
// data; no other wave touches the buffer).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The check for the pixels [p, min(p + 4, npix)) of a lane in a wave's tail
// (lanes may have no pixels; each lane with a bad value reports itself).
__device__ __forceinline__ void tail_check(const float *mean, const float *var, int64_t p, int64_t npix,
                                           const InputCheck &chk)
{
    bool bad = false;
    for (int64_t t = 3 * p; t < 3 * p + 12 && t < 3 * npix; ++t) bad |= mean_invalid(mean[t]) | var_invalid(var[t]);
    if (bad) atomicOr(chk.flags, chk.bit);
}

// log(2*SLM) of the kWavePixels pixels [p0, p0 + 256) of one view, all inside
// the view, p0 a multiple of 4. Each global load instruction of the wave reads
// one contiguous span (64 x 16 B of means or variances, 64 x 4 B of image
// bytes); the lanes then regroup the data per pixel quad through LDS, and lane
// l writes pixels p0 + 4l .. p0 + 4l + 3 with one 16-byte store. A strided
// per-quad load (48 B apart per lane) touches three times the cache lines per
// instruction and measured ~40 % slower.
__device__ __forceinline__ void slm_wave(const uint8_t *img, const float *mean, const float *var, float *out,
                                         int64_t p0, float k0, SlmStage &st, const float *fg,
                                         InputCheck chk = InputCheck{nullptr, 0})
{
    const int lane = static_cast<int>(threadIdx.x & 63);
    const f32x4 *mp = reinterpret_cast<const f32x4 *>(mean + 3 * p0);
    const f32x4 *vp = reinterpret_cast<const f32x4 *>(var + 3 * p0);
    const uint32_t *ip = reinterpret_cast<const uint32_t *>(img + 3 * p0);
    f32x4 m[3], v[3];
    uint32_t w[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        m[r] = __builtin_nontemporal_load(mp + lane + 64 * r);
        v[r] = __builtin_nontemporal_load(vp + lane + 64 * r);
        w[r] = __builtin_nontemporal_load(ip + lane + 64 * r);
    }
    if (chk.flags) report_wave(chk, vec_invalid(m[0], v[0]) | vec_invalid(m[1], v[1]) | vec_invalid(m[2], v[2]));
    Quad q;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = m[r];
        st.w[lane + 64 * r] = w[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q.m[r] = st.f[3 * lane + r];
        q.w[r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) st.f[lane + 64 * r] = v[r];
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) q.v[r] = st.f[3 * lane + r];
    wave_lds_sync();
    *reinterpret_cast<f32x4 *>(out + p0 + 4 * lane) = quad_log2slm(q, quad_k0(q, k0, fg));
}

// The same for a wave whose span [p0, p0 + 256) reaches past npix: lane l
// converts its quad p0 + 4l directly, or the pixels of it below npix.
__device__ __forceinline__ void slm_wave_tail(const uint8_t *img, const float *mean, const float *var, float *out,
                                              int64_t p0, int64_t npix, float k0, const float *fg,
                                              InputCheck chk = InputCheck{nullptr, 0})
{
    const int64_t p = p0 + 4 * static_cast<int64_t>(threadIdx.x & 63);
    if (chk.flags) tail_check(mean, var, p, npix, chk);
    if (p + 4 <= npix) {
        Quad q;
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(img + 3 * p);
        const f32x4 *mp = reinterpret_cast<const f32x4 *>(mean + 3 * p);
        const f32x4 *vp = reinterpret_cast<const f32x4 *>(var + 3 * p);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            q.w[r] = iw[r];
            q.m[r] = mp[r];
            q.v[r] = vp[r];
        }
        *reinterpret_cast<f32x4 *>(out + p) = quad_log2slm(q, quad_k0(q, k0, fg));
    } else {
        for (int64_t t = p; t < npix; ++t) {
            const uint8_t *I = img + 3 * t;
            const float *mm = mean + 3 * t, *vv = var + 3 * t;
            const float kt = fg ? k0 - fg[colour_bin(I[0], I[1], I[2])] : k0;
            out[t] = log2slm(I[0], I[1], I[2], mm[0], mm[1], mm[2], vv[0], vv[1], vv[2], kt);
        }
    }
}

// ---- two frames of one rig per pass ------------------------------------------
// Consecutive frames of a sequence share the cameras and the background model.
// Their maps are kept interleaved ("pair maps": pixel p of the view whose map
// starts at map_off holds frame A's log(2*SLM) at float 2*(map_off + p) and
// frame B's right after), so that one projection and one 8-byte gather per
// voxel-view serve both frames, and the likelihood of both frames reads the
// background model once.

// slm_wave for two frames: the means and variances are loaded once; lane l
// converts pixels p0 + 4l .. p0 + 4l + 3 of both frames, and the results leave
// in two lane-contiguous 16-byte stores.
__device__ __forceinline__ void slm_wave_pair(const uint8_t *img_a, const uint8_t *img_b, const float *mean,
                                              const float *var, float *out2, int64_t p0, float k0, SlmStage &st,
                                              const float *fg, InputCheck chk)
{
    const int lane = static_cast<int>(threadIdx.x & 63);
    const f32x4 *mp = reinterpret_cast<const f32x4 *>(mean + 3 * p0);
    const f32x4 *vp = reinterpret_cast<const f32x4 *>(var + 3 * p0);
    const uint32_t *ia = reinterpret_cast<const uint32_t *>(img_a + 3 * p0);
    const uint32_t *ib = reinterpret_cast<const uint32_t *>(img_b + 3 * p0);
    f32x4 m[3], v[3];
    uint32_t wa[3], wb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        m[r] = __builtin_nontemporal_load(mp + lane + 64 * r);
        v[r] = __builtin_nontemporal_load(vp + lane + 64 * r);
        wa[r] = __builtin_nontemporal_load(ia + lane + 64 * r);
        wb[r] = __builtin_nontemporal_load(ib + lane + 64 * r);
    }
    if (chk.flags) report_wave(chk, vec_invalid(m[0], v[0]) | vec_invalid(m[1], v[1]) | vec_invalid(m[2], v[2]));
    Quad qa, qb;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = m[r];
        st.w[lane + 64 * r] = wa[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        qa.m[r] = st.f[3 * lane + r];
        qa.w[r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = v[r];
        st.w[lane + 64 * r] = wb[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        qa.v[r] = st.f[3 * lane + r];
        qb.w[r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        qb.m[r] = qa.m[r];
        qb.v[r] = qa.v[r];
    }
    const f32x4 ra = quad_log2slm(qa, quad_k0(qa, k0, fg));
    const f32x4 rb = quad_log2slm(qb, quad_k0(qb, k0, fg));
    // regrouped through LDS so that each store instruction of the wave writes
    // one contiguous kilobyte (the stage's reads above are ordered before)
    st.f[2 * lane] = f32x4{ra.x, rb.x, ra.y, rb.y};
    st.f[2 * lane + 1] = f32x4{ra.z, rb.z, ra.w, rb.w};
    wave_lds_sync();
    f32x4 *o = reinterpret_cast<f32x4 *>(out2 + 2 * p0);
    o[lane] = st.f[lane];
    o[64 + lane] = st.f[64 + lane];
}

// slm_wave_tail for two frames.
__device__ __forceinline__ void slm_wave_pair_tail(const uint8_t *img_a, const uint8_t *img_b, const float *mean,
                                                   const float *var, float *out2, int64_t p0, int64_t npix, float k0,
                                                   const float *fg, InputCheck chk)
{
    const int64_t p = p0 + 4 * static_cast<int64_t>(threadIdx.x & 63);
    if (chk.flags) tail_check(mean, var, p, npix, chk);
    for (int64_t t = p; t < p + 4 && t < npix; ++t) {
        const uint8_t *A = img_a + 3 * t, *B = img_b + 3 * t;
        const float *mm = mean + 3 * t, *vv = var + 3 * t;
        const float ka = fg ? k0 - fg[colour_bin(A[0], A[1], A[2])] : k0;
        const float kb = fg ? k0 - fg[colour_bin(B[0], B[1], B[2])] : k0;
        out2[2 * t] = log2slm(A[0], A[1], A[2], mm[0], mm[1], mm[2], vv[0], vv[1], vv[2], ka);
        out2[2 * t + 1] = log2slm(B[0], B[1], B[2], mm[0], mm[1], mm[2], vv[0], vv[1], vv[2], kb);
    }
}

// ---- four frames of one rig per pass -----------------------------------------
// "Quad maps" interleave four frames' maps the same way: pixel p of the view
// whose map starts at map_off holds frame f's log(2*SLM) at float
// 4*(map_off + p) + f, so one 16-byte gather per voxel-view serves all four.

// slm_wave for four frames: the means and variances are loaded once and
// regrouped once; the four images' words are regrouped one after another
// through the same LDS words. Lane l converts pixels p0 + 4l .. p0 + 4l + 3 of
// the four frames; the results leave in four lane-contiguous 16-byte stores.
__device__ __forceinline__ void slm_wave_quad(const uint8_t *const (&img)[4], const float *mean, const float *var,
                                              float *out4, int64_t p0, float k0, SlmStage &st, const float *fg,
                                              InputCheck chk)
{
    const int lane = static_cast<int>(threadIdx.x & 63);
    const f32x4 *mp = reinterpret_cast<const f32x4 *>(mean + 3 * p0);
    const f32x4 *vp = reinterpret_cast<const f32x4 *>(var + 3 * p0);
    f32x4 m[3], v[3];
    uint32_t w[4][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        m[r] = __builtin_nontemporal_load(mp + lane + 64 * r);
        v[r] = __builtin_nontemporal_load(vp + lane + 64 * r);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const uint32_t *ip = reinterpret_cast<const uint32_t *>(img[f] + 3 * p0);
#pragma unroll
        for (int r = 0; r < 3; ++r) w[f][r] = __builtin_nontemporal_load(ip + lane + 64 * r);
    }
    if (chk.flags) report_wave(chk, vec_invalid(m[0], v[0]) | vec_invalid(m[1], v[1]) | vec_invalid(m[2], v[2]));
    Quad q;
    uint32_t qw[4][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = m[r];
        st.w[lane + 64 * r] = w[0][r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q.m[r] = st.f[3 * lane + r];
        qw[0][r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        st.f[lane + 64 * r] = v[r];
        st.w[lane + 64 * r] = w[1][r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q.v[r] = st.f[3 * lane + r];
        qw[1][r] = st.w[3 * lane + r];
    }
#pragma unroll
    for (int f = 2; f < 4; ++f) {
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 3; ++r) st.w[lane + 64 * r] = w[f][r];
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 3; ++r) qw[f][r] = st.w[3 * lane + r];
    }
    wave_lds_sync();
    f32x4 res[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int r = 0; r < 3; ++r) q.w[r] = qw[f][r];
        res[f] = quad_log2slm(q, quad_k0(q, k0, fg));
    }
    // Regroup through LDS so that each store instruction of the wave writes
    // one contiguous kilobyte (64 lanes x one pixel's four frames): pixel e of
    // the wave (entry e of the stage) goes out from lane e % 64.
    st.f[4 * lane + 0] = f32x4{res[0].x, res[1].x, res[2].x, res[3].x};
    st.f[4 * lane + 1] = f32x4{res[0].y, res[1].y, res[2].y, res[3].y};
    st.f[4 * lane + 2] = f32x4{res[0].z, res[1].z, res[2].z, res[3].z};
    st.f[4 * lane + 3] = f32x4{res[0].w, res[1].w, res[2].w, res[3].w};
    wave_lds_sync();
    f32x4 *o = reinterpret_cast<f32x4 *>(out4 + 4 * p0);
#pragma unroll
    for (int s = 0; s < 4; ++s) o[64 * s + lane] = st.f[64 * s + lane];
}

// slm_wave_tail for four frames.
__device__ __forceinline__ void slm_wave_quad_tail(const uint8_t *const (&img)[4], const float *mean,
                                                   const float *var, float *out4, int64_t p0, int64_t npix, float k0,
                                                   const float *fg, InputCheck chk)
{
    const int64_t p = p0 + 4 * static_cast<int64_t>(threadIdx.x & 63);
    if (chk.flags) tail_check(mean, var, p, npix, chk);
    for (int64_t t = p; t < p + 4 && t < npix; ++t) {
        const float *mm = mean + 3 * t, *vv = var + 3 * t;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const uint8_t *I = img[f] + 3 * t;
            const float kt = fg ? k0 - fg[colour_bin(I[0], I[1], I[2])] : k0;
            out4[4 * t + f] = log2slm(I[0], I[1], I[2], mm[0], mm[1], mm[2], vv[0], vv[1], vv[2], kt);
        }
    }
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

// Tile t of an ntx x nty x nzc tile grid taken octant by octant: the grid is
// halved along each axis (first halves rounded up), the eight octants follow
// one another, and an octant of more than kOctantLeaf tiles is split the same
// way again; the tiles of a leaf block run z-major. With contiguous per-XCD
// tile ranges (xcd_remap, the pipelined launches), an XCD works on one
// compact block of the grid (one octant when the tile count splits evenly),
// and the workgroups it runs at a time on a few neighbouring leaf blocks, whose
// projections cover smaller image areas than a z-slab of the block. (At 256^3
// voxels x 12 views of 1280x720, four frames per launch, splitting octants
// down to 256 tiles took a launch from 582 to 519 us; one level serves the
// 128^3 grid's 2048 tiles.) A bijection for every grid shape (empty octants
// are skipped).
constexpr uint32_t kOctantLeaf = 256;

__device__ __forceinline__ void octant_tile(uint32_t t, uint32_t ntx, uint32_t nty, uint32_t nzc, uint32_t &txi,
                                            uint32_t &tyi, uint32_t &zc)
{
    uint32_t bx = 0, by = 0, bz = 0, sx = ntx, sy = nty, sz = nzc;
    do {
        const uint32_t hx = (sx + 1) / 2, hy = (sy + 1) / 2, hz = (sz + 1) / 2;
        uint32_t o = 0, cx = hx, cy = hy, cz = hz;
        for (; o < 8; ++o) {
            cx = (o & 1) ? sx - hx : hx;
            cy = (o & 2) ? sy - hy : hy;
            cz = (o & 4) ? sz - hz : hz;
            const uint32_t cnt = cx * cy * cz;
            if (t < cnt) break;
            t -= cnt;
        }
        bx += (o & 1) ? hx : 0;
        by += (o & 2) ? hy : 0;
        bz += (o & 4) ? hz : 0;
        sx = cx;
        sy = cy;
        sz = cz;
    } while (sx * sy * sz > kOctantLeaf);
    const uint32_t plane = sx * sy;
    const uint32_t lz = t / plane, r = t - lz * plane;
    const uint32_t ly = r / sx, lx = r - ly * sx;
    txi = bx + lx;
    tyi = by + ly;
    zc = bz + lz;
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

// Buffer resource over one view's likelihood map (gfx9 descriptor: raw,
// no stride, bounds-checked against num_records bytes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t map_rsrc(const float *map, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(map), static_cast<short>(0), static_cast<int>(bytes),
                                             0x00020000);
}

// One float of a map; 0 when the byte offset is at or past num_records.
__device__ __forceinline__ float map_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
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

// Bit v of the result is set when every voxel centre of this wave's box
// [i_lo,i_hi] x [j_lo,j_hi] x [k_lo,k_hi] (phantom lanes past the grid edge
// included) projects in view v with depth > 0 to a point at least 1/64 px
// inside the image, in nearest-pixel coordinates u + 1/2, v + 1/2 (the P rows
// are pre-offset). Perspective projection maps the box into the convex hull of
// its projected corners, and the FP32 error of a lane's projection (~1e-4 px)
// is far below the margin, so such a view needs no per-voxel bounds test.
// Lane l tests corner (l & 7) of view (l >> 3) + 8*pass; n <= 16 views.
template <class Views>
__device__ __forceinline__ uint32_t wave_inside_mask(const Views &views, int n, const GridDesc &a, int i_lo,
                                                     int i_hi, int j_lo, int j_hi, int k_lo, int k_hi)
{
    constexpr float kMargin = 1.0f / 64.0f;
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int corner = lane & 7;
    const float X = a.ox + a.h * (static_cast<float>((corner & 1) ? i_hi : i_lo) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>((corner & 2) ? j_hi : j_lo) + 0.5f);
    const float Z = a.oz + a.h * (static_cast<float>((corner & 4) ? k_hi : k_lo) + 0.5f);
    uint32_t mask = 0;
    for (int pass = 0; pass * 8 < n; ++pass) {
        const int v = pass * 8 + (lane >> 3);
        bool ok = true;
        if (v < n) {
            const ViewGeom &g = views(v);
            const float c = fmaf(g.P[10], Z, fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11])));
            const float rc = __builtin_amdgcn_rcpf(c);      // ~1 ulp: far inside the margin
            const float u = fmaf(g.P[2], Z, fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]))) * rc;
            const float w = fmaf(g.P[6], Z, fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]))) * rc;
            ok = c > 0.0f && u >= kMargin && u <= static_cast<float>(g.W) - kMargin && w >= kMargin &&
                 w <= static_cast<float>(g.H) - kMargin;
        }
        const uint64_t bad = __ballot(!ok);
        for (int q = 0; q < 8; ++q) {
            const int vv = pass * 8 + q;
            if (vv < n && ((bad >> (8 * q)) & 0xffull) == 0) mask |= 1u << vv;
        }
    }
    return mask;
}

// Eq. 3-9 for one lane's column segment of KZ voxels, (i, j, k0..k0+KZ-1):
// for every view in order k = 0..n-1, project the voxel centre, read the view's
// log(2*SLM) at the nearest pixel (or bilinearly) and add it to the logit;
// then posterior = sigmoid(logit) and occupancy = posterior > tau. The view
// order is fixed and the fast and checked nearest paths pick the same pixel,
// so every lane layout and work decomposition produces the same bits.
// views(v) returns the ViewGeom of view v (P pre-offset by half of row 2 for
// nearest sampling). The lanes of a wave form a TX x (64/TX) slab of columns.
template <int TX, int KZ, int SAMPLING, class Views>
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
        const int lane = static_cast<int>(threadIdx.x & 63);
        const int i_lo = i - (lane % TX), j_lo = j - (lane / TX);
        const uint32_t inside = wave_inside_mask(views, n, a, i_lo, i_lo + TX - 1, j_lo, j_lo + 64 / TX - 1, k0,
                                                 k0 + KZ - 1);
        // Software pipeline over the views: the byte offsets of view v are
        // computed and its KZ gathers issued before the values of view v-1
        // are added, so every wave keeps one view's gathers in flight while
        // it does the next view's arithmetic (adds stay in view order).
        // Gathers are raw buffer loads from the view's map (32-bit offsets,
        // W*H < 2^30): a voxel-view outside its image gets an offset past the
        // end, for which the hardware returns 0, i.e. adds nothing.
        auto offsets = [&](int v, uint32_t (&off)[KZ], __amdgpu_buffer_rsrc_t &rsrc) {
            const ViewGeom &g = views(v);
            const uint32_t W = static_cast<uint32_t>(g.W), H = static_cast<uint32_t>(g.H);
            rsrc = map_rsrc(lmap + g.map_off, W * H * 4u);
            const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
            const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
            const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
            if (inside & (1u << v)) {
                // every lane lands inside the image: truncation is the floor
#pragma unroll
                for (int kk = 0; kk < KZ; ++kk) {
                    const float r = __builtin_amdgcn_rcpf(fmaf(g.P[10], Z[kk], cx));
                    const uint32_t x = static_cast<uint32_t>(fmaf(g.P[2], Z[kk], ax) * r);
                    const uint32_t y = static_cast<uint32_t>(fmaf(g.P[6], Z[kk], bx) * r);
                    off[kk] = (__umul24(y, W) + x) * 4u;
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < KZ; ++kk) {
                    const float c = fmaf(g.P[10], Z[kk], cx);
                    const float r = __builtin_amdgcn_rcpf(c);
                    const int x = static_cast<int>(floorf(fmaf(g.P[2], Z[kk], ax) * r));
                    const int y = static_cast<int>(floorf(fmaf(g.P[6], Z[kk], bx) * r));
                    const bool ok = c > 0.0f && static_cast<uint32_t>(x) < W && static_cast<uint32_t>(y) < H;
                    off[kk] = ok ? (__umul24(static_cast<uint32_t>(y), W) + static_cast<uint32_t>(x)) * 4u
                                 : 0xFFFFFFFFu;
                }
            }
        };
        // Two value sets used in turn (no register copies, which would make
        // the wave wait for the gathers it just issued).
        uint32_t off[KZ];
        __amdgpu_buffer_rsrc_t rsrc;
        float va[KZ], vb[KZ];
        auto gather = [&](float (&val)[KZ]) {
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) val[kk] = map_load(rsrc, off[kk]);
        };
        auto accumulate = [&](const float (&val)[KZ]) {
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) L[kk] += val[kk];
        };
        if (n > 0) {
            offsets(0, off, rsrc);
            gather(va);
            int v = 1;
            for (; v + 1 < n; v += 2) {
                offsets(v, off, rsrc);
                gather(vb);
                accumulate(va);
                offsets(v + 1, off, rsrc);
                gather(va);
                accumulate(vb);
            }
            if (v < n) {
                offsets(v, off, rsrc);
                gather(vb);
                accumulate(va);
                accumulate(vb);
            } else {
                accumulate(va);
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
            const Proj64 p = proj64_column(g, Xd, Yd);
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const double Zd = static_cast<double>(a.oz) + static_cast<double>(a.h) * (k0 + kk + 0.5);
                const double c = fma(p.pz2, Zd, p.cx);
                if (!(c > 0.0)) continue;
                const double r = 1.0 / c;
                const double u = fma(p.pz0, Zd, p.ax) * r;
                const double w = fma(p.pz1, Zd, p.bx) * r;
                const double x0 = floor(u), y0 = floor(w);
                const float fx = static_cast<float>(u - x0), fy = static_cast<float>(w - y0);
                L[kk] += bilinear_sample(map, g.W, g.H, x0, y0, fx, fy);
            }
        }
    }

    if (i >= a.nx || j >= a.ny) return;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    int64_t idx = (static_cast<int64_t>(k0) * a.ny + j) * a.nx + i;
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk, idx += plane) {
        if (k0 + kk < a.nz) {
            const float p = sigmoid_fast(L[kk]);
            post[idx] = p;
            if (occ) occ[idx] = p > tau ? 1 : 0;
        }
    }
}


// Slab position (y * 32 + x in a wave's 32 x 2 columns) of lane l: each group
// of 4 lanes holds 2 x 2 columns. The L1 serves a gather as one access per
// (4-lane group, 64-byte chunk) pair, and 2 x 2 columns share chunks of a
// quad map more often than 4 columns of one row (a CPU model of this workload:
// 44.5 against 48.9 accesses per gather for quad maps, 37.3 against 43.1 for
// pair maps; the four-frame fusion half 4 % faster).
__device__ __forceinline__ int quad_lane_pos(int l) { return (((l >> 1) & 1) << 5) + 2 * (l >> 2) + (l & 1); }

// Eq. 3-9 of fuse_column (nearest sampling) for two frames of one rig at
// once, from pair maps: each voxel-view is projected once and one 8-byte load
// brings both frames' values; each frame's logit adds its values in view
// order, so both posteriors have the bits fuse_column gives each frame alone.
template <int TX, int KZ, class Views>
__device__ __forceinline__ void fuse_column_pair(const Views &views, int n, const float *lmap2, const GridDesc &a,
                                                 int i, int j, int k0, float L0, float tau, float *post_a,
                                                 uint8_t *occ_a, float *post_b, uint8_t *occ_b, float *wave_stage)
{
    const float X = a.ox + a.h * (static_cast<float>(i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(j) + 0.5f);
    float Z[KZ], La[KZ], Lb[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        Z[kk] = a.oz + a.h * (static_cast<float>(k0 + kk) + 0.5f);
        La[kk] = L0;
        Lb[kk] = L0;
    }
    static_assert(TX == 32 && KZ == 4, "lanes hold 2 x 2 columns of a 32 x 2 slab, 4 voxels each");
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int pos = quad_lane_pos(lane);
    const int i_lo = i - (pos % TX), j_lo = j - (pos / TX);
    const uint32_t inside = wave_inside_mask(views, n, a, i_lo, i_lo + TX - 1, j_lo, j_lo + 64 / TX - 1, k0,
                                             k0 + KZ - 1);
    for (int v = 0; v < n; ++v) {
        const ViewGeom &g = views(v);
        const uint32_t W = static_cast<uint32_t>(g.W), H = static_cast<uint32_t>(g.H);
        const float2 *map = reinterpret_cast<const float2 *>(lmap2) + g.map_off;
        const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
        const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
        const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
        float2 val[KZ];
        if (inside & (1u << v)) {
            // every lane lands inside the image: truncation is the floor
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float r = __builtin_amdgcn_rcpf(fmaf(g.P[10], Z[kk], cx));
                const uint32_t x = static_cast<uint32_t>(fmaf(g.P[2], Z[kk], ax) * r);
                const uint32_t y = static_cast<uint32_t>(fmaf(g.P[6], Z[kk], bx) * r);
                val[kk] = map[__umul24(y, W) + x];
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float c = fmaf(g.P[10], Z[kk], cx);
                const float r = __builtin_amdgcn_rcpf(c);
                const int x = static_cast<int>(floorf(fmaf(g.P[2], Z[kk], ax) * r));
                const int y = static_cast<int>(floorf(fmaf(g.P[6], Z[kk], bx) * r));
                const bool ok = c > 0.0f && static_cast<uint32_t>(x) < W && static_cast<uint32_t>(y) < H;
                val[kk] = ok ? map[__umul24(static_cast<uint32_t>(y), W) + static_cast<uint32_t>(x)] : make_float2(0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            La[kk] += val[kk].x;
            Lb[kk] += val[kk].y;
        }
    }
    // A wave whose 32 x 2 x 4 voxels all lie in the grid, with rows that start
    // 16-byte aligned, regroups both frames' outputs through LDS and stores
    // whole 16-byte pieces of rows non-temporally, as fuse_column_quad does.
    bool aligned_rows = (a.nx & 15) == 0;
    for (const void *q : {static_cast<const void *>(post_a), static_cast<const void *>(post_b),
                          static_cast<const void *>(occ_a), static_cast<const void *>(occ_b)})
        aligned_rows = aligned_rows && (reinterpret_cast<uintptr_t>(q) & 15) == 0;
    if (aligned_rows && i_lo + 31 < a.nx && j_lo + 1 < a.ny && k0 + KZ - 1 < a.nz) {
        // stage entry (f * KZ + kk) * 64 + pos: voxel (i_lo + pos % 32, j_lo + pos / 32, k0 + kk), frame f
        uint8_t *stage_b = reinterpret_cast<uint8_t *>(wave_stage + 2 * KZ * 64);
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const float pa = sigmoid_fast(La[kk]), pb = sigmoid_fast(Lb[kk]);
            wave_stage[kk * 64 + pos] = pa;
            wave_stage[(KZ + kk) * 64 + pos] = pb;
            stage_b[kk * 64 + pos] = pa > tau ? 1 : 0;
            stage_b[(KZ + kk) * 64 + pos] = pb > tau ? 1 : 0;
        }
        wave_lds_sync();
        const int r = lane >> 3, c = lane & 7;           // row r = (kk, y) = (r / 2, r % 2), 16-byte piece c
        const int64_t row = (static_cast<int64_t>(k0 + (r >> 1)) * a.ny + j_lo + (r & 1)) * a.nx + i_lo;
        __builtin_nontemporal_store(*reinterpret_cast<const f32x4 *>(wave_stage + (r >> 1) * 64 + (r & 1) * 32 + 4 * c),
                                    reinterpret_cast<f32x4 *>(post_a + row + 4 * c));
        __builtin_nontemporal_store(
            *reinterpret_cast<const f32x4 *>(wave_stage + (KZ + (r >> 1)) * 64 + (r & 1) * 32 + 4 * c),
            reinterpret_cast<f32x4 *>(post_b + row + 4 * c));
        if (lane < 32) {
            // lane l: frame l / 16, row (l / 2) % 8, half l % 2 of the row's 32 bytes
            const int f = lane >> 4, rr = (lane >> 1) & 7, half = lane & 1;
            const int64_t orow = (static_cast<int64_t>(k0 + (rr >> 1)) * a.ny + j_lo + (rr & 1)) * a.nx + i_lo;
            uint8_t *const dst = f == 0 ? occ_a : occ_b;
            if (dst)
                __builtin_nontemporal_store(
                    *reinterpret_cast<const f32x4 *>(stage_b + (f * KZ + (rr >> 1)) * 64 + (rr & 1) * 32 + 16 * half),
                    reinterpret_cast<f32x4 *>(dst + orow + 16 * half));
        }
        return;
    }
    if (i >= a.nx || j >= a.ny) return;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    int64_t idx = (static_cast<int64_t>(k0) * a.ny + j) * a.nx + i;
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk, idx += plane) {
        if (k0 + kk < a.nz) {
            const float pa = sigmoid_fast(La[kk]), pb = sigmoid_fast(Lb[kk]);
            post_a[idx] = pa;
            post_b[idx] = pb;
            if (occ_a) occ_a[idx] = pa > tau ? 1 : 0;
            if (occ_b) occ_b[idx] = pb > tau ? 1 : 0;
        }
    }
}

// Eq. 3-9 of fuse_column (nearest sampling) for four frames of one rig at
// once, from quad maps: one projection and one 16-byte load per voxel-view;
// each frame's logit adds its values in view order, so every posterior has
// the bits fuse_column gives that frame alone. post[f] / occ[f] are frame f's
// outputs (occ[f] nullable).
template <int TX, int KZ, class Views>
__device__ __forceinline__ void fuse_column_quad(const Views &views, int n, const float *lmap4, const GridDesc &a,
                                                 int i, int j, int k0, float L0, float tau, float *const (&post)[4],
                                                 uint8_t *const (&occ)[4], float *wave_stage)
{
    const float X = a.ox + a.h * (static_cast<float>(i) + 0.5f);
    const float Y = a.oy + a.h * (static_cast<float>(j) + 0.5f);
    float Z[KZ], L[KZ][4];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        Z[kk] = a.oz + a.h * (static_cast<float>(k0 + kk) + 0.5f);
#pragma unroll
        for (int f = 0; f < 4; ++f) L[kk][f] = L0;
    }
    static_assert(TX == 32, "lanes hold 2 x 2 columns of a 32 x 2 slab (quad_lane_pos)");
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int pos = quad_lane_pos(lane);
    const int i_lo = i - (pos % TX), j_lo = j - (pos / TX);
    const uint32_t inside = wave_inside_mask(views, n, a, i_lo, i_lo + TX - 1, j_lo, j_lo + 64 / TX - 1, k0,
                                             k0 + KZ - 1);
    for (int v = 0; v < n; ++v) {
        const ViewGeom &g = views(v);
        const uint32_t W = static_cast<uint32_t>(g.W), H = static_cast<uint32_t>(g.H);
        // raw buffer loads with 32-bit byte offsets (the host takes this path
        // only when every view's quad map is below 4 GiB); an offset past
        // the end returns 0, which is what a voxel-view outside its image adds
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(lmap4 + 4 * g.map_off), static_cast<short>(0), static_cast<int>(W * H * 16u), 0x00020000);
        const float ax = fmaf(g.P[0], X, fmaf(g.P[1], Y, g.P[3]));
        const float bx = fmaf(g.P[4], X, fmaf(g.P[5], Y, g.P[7]));
        const float cx = fmaf(g.P[8], X, fmaf(g.P[9], Y, g.P[11]));
        uint32_t off[KZ];
        if (inside & (1u << v)) {
            // every lane lands inside the image: truncation is the floor
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float r = __builtin_amdgcn_rcpf(fmaf(g.P[10], Z[kk], cx));
                const uint32_t x = static_cast<uint32_t>(fmaf(g.P[2], Z[kk], ax) * r);
                const uint32_t y = static_cast<uint32_t>(fmaf(g.P[6], Z[kk], bx) * r);
                off[kk] = (__umul24(y, W) + x) * 16u;
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float c = fmaf(g.P[10], Z[kk], cx);
                const float r = __builtin_amdgcn_rcpf(c);
                const int x = static_cast<int>(floorf(fmaf(g.P[2], Z[kk], ax) * r));
                const int y = static_cast<int>(floorf(fmaf(g.P[6], Z[kk], bx) * r));
                const bool ok = c > 0.0f && static_cast<uint32_t>(x) < W && static_cast<uint32_t>(y) < H;
                off[kk] = ok ? (__umul24(static_cast<uint32_t>(y), W) + static_cast<uint32_t>(x)) * 16u : 0xFFFFFFFFu;
            }
        }
        f32x4 val[KZ];
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk)
            val[kk] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, static_cast<int>(off[kk]), 0, 0));
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            L[kk][0] += val[kk].x;
            L[kk][1] += val[kk].y;
            L[kk][2] += val[kk].z;
            L[kk][3] += val[kk].w;
        }
    }
    // A wave whose 32 x 2 x KZ voxels all lie in the grid, with rows that
    // start 16-byte aligned, regroups its outputs through LDS so that each
    // store instruction writes whole 16-byte pieces of rows (8 rows of 32
    // posteriors, or 4 frames x 8 rows of 32 occupancy bytes): one cache
    // access per 64 bytes, where per-voxel stores cost one per 4 lanes. The
    // stores are non-temporal: the four outputs (20 bytes per voxel) are not
    // read again by this launch and would otherwise take the L2 and MALL room
    // of the quad maps the gathers read (at 256^3 x 12 views: 335 MB of
    // outputs against 177 MB of maps per launch, fusion 374 -> 262 us).
    static_assert(TX != 32 || KZ == 4, "the regrouped stores cover 32 x 2 x 4 voxels");
    bool aligned_rows = TX == 32 && (a.nx & 15) == 0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
        aligned_rows = aligned_rows && (reinterpret_cast<uintptr_t>(post[f]) & 15) == 0 &&
                       (reinterpret_cast<uintptr_t>(occ[f]) & 15) == 0;
    if (aligned_rows && i_lo + 31 < a.nx && j_lo + 1 < a.ny && k0 + KZ - 1 < a.nz) {
        // stage entry (f * KZ + kk) * 64 + pos: voxel (i_lo + pos % 32, j_lo + pos / 32, k0 + kk), frame f
        uint8_t *stage_b = reinterpret_cast<uint8_t *>(wave_stage);
        uint32_t ob[KZ];
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            ob[kk] = 0;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float p = sigmoid_fast(L[kk][f]);
                wave_stage[(f * KZ + kk) * 64 + pos] = p;
                ob[kk] |= (p > tau ? 1u : 0u) << (8 * f);
            }
        }
        wave_lds_sync();
        const int r = lane >> 3, c = lane & 7;           // row r = (kk, y) = (r / 2, r % 2), 16-byte piece c
        const int64_t row = (static_cast<int64_t>(k0 + (r >> 1)) * a.ny + j_lo + (r & 1)) * a.nx + i_lo;
#pragma unroll
        for (int f = 0; f < 4; ++f)
            __builtin_nontemporal_store(
                *reinterpret_cast<const f32x4 *>(wave_stage + (f * KZ + (r >> 1)) * 64 + (r & 1) * 32 + 4 * c),
                reinterpret_cast<f32x4 *>(post[f] + row + 4 * c));
        wave_lds_sync();
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk)
#pragma unroll
            for (int f = 0; f < 4; ++f) stage_b[(f * KZ + kk) * 64 + pos] = static_cast<uint8_t>(ob[kk] >> (8 * f));
        wave_lds_sync();
        {
            // lane l: frame l / 16, row (l / 2) % 8, half l % 2 of the row's 32 bytes
            const int f = lane >> 4, rr = (lane >> 1) & 7, half = lane & 1;
            const int64_t orow = (static_cast<int64_t>(k0 + (rr >> 1)) * a.ny + j_lo + (rr & 1)) * a.nx + i_lo;
            uint8_t *const dst = f == 0 ? occ[0] : f == 1 ? occ[1] : f == 2 ? occ[2] : occ[3];
            if (dst)
                __builtin_nontemporal_store(
                    *reinterpret_cast<const f32x4 *>(stage_b + (f * KZ + (rr >> 1)) * 64 + (rr & 1) * 32 + 16 * half),
                    reinterpret_cast<f32x4 *>(dst + orow + 16 * half));
        }
        return;
    }
    if (i >= a.nx || j >= a.ny) return;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    int64_t idx = (static_cast<int64_t>(k0) * a.ny + j) * a.nx + i;
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk, idx += plane) {
        if (k0 + kk < a.nz) {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float p = sigmoid_fast(L[kk][f]);
                post[f][idx] = p;
                if (occ[f]) occ[f][idx] = p > tau ? 1 : 0;
            }
        }
    }
}

}  // namespace dev
}  // namespace psfs
