// Internal interface of the particle-weight kernels (annealed particle
// filter, Sec. 2.3.1-2.3.2, Eq. 10 and 14-16). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "psfs.h"

namespace psfs {

constexpr int kPartViews = PSFS_MAX_VIEWS;
constexpr int kCylinders = PSFS_CYLINDERS;        // body-model cylinders per particle
constexpr int kSections = 8;                       // cross-sections sampled per cylinder
constexpr int kCylFloats = 8;                      // A xyz, B xyz, rA, rB

struct PartView {
    const float *sil;                   // [h][w] silhouette map
    const float *edge;                  // [h][w] edge map
    int32_t w, h;
    float P[12];                        // row-major 3x4 projection
};

// Weights: one workgroup per particle, one wave per view.
struct PartArgs {
    PartView view[kPartViews];
    const float *cyl;                   // [np][kCylinders][kCylFloats], 16-byte aligned
    double *logw;                       // [np]
    double *terms;                      // nullable [np][n][2]: Sigma_e, Sigma_r per view
    int64_t np;
    int32_t n;
};

// Normalisation over the particles (Eq. 10) with the annealing exponent beta.
struct NormArgs {
    const double *logw;
    double *weights;
    int64_t np;
    double beta;
};

hipError_t launch_particle_weights(const PartArgs &a, hipStream_t s);
hipError_t launch_particle_normalise(const NormArgs &a, hipStream_t s);

}  // namespace psfs
