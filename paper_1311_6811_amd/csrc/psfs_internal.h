// Internal declarations shared by the host API and the kernels of libpsfs.
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "psfs.h"

namespace psfs {

constexpr int kMaxViews = PSFS_MAX_VIEWS;
constexpr int kMapAlignFloats = 64;     // per-view likelihood-map offset alignment
constexpr int kNumXcd = 8;              // MI355X: 8 accelerator complex dies, 32 CUs each

// One view's inputs to the likelihood-map kernel (Eq. 1-2).
struct SlmView {
    const uint8_t *img;                 // [npix][3] u8
    const float *mean;                  // [npix][3]
    const float *var;                   // [npix][3]
    int64_t npix;
    int64_t map_off;                    // float offset of this view's map
};

struct SlmArgs {
    SlmView view[kMaxViews];
    float *lmap;
    const float *fg;                    // nullable: log density per colour bin of a learned foreground model
    uint32_t *check;                    // nullable: bit k set when view k's background holds an invalid value
    float k0;                           // -1.5*log(2*pi) - log_u; -1.5*log(2*pi) with fg
    int32_t n;
};

// Learned foreground colour model: histogram of the marked pixels of all
// views, then the log density per colour bin.
struct FgArgs {
    SlmView view[kMaxViews];            // img, npix and map_off are used
    const uint8_t *mask[kMaxViews];     // nullable per view: nonzero = foreground; else lmap > 0
    const float *lmap;
    uint32_t *counts;                   // [4096]
    float *logd;                        // [4096]
    int32_t n;
};

// One view as the fusion kernels see it (Eq. 3-9). For nearest sampling the
// host adds half of row 2 to rows 0 and 1, so floor(row0.X / row2.X) is the
// nearest pixel floor(u + 1/2).
struct ViewGeom {
    float P[12];
    int32_t W, H;
    int64_t map_off;
};

struct GridDesc {
    int nx, ny, nz;
    float ox, oy, oz, h;                // grid origin (corner) and voxel edge
};

struct FuseArgs {
    ViewGeom view[kMaxViews];
    const float *lmap;
    float *post;
    uint8_t *occ;                       // nullable
    int32_t n, nx, ny, nz;
    float ox, oy, oz, h;                // grid origin (corner) and voxel edge
    float L0;                           // logit(prior)
    float tau;                          // threshold on the posterior
};

// Frame B's images of a two-frame pass (frame A's travel in SlmArgs).
struct PairImages {
    const uint8_t *img[kMaxViews];
};

// Frames B, C and D of a four-frame pass (frame A's travel in SlmArgs).
struct QuadImages {
    const uint8_t *img[3][kMaxViews];
};

// Outputs of frames B, C and D of a four-frame pass (frame A's travel in
// FuseArgs); occ entries are nullable.
struct QuadOut {
    float *post[3];
    uint8_t *occ[3];
};

// Shape of the pipelined launch (likelihood of the next frame + fusion of
// the current one).
struct PipeArgs {
    int32_t slm_per_view;               // likelihood workgroups per view
    int32_t slm_rounds;                 // ceil(views * slm_per_view / kNumXcd)
    int32_t fuse_rounds;                // ceil(fuse_tiles / kNumXcd)
    int64_t fuse_tiles;
};

// Differentiable variant: bilinear logits, BCE loss and adjoint (one view
// geometry per view with the raw camera matrix).
struct DiffArgs {
    ViewGeom view[kMaxViews];
    double Pd[kMaxViews][12];           // each view's camera matrix widened to FP64 (the FP64 projection's operands)
    const float *lmap;                  // log(2*SLM) maps
    float *adj;                         // adjoint maps dLoss/dlog(2*SLM), int64 fixed point, same element layout
    const uint8_t *labels;              // [nz][ny][nx] 0/1
    float *logits;                      // [nz][ny][nx]
    const float *grad_loss;             // device scalar (backward)
    double *loss_part;                  // one partial sum per forward workgroup
    float *cam_part;                    // [backward workgroup][n][12] partial camera gradients
    int32_t n, nx, ny, nz;
    float ox, oy, oz, h;
    float L0;                           // logit(prior)
    float inv_count;                    // 1 / |loss region| (0 for an empty region)
    int32_t sub[6];                     // loss region [i0,i1) x [j0,j1) x [k0,k1)
};

// Pixel chain: adjoint maps -> gradients of the background means/variances.
struct ChainView {
    const uint8_t *img;
    const float *mean;
    const float *var;
    float *gmean;
    float *gvar;
    int64_t npix;
    int64_t map_off;
};

struct ChainArgs {
    ChainView view[kMaxViews];
    const float *adj;                   // int64 fixed-point adjoint maps (see diff.hip)
    const float *grad_loss;
    const float *cam_part;              // [cam_parts][n][12] partial camera gradients of the backward workgroups
    int64_t cam_parts;
    float *gP;                          // [n][12] camera-matrix gradients
    float inv_count;
    float k0;
    int32_t n;
};

// Batched pass: one device descriptor table of views and frames.
struct BatchView {
    ViewGeom g;                         // map_off indexes the batch's map arena
    const uint8_t *img;
    const float *mean;
    const float *var;
    int64_t npix;
};

struct BatchFrame {
    GridDesc grid;
    int32_t n, view0;                   // views [view0, view0 + n) of the table
    float *post;
    uint8_t *occ;                       // nullable
};

struct BatchArgs {
    const BatchView *views;
    const BatchFrame *frames;           // table order = launch-chain order
    float *lmap;                        // map arena
    float k0, L0, tau;
};

// Smoothing, threshold and surface extraction of one posterior grid.
struct SurfArgs {
    const float *post;                  // [nz][ny][nx]
    float *smoothed;                    // nullable, [nz][ny][nx]
    uint8_t *occ;                       // [nz][ny][nx]
    int32_t *out;                       // ascending surface indices, first `capacity`
    int64_t capacity;
    int64_t *count;                     // device: number of surface voxels
    int32_t *counts;                    // workspace: per-block surface counts
    uint8_t *flags;                     // workspace: surface flag per voxel
    int64_t nvox;
    int32_t nblocks;
    int32_t nx, ny, nz;
    int32_t step_i, step_j, step_k;     // 256 voxels as (256 % nx, (256 / nx) % ny, 256 / (nx*ny))
    float tau;
};

// Voxel colouring of a list of voxels (depth-buffer visibility).
struct ColourArgs {
    ViewGeom view[kMaxViews];           // nearest-pixel P (pre-offset), W, H; map_off = offset in zbuf
    const uint8_t *img[kMaxViews];      // [H][W][3]
    const int32_t *list;                // linear voxel indices
    int64_t nlist;
    unsigned long long *zbuf;           // workspace: (depth bits << 32 | position) per pixel
    int64_t zbuf_len;
    float *colour;                      // [nlist][3]: mean RGB over the views that see the voxel
    int32_t *views;                     // [nlist]: number of views that see the voxel
    int64_t nvox;
    int32_t n, nx, ny;
    float ox, oy, oz, h;
};

struct TileCfg {
    int tx, ty, kz;                     // x-by-y lanes per workgroup, z voxels per lane
};

int tile_count();
const TileCfg &tile_cfg(int tile);
int default_tile();

hipError_t launch_slm(const SlmArgs &a, int64_t max_npix, hipStream_t s);
hipError_t launch_fuse(const FuseArgs &a, int tile, int sampling, hipStream_t s);
// sa.n == 0: no likelihood part; fa.post == nullptr: no fusion part.
hipError_t launch_pipeline(const SlmArgs &sa, const FuseArgs &fa, int tile, int sampling, int64_t max_npix,
                           hipStream_t s);
// Two frames of one rig per launch (nearest sampling, tile 8x32x4): pair maps
// of the next two frames (sa: frame A's images and the shared background, ib:
// frame B's images, sa.lmap: pair-map buffer) beside the fusion of the
// current pair (fa.lmap: pair maps; fa.post/occ: frame A; post_b/occ_b: B).
hipError_t launch_pipeline_pair(const SlmArgs &sa, const PairImages &ib, const FuseArgs &fa, float *post_b,
                                uint8_t *occ_b, int64_t max_npix, hipStream_t s);
// Four frames of one rig per launch (nearest sampling, tile 32x8x4), as
// launch_pipeline_pair with quad maps (four floats per pixel, frame-minor) and
// frames B-D in qi / qo.
hipError_t launch_pipeline_quad(const SlmArgs &sa, const QuadImages &qi, const FuseArgs &fa, const QuadOut &qo,
                                int64_t max_npix, hipStream_t s);
int64_t diff_fwd_blocks(int nx, int ny, int nz);
int64_t diff_bwd_blocks(int nx, int ny, int nz);
hipError_t launch_diff_forward(const DiffArgs &a, float *loss, hipStream_t s);
hipError_t launch_diff_backward(const DiffArgs &a, const ChainArgs &c, int64_t map_floats, int64_t max_npix,
                                float *gP, hipStream_t s);
// Batch: likelihood workgroups per view for views of up to max_npix pixels;
// fusion bricks of a frame for a tile; whether a tile runs the pipelined
// launches (256 lanes) or separate ones; one step of the launch chain (the
// likelihood of table frame fl beside the fusion of table frame ff, either
// of them -1 for none).
int64_t batch_slm_blocks_per_view(int64_t max_npix);
int64_t batch_bricks(int nx, int ny, int nz, int tile);
bool batch_pipelined_tile(int tile);
hipError_t launch_batch_step(const BatchArgs &a, int tile, int sampling, int fl, int64_t slm_per_view, int nviews_l,
                             int ff, int64_t fuse_tiles, hipStream_t s);
hipError_t launch_threshold(const float *post, int64_t n, float tau, uint8_t *occ, hipStream_t s);
int64_t surface_blocks(int64_t nvox);
hipError_t launch_colour(const ColourArgs &a, hipStream_t s);
hipError_t launch_foreground(const FgArgs &a, int64_t max_npix, hipStream_t s);
hipError_t launch_surface(const SurfArgs &a, hipStream_t s);   // a.nvox == 0: writes count 0 only

}  // namespace psfs
