/*
 * psfs.h -- C ABI of the MI355X (gfx950) probabilistic shape-from-silhouette
 * occupancy library.
 *
 * The method (Song, Bian et al., "Digitize Your Body and Action in 3-D at Over
 * 10 FPS", Sec. 2.2.2):
 *   - Eq. 1-2: every pixel of every view gets a silhouette likelihood
 *     SLM = P(F=1 | I) from a per-pixel single-Gaussian background model
 *     N(I | mu, var) against a uniform foreground density u, with equal priors.
 *   - Eq. 3-9: every voxel of a regular grid gets the occupancy posterior
 *     P(V=1 | {S}) by fusing, over the views, the SLM value at the pixel its
 *     centre projects to, with a latent occluder summed out. Summed out with
 *     P(O)=1/2, Eq. 5-9 say that each view that sees the voxel multiplies the
 *     prior odds by 2*SLM; the library evaluates exactly that, in FP32 in the
 *     log domain: logit P = logit(prior) + sum_k log(2*SLM_k).
 *   - Sec. 2.2.2 (last step): the posterior is thresholded to an occupancy grid.
 *
 * Conventions (all functions):
 *   - Memory: the caller owns every device buffer and the stream. The library
 *     copies host structs, borrows device pointers until the enqueued work has
 *     passed on the stream, and allocates no device memory except inside a
 *     batch object (its device descriptor table, see psfs_batch_create).
 *     Scratch lives in a caller-provided workspace whose size the library
 *     reports.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream). Every compute call is asynchronous; faults surface at the
 *     caller's synchronisation. A plan holds no device state: cameras, grid,
 *     parameters and buffer addresses are copied into each launch's
 *     arguments, so one plan may feed work on several streams at once (each
 *     with its own workspace and outputs), and changing its settings after a
 *     call does not change work already enqueued. Calls can be captured into
 *     HIP graphs: no call records a memset.
 *   - Errors: every `int` function returns a psfs_status. Arguments are
 *     validated before anything is enqueued; on an error nothing is enqueued
 *     and psfs_last_error() holds a thread-local message. HIP runtime failures
 *     return PSFS_E_HIP. No C++ exception crosses this ABI.
 *   - Threads: a plan or batch is not thread-safe; distinct ones are.
 *   - Layouts: images are u8 RGB [H][W][3]; background mean and variance are
 *     FP32 [H][W][3]; a camera matrix P is FP32 row-major 3x4 mapping world
 *     metres (homogeneous) to pixels, with pixel centres at integer
 *     coordinates; voxel grids are [nz][ny][nx] with x fastest and voxel
 *     (i,j,k) centred at origin + voxel * (i+1/2, j+1/2, k+1/2).
 *   - Alignment: mean, var, likelihood-map and posterior pointers must be
 *     16-byte aligned, image pointers 4-byte aligned (PSFS_E_ARG otherwise).
 */
#ifndef PSFS_H
#define PSFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSFS_VERSION 1
#define PSFS_MAX_VIEWS 16
#define PSFS_FG_BINS 4096       /* colour bins of the learned foreground model */

enum psfs_status {
    PSFS_OK = 0,
    PSFS_E_ARG = -1,        /* null/misaligned pointer, bad enum value */
    PSFS_E_RANGE = -2,      /* a size or value outside its documented range */
    PSFS_E_NOT_READY = -3,  /* cameras, grid or a background not set yet */
    PSFS_E_WORKSPACE = -4,  /* workspace missing or smaller than required */
    PSFS_E_HIP = -5,        /* HIP runtime error; text in psfs_last_error() */
    PSFS_E_DEVICE = -6,     /* the current device is not a gfx950 GPU */
    PSFS_E_STALE = -7,      /* batch update changes the captured shapes */
    PSFS_E_INPUT = -8       /* invalid input values found by the optional device
                               check (psfs_set_input_check / psfs_input_status) */
};

enum psfs_sampling {
    PSFS_NEAREST = 0,       /* pixel x = floor(u + 1/2), y = floor(v + 1/2) (Eq. 3-9) */
    PSFS_BILINEAR = 1       /* log(2*SLM) interpolated from taps floor(u)+{0,1},
                               floor(v)+{0,1}; taps outside the image count 0 */
};

/* One view: image size and the 3x4 projection (u*c, v*c, c) = P [X; 1].
 * A voxel is seen by the view when c > 0 and its pixel lies in the image. */
typedef struct psfs_camera {
    int32_t width, height;  /* 1..65535 each, width*height < 2^30 (byte offsets
                               into one map fit in 32 bits) */
    float P[12];            /* row-major 3x4, finite */
} psfs_camera;

/* Regular voxel grid; any dimension may be 0 (an empty grid: calls are no-ops).
 * nx*ny*nz < 2^31. */
typedef struct psfs_grid {
    int32_t nx, ny, nz;
    float origin[3];        /* corner of voxel (0,0,0), metres */
    float voxel;            /* edge length, > 0 */
} psfs_grid;

/* Model parameters (defaults from psfs_default_params):
 *   prior      P(V=1) in Eq. 3, in (0,1); default 1/2
 *   log_u      log of the uniform foreground density of Eq. 1; default
 *              -3*ln(256) (uniform over the 8-bit RGB cube); finite
 *   threshold  occupancy = (posterior > threshold), in [0,1]; default 1/2
 *   sampling   psfs_sampling used by psfs_fuse/psfs_reconstruct */
typedef struct psfs_params {
    float prior;
    float log_u;
    float threshold;
    int32_t sampling;
} psfs_params;

typedef struct psfs_plan psfs_plan;     /* opaque, host-only */

int psfs_version(void);
const char *psfs_status_str(int status);
/* Thread-local text of the last failing call on this thread ("" if none). */
const char *psfs_last_error(void);
void psfs_default_params(psfs_params *out);

/* ---------------------------------------------------------------- plans */

int psfs_plan_create(psfs_plan **out);
void psfs_plan_destroy(psfs_plan *plan);                 /* NULL-safe */

/* Copies n (0..PSFS_MAX_VIEWS) cameras. Forgets every background set before. */
int psfs_set_cameras(psfs_plan *plan, int n, const psfs_camera *cams);
int psfs_set_grid(psfs_plan *plan, const psfs_grid *grid);
int psfs_set_params(psfs_plan *plan, const psfs_params *params);
/* Background model of view `view` (Eq. 1): borrowed device pointers to FP32
 * [H][W][3] means and variances (variances > 0 and finite, means finite;
 * checked on the device only when the input check below is on). The caller
 * keeps them alive while work that reads them runs. */
int psfs_set_background(psfs_plan *plan, int view, const float *mean_dev, const float *var_dev);

/* Optional device check of the background model (Eq. 1 is defined only for
 * positive finite variances). flags_dev: a caller-owned, 4-byte aligned device
 * word, zero before the first checked call (NULL turns the check off, the
 * default). While it is set, every likelihood pass of this plan
 * (psfs_likelihood, psfs_reconstruct, the pipelined steps, psfs_diff_forward)
 * also tests each mean (finite) and variance (positive and finite) it reads
 * and sets bit k of *flags_dev when view k holds an invalid value; the maps
 * and posteriors it writes are then meaningless (NaN or infinite values), but
 * no kernel faults. Batches are not checked. */
int psfs_set_input_check(psfs_plan *plan, uint32_t *flags_dev);
/* After the caller has synchronised with the checked work: reads the flags
 * (a blocking 4-byte copy). Returns PSFS_OK if no invalid value was seen, else
 * clears the word and returns PSFS_E_INPUT with the views named in
 * psfs_last_error(); PSFS_E_NOT_READY if no flags are set. */
int psfs_input_status(psfs_plan *plan);

/* Likelihood-map layout: view k occupies floats [offset(k), offset(k) + W_k*H_k)
 * of one buffer, offsets padded to multiples of 64 floats. Returns the total
 * number of floats / the offset of view k, or a negative psfs_status. */
int64_t psfs_lmap_floats(const psfs_plan *plan);
int64_t psfs_lmap_offset(const psfs_plan *plan, int view);

/* Workspace of psfs_reconstruct: the likelihood maps. 0 if cameras unset. */
size_t psfs_workspace_bytes(const psfs_plan *plan);

/* ------------------------------------------------------- forward pass */

/* Eq. 1-2 for every view: lmap[offset(k) + y*W_k + x] = log(2*SLM) of pixel
 * (x, y) of view k, FP32. images_dev: host array of n device pointers. */
int psfs_likelihood(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap_dev,
                    void *stream);

/* Eq. 3-9 from likelihood maps in the psfs_lmap_* layout: posterior FP32
 * [nz][ny][nx]; occ (nullable) u8 [nz][ny][nx] = posterior > threshold.
 * Sampling per params (nearest by default; bilinear gives the posterior of the
 * differentiable variant). */
int psfs_fuse(psfs_plan *plan, const float *lmap_dev, float *posterior_dev, uint8_t *occ_dev,
              void *stream);

/* psfs_likelihood into the workspace, then psfs_fuse. */
int psfs_reconstruct(psfs_plan *plan, const uint8_t *const *images_dev, float *posterior_dev,
                     uint8_t *occ_dev, void *workspace_dev, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as psfs_reconstruct, bit for bit, with the likelihood maps in a
 * static device array of the library instead of a workspace argument. The
 * array holds PSFS_STATIC_SCRATCH_BYTES on every GPU the library runs this
 * call on, from the first call on that GPU until the process ends; the call
 * itself allocates nothing. Plans whose maps need more
 * (psfs_workspace_bytes > PSFS_STATIC_SCRATCH_BYTES) get PSFS_E_RANGE before
 * anything is enqueued. All calls on one GPU share its array: two calls whose
 * work overlaps on that GPU (different streams, or graph replays running
 * concurrently) race on the maps; calls ordered on one stream do not. */
#define PSFS_STATIC_SCRATCH_BYTES (48u << 20)
int psfs_reconstruct_static(psfs_plan *plan, const uint8_t *const *images_dev, float *posterior_dev,
                            uint8_t *occ_dev, void *stream);

/* One step of a frame sequence seen by one rig, as one launch: the
 * likelihood maps of the next frame (Eq. 1-2, as psfs_likelihood of
 * images_dev into lmap_next_dev) and the fusion of the current frame (Eq. 3-9,
 * as psfs_fuse of lmap_cur_dev into posterior_dev / occ_dev), the two parts
 * running side by side on the GPU. Frame t's maps come from step t-1, so with
 * two map buffers used in turn a sequence costs one launch per frame (the
 * paper overlaps transfers, CPU work and kernels through several command
 * queues, Sec. 3.3.2; here the overlap is inside one launch).
 *   images_dev      n device pointers of the next frame, or NULL: no
 *                   likelihood part (backgrounds must be set otherwise)
 *   lmap_next_dev   psfs_lmap_floats floats, 16-byte aligned (unused if
 *                   images_dev is NULL)
 *   lmap_cur_dev    maps of the current frame in the same layout, written by
 *                   an earlier call; must not overlap lmap_next_dev
 *   posterior_dev   FP32 [nz][ny][nx] of the current frame, or NULL: no fusion
 *                   part (then occ_dev must be NULL too)
 *   occ_dev         nullable u8 [nz][ny][nx]
 * Results are bit-identical to psfs_likelihood and psfs_fuse. Both parts NULL
 * is a no-op. Cameras and grid must be set (PSFS_E_NOT_READY). */
int psfs_pipeline_step(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap_next_dev,
                       const float *lmap_cur_dev, float *posterior_dev, uint8_t *occ_dev, void *stream);

/* The same step for two frames of the sequence at once (frames A and B, e.g.
 * t and t+1), which share the rig and the background model: one launch
 * computes the pair maps of the next two frames beside the fusion of the
 * current two. Pair maps interleave the two frames' maps: the value of pixel p
 * of view k is at float 2 * (psfs_lmap_offset(k) + p) for frame A and the next
 * float for frame B (2 * psfs_lmap_floats floats per buffer). Each voxel-view
 * is projected once for both frames and the background model is read once for
 * both, so a pair costs less than two single steps; every result is
 * bit-identical to psfs_likelihood and psfs_fuse of each frame alone.
 * Nearest sampling only (PSFS_E_ARG otherwise); the fixed tile is 8x32 lanes x
 * 4 voxels per lane.
 *   images_a_dev, images_b_dev  n device pointers each of the next two frames,
 *                   or both NULL: no likelihood part
 *   lmap2_next_dev  pair maps written by this step, 16-byte aligned
 *   lmap2_cur_dev   pair maps of the current two frames, from an earlier call;
 *                   must not overlap lmap2_next_dev
 *   posterior_a_dev, posterior_b_dev  FP32 [nz][ny][nx] of the current two
 *                   frames, 16-byte aligned, or both NULL: no fusion part
 *   occ_a_dev, occ_b_dev  nullable u8 [nz][ny][nx] (NULL without posteriors)
 * Both parts absent is a no-op. Cameras and grid must be set
 * (PSFS_E_NOT_READY), and the backgrounds for the likelihood part. */
int psfs_pipeline_step_pair(psfs_plan *plan, const uint8_t *const *images_a_dev,
                            const uint8_t *const *images_b_dev, float *lmap2_next_dev,
                            const float *lmap2_cur_dev, float *posterior_a_dev, uint8_t *occ_a_dev,
                            float *posterior_b_dev, uint8_t *occ_b_dev, void *stream);

/* The same step for four frames of the sequence at once (frames 0-3, e.g.
 * t .. t+3), which share the rig and the background model. Quad maps
 * interleave the four frames' maps: the value of pixel p of view k for frame f
 * is at float 4 * (psfs_lmap_offset(k) + p) + f (4 * psfs_lmap_floats floats
 * per buffer). Each voxel-view is projected once and gathered with one
 * 16-byte load for the four frames, and the background model is read once for
 * the four; every result is bit-identical to psfs_likelihood and psfs_fuse of
 * each frame alone (Eq. 1-2 per pixel, Eq. 3-9 per voxel, Sec. 2.2.2).
 * Nearest sampling only (PSFS_E_ARG otherwise), and every view's image below
 * 2^28 pixels (PSFS_E_RANGE otherwise); the fixed tile is 32x8 lanes x 4
 * voxels per lane.
 *   images_dev      host array of 4*n device pointers, frame-major (frame f,
 *                   view k at f*n + k), each 4-byte aligned; or NULL: no
 *                   likelihood part
 *   lmap4_next_dev  quad maps written by this step, 16-byte aligned
 *   lmap4_cur_dev   quad maps of the current four frames, from an earlier call;
 *                   must not overlap lmap4_next_dev
 *   posterior_dev   host array of 4 device pointers, FP32 [nz][ny][nx] of the
 *                   current four frames, each 16-byte aligned; or NULL: no
 *                   fusion part
 *   occ_dev         NULL, or a host array of 4 nullable u8 [nz][ny][nx]
 *                   device pointers (must be NULL without posteriors)
 * Both parts absent is a no-op. Cameras and grid must be set
 * (PSFS_E_NOT_READY), and the backgrounds for the likelihood part. The host
 * arrays are read before the call returns; the device buffers belong to the
 * caller and must stay valid until the enqueued work is done. */
int psfs_pipeline_step_quad(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap4_next_dev,
                            const float *lmap4_cur_dev, float *const *posterior_dev,
                            uint8_t *const *occ_dev, void *stream);

/* occ[i] = posterior[i] > tau for i < nvox (Sec. 2.2.2 thresholding);
 * tau in [0,1]; nvox >= 0. */
int psfs_threshold(const float *posterior_dev, int64_t nvox, float tau, uint8_t *occ_dev,
                   void *stream);

/* ------------------------------------------ foreground model after frame 1 */

/* Eq. 1-2 take the foreground colour density as uniform (log_u), as nothing
 * is known of the foreground's colours at the first frame (Sec. 2.2.2). For later frames a
 * learned model can replace it (the paper implies one, without describing
 * it; this is the reading taken): a histogram of PSFS_FG_BINS colour bins
 * (bin = (R >> 4) * 256 + (G >> 4) * 16 + (B >> 4)) of the foreground pixels
 * of a frame, pooled over the views, Laplace-smoothed into the density of one
 * colour value, log((count + 1) / ((N + 4096) * 4096)) per bin.
 *   images_dev       n device pointers, u8 [H][W][3] (the frame to learn from)
 *   masks_dev        host array of n nullable device pointers to u8 [H][W]
 *                    (nonzero = foreground), or NULL; a view without a mask
 *                    takes its foreground pixels from lmap_dev: log(2*SLM) > 0
 *                    (SLM > 1/2), maps in the psfs_lmap_* layout
 *   log_density_dev  FP32 [PSFS_FG_BINS] output
 *   workspace        PSFS_FG_BINS * 4 bytes (the counts)
 * Needs cameras. */
int psfs_foreground_model(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *const *masks_dev,
                          const float *lmap_dev, float *log_density_dev, void *workspace_dev,
                          size_t workspace_bytes, void *stream);

/* Use a learned model (FP32 [PSFS_FG_BINS] log densities on the device,
 * borrowed until replaced) in psfs_likelihood, psfs_reconstruct and
 * psfs_pipeline_step: SLM = F(I) / (F(I) + N(I | mu, var)) with
 * F(I) = exp(log_density[bin(I)]) in place of u. NULL restores the uniform
 * density. The differentiable variant and batches keep the uniform density. */
int psfs_set_foreground(psfs_plan *plan, const float *log_density_dev);

/* ------------------------------------------- smoothing and surface voxels */

/* Workspace of psfs_surface (per-block counts). 0 if the grid is unset. */
size_t psfs_surface_workspace_bytes(const psfs_plan *plan);

/* The step after the posterior (Sec. 2.2.2, last paragraph; the paper merges
 * smoothing with voxel generation, Sec. 3.3.1, and removes inner voxels on the
 * CPU, Sec. 3.3.3 step e). For the plan's grid and threshold:
 *   smoothed[v] = mean of posterior over the 3x3x3 voxels around v that lie
 *                 in the grid (FP32, summed in a fixed order);
 *   occ[v]      = smoothed[v] > threshold (u8 0/1);
 *   surface     = ascending linear indices (k*ny + j)*nx + i of the occupied
 *                 voxels with at least one of their 6 face neighbours
 *                 unoccupied or outside the grid.
 * Arguments:
 *   posterior_dev  FP32 [nz][ny][nx] (4-byte aligned)
 *   smoothed_dev   nullable FP32 [nz][ny][nx]
 *   occ_dev        u8 [nz][ny][nx], required (the surface test reads it back)
 *   surface_dev    int32 [capacity]; the first min(count, capacity) entries
 *                  are written (NULL allowed when capacity == 0)
 *   count_dev      one int64 on the device: the number of surface voxels,
 *                  also when it exceeds capacity
 *   workspace      psfs_surface_workspace_bytes bytes, 4-byte aligned
 * Needs only the grid (PSFS_E_NOT_READY otherwise); cameras are not used.
 * An empty grid writes count 0. */
int psfs_surface(psfs_plan *plan, const float *posterior_dev, float *smoothed_dev, uint8_t *occ_dev,
                 int32_t *surface_dev, int64_t capacity, int64_t *count_dev, void *workspace_dev,
                 size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------- voxel colour */

/* Workspace of psfs_colour: one 8-byte depth-buffer entry per likelihood-map
 * element (psfs_lmap_floats of them). 0 if cameras are unset. */
size_t psfs_colour_workspace_bytes(const psfs_plan *plan);

/* Colour of listed voxels from the views that see them (the paper's colour
 * rendering of the reconstructed voxels, Sec. 3.1.1 and Sec. 3.3.3; its rule
 * is not given, this one is): each voxel centre is projected into every view
 * with the nearest-pixel rule of psfs_fuse; at every pixel the listed voxel
 * with the smallest depth (third row of P applied to the centre, FP32) is
 * visible, an equal depth going to the earlier list entry; a voxel's colour is
 * the mean RGB of the pixels where it is visible, over those views.
 *   images_dev  n device pointers, u8 [H][W][3] (4-byte aligned)
 *   voxels_dev  int32 linear indices (k*ny + j)*nx + i, `count` of them, e.g.
 *               the psfs_surface list; entries outside the grid are seen by
 *               no view
 *   colour_dev  FP32 [count][3]: the mean colour, 0 for a voxel no view sees
 *   views_dev   int32 [count]: the number of views in which it is visible
 * Needs cameras and grid. count in [0, 2^31). */
int psfs_colour(psfs_plan *plan, const uint8_t *const *images_dev, const int32_t *voxels_dev, int64_t count,
                float *colour_dev, int32_t *views_dev, void *workspace_dev, size_t workspace_bytes,
                void *stream);

/* ------------------------------------------ particle weights (tracking) */

#define PSFS_CYLINDERS 10       /* cylinders of the body model (Table 1) */

/* Weights of one layer's particle set in the annealed particle filter
 * (Sec. 2.3.1 step 3, Eq. 10; Sec. 2.3.2, Eq. 14-16). A particle is its body
 * model: PSFS_CYLINDERS cylinders (A xyz, B xyz, rA, rB), radii >= 0. The paper
 * does not say which points of the model
 * are sampled; the reading taken: per cylinder and view (camera centre C, from
 * P), 8 cross-sections at t = (m + 1/2) / 8 with centre X = A + t (B - A),
 * radius r = rA + t (rB - rA); u = the unit component of X - C across the
 * axis (length rho), e = unit axis x u;
 *   outline points (Eq. 14)     X - (r^2/rho) u +- r sqrt(1 - r^2/rho^2) e
 *                               (where the viewing ray touches the circle)
 *   silhouette points (Eq. 15)  X, X +- (r/2) e.
 * Each point reads the edge or silhouette map at its nearest pixel (the rule
 * of psfs_fuse, computed in FP64); p = 0 behind the camera, outside the image,
 * and for the five points of a cross-section with rho <= r or with geometry
 * that is not finite (A = B, a non-finite coordinate or radius). Per view
 * Sigma_e = mean of 1 - p over the 160 outline points, Sigma_r over the 240
 * silhouette points; log w = -(sum over views of Sigma_e + Sigma_r), views
 * added in order; normalised weights = w^beta / sum over particles of w^beta
 * (beta: the layer's annealing exponent; 1 = Eq. 16 as printed).
 *   cylinders_dev   FP32 [np][PSFS_CYLINDERS][8], 16-byte aligned
 *   silhouette_dev, edge_dev
 *                   host arrays of n device pointers, FP32 [H][W] maps of view
 *                   k (finite; 4-byte aligned)
 *   beta            finite, >= 0; used only for weights_dev
 *   log_w_dev       FP64 [np] output, required
 *   weights_dev     nullable FP64 [np]: normalised weights
 *   terms_dev       nullable FP64 [np][n][2]: (Sigma_e, Sigma_r) per view
 * Needs cameras (n = 0 gives log w = 0). np in [0, 2^31); np = 0 is a no-op.
 * Results are reproducible bit for bit. No workspace. */
int psfs_particle_weights(psfs_plan *plan, const float *cylinders_dev, int64_t np,
                          const float *const *silhouette_dev, const float *const *edge_dev, double beta,
                          double *log_w_dev, double *weights_dev, double *terms_dev, void *stream);

/* ---------------------------------------- differentiable variant (bilinear) */

/* Workspace of psfs_diff_forward / psfs_diff_backward: likelihood maps,
 * adjoint maps and reduction partials. 0 if cameras or grid unset. */
size_t psfs_diff_workspace_bytes(const psfs_plan *plan);

/* Logits L = logit(prior) + sum_k l~_k with l~_k the bilinear sample of view
 * k's log(2*SLM) (PSFS_BILINEAR rule, whatever params.sampling says), FP32
 * [nz][ny][nx]; and the mean binary cross-entropy with logits against the u8
 * 0/1 labels over the region sub = {i0,i1,j0,j1,k0,k1} (half-open, host
 * array; NULL = whole grid), written as one FP32 to loss_dev.
 * The workspace keeps the likelihood maps for psfs_diff_backward. */
int psfs_diff_forward(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *labels_dev,
                      const int32_t *sub, float *logits_dev, float *loss_dev,
                      void *workspace_dev, size_t workspace_bytes, void *stream);

/* Gradient of grad_loss * loss with respect to every view's background mean
 * and variance (FP32 [H][W][3] each; host arrays of n device pointers) and
 * camera matrices (FP32 [n][12], row-major). grad_loss_dev points to one FP32
 * on the device. Requires the workspace exactly as psfs_diff_forward left it
 * for the same plan, images, labels and sub; projections are recomputed, not
 * stored. Every output element is overwritten. */
int psfs_diff_backward(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *labels_dev,
                       const int32_t *sub, const float *logits_dev, const float *grad_loss_dev,
                       float *const *gmean_dev, float *const *gvar_dev, float *gP_dev,
                       void *workspace_dev, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ batching */

/* One frame of a batch: its own grid, views, images, background and outputs.
 * Host arrays (cams, images_dev, mean_dev, var_dev) are copied at create /
 * update; device pointers are borrowed. */
typedef struct psfs_frame {
    psfs_grid grid;
    int32_t n;                          /* 1..PSFS_MAX_VIEWS */
    const psfs_camera *cams;
    const uint8_t *const *images_dev;
    const float *const *mean_dev;
    const float *const *var_dev;
    float *posterior_dev;               /* [nz][ny][nx] */
    uint8_t *occ_dev;                   /* nullable */
} psfs_frame;

typedef struct psfs_batch psfs_batch;  /* opaque */

/* Plans a batch of nframes (1..65536) frames of uneven shapes, taken in
 * an order that pairs similar likelihood and fusion costs, and processed by a chain of nframes + 1
 * launches: launch i computes the likelihood maps of frame i (Eq. 1-2) beside
 * the fusion of frame i-1 (Eq. 3-9, threshold of Sec. 2.2.2), as the
 * frame-sequence step does for one rig (two launches per step for the
 * 128-lane tile). The launches read the frames from a device descriptor table
 * and are captured into a HIP graph on the first run and replayed afterwards. Every frame's
 * result is bit-identical to psfs_reconstruct of that frame alone (same
 * params). Uses params.sampling (nearest, or the bilinear posterior).
 * Allocates a device descriptor table and a pinned host staging copy on the
 * current device; psfs_batch_destroy frees them. */
int psfs_batch_create(psfs_batch **out, const psfs_params *params, int nframes,
                      const psfs_frame *frames);
size_t psfs_batch_workspace_bytes(const psfs_batch *batch);
/* Runs the batch on `stream`: uploads the descriptor table if it changed,
 * then replays the captured graph (captured on the first run, and again when
 * the workspace pointer or the tile changes). On the null stream, or on a
 * stream the caller is capturing, the kernels are launched directly. Runs of
 * one batch must be ordered (one stream, or synchronised by the caller); they
 * share the workspace, which holds the likelihood maps of every frame. Must
 * run on the device the batch was created on (PSFS_E_DEVICE otherwise). */
int psfs_batch_run(psfs_batch *batch, void *workspace_dev, size_t workspace_bytes, void *stream);
/* Replaces the frames' pointers, camera matrices and grid placement (origin,
 * voxel size). The shape signature (frame count, per-frame grid dims, view
 * counts and image sizes) must be unchanged (PSFS_E_STALE otherwise); the
 * captured graph is then reused and only the descriptor table is re-sent. */
int psfs_batch_update(psfs_batch *batch, int nframes, const psfs_frame *frames);
/* Waits for the batch's outstanding work on the device, then frees it. NULL-safe. */
void psfs_batch_destroy(psfs_batch *batch);

/* Fusion tile of the batch (index into the tile table below; -1 = default). */
int psfs_batch_set_tile(psfs_batch *batch, int tile);
int psfs_batch_get_tile(const psfs_batch *batch);

/* Autotuner: times every fusion tile on this batch (2 warm-up + 5 timed runs
 * each, HIP events on `stream`, blocking) and keeps the fastest. The choice is
 * cached on disk as JSON keyed by device, CU count, sampling and a hash of the
 * shape signature (file: $PSFS_AUTOTUNE_CACHE, else
 * $HOME/.cache/psfs/autotune.json); a cached choice is reused without timing
 * unless force != 0. Tiles never change results, only speed. */
int psfs_batch_tune(psfs_batch *batch, void *workspace_dev, size_t workspace_bytes, void *stream, int force,
                    int *best_tile);


/* Kernel variant selection used by the batch and forward paths:
 * tile = index into the library's fusion tile table (see psfs_tile_count),
 * or -1 for the tuned/default choice. A tile is a workgroup of tx x ty voxel
 * columns of kz voxels each. On the 16 x 16 x 8 tile the one-frame nearest
 * paths of a plan stage each block's per-view pixel boxes in LDS and read
 * them there; every other tile and path gathers from the maps directly. */
int psfs_tile_count(void);
int psfs_tile_describe(int tile, int32_t *tx, int32_t *ty, int32_t *kz);
/* Fusion tile of a plan's one-frame paths (psfs_fuse, psfs_reconstruct,
 * psfs_pipeline_step); -1 = default. The two- and four-frame steps use fixed
 * tiles. Tiles never change results, only speed. */
int psfs_set_tile(psfs_plan *plan, int tile);
int psfs_get_tile(const psfs_plan *plan);     /* the tile in use, or a negative psfs_status */

/* Plan autotuner: computes the plan's likelihood maps of `images_dev` once,
 * then times the fusion with every tile (2 warm-up + 5 timed launches each,
 * HIP events on `stream`, blocking) and sets the fastest on the plan. The
 * choice is cached in the same JSON file as the batch tuner's, keyed by
 * device, CU count, sampling, grid edge class (ceil log2 of the longest grid
 * side), view count and image class (ceil log2 of the largest view's pixel
 * count); a cached choice is applied without timing unless force != 0.
 * workspace_dev: psfs_tune_workspace_bytes(plan) bytes, 256-byte aligned
 * (maps, a posterior and an occupancy grid; overwritten). */
size_t psfs_tune_workspace_bytes(const psfs_plan *plan);
int psfs_tune(psfs_plan *plan, const uint8_t *const *images_dev, void *workspace_dev, size_t workspace_bytes,
              void *stream, int force, int *best_tile);

#ifdef __cplusplus
}
#endif

#endif /* PSFS_H */
