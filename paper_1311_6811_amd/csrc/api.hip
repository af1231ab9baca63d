// Host side of libpsfs: plans, argument validation, workspace layout and
// kernel launches behind the C ABI of psfs.h. Every entry point validates its
// arguments before enqueueing anything and never lets an exception escape.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "host_util.h"
#include "particles.h"

struct psfs_plan {
    int n = -1;                                     // -1: cameras not set
    psfs_camera cams[PSFS_MAX_VIEWS];
    bool has_grid = false;
    psfs_grid grid{};
    psfs_params params{};
    const float *mean[PSFS_MAX_VIEWS] = {};
    const float *var[PSFS_MAX_VIEWS] = {};
    const float *fg = nullptr;                      // learned foreground model (log density per bin)
    uint32_t *check = nullptr;                      // input-check flags (caller's device word), or off
    int tile = -1;
};

namespace psfs {
namespace host {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PSFS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool finite_all(const float *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// Per-device check that the current device is gfx950 (cached).
int check_device()
{
    static std::mutex mu;
    static signed char state[256] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 256) return fail(PSFS_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (state[dev] == 1) return PSFS_OK;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        state[dev] = -1;
        return fail(PSFS_E_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    }
    state[dev] = 1;
    return PSFS_OK;
}

int64_t padded_pixels(int width, int height)
{
    const int64_t np = static_cast<int64_t>(width) * height;
    return (np + kMapAlignFloats - 1) / kMapAlignFloats * kMapAlignFloats;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace host

namespace {

using namespace host;

int64_t map_floats(const psfs_plan *p)
{
    int64_t total = 0;
    for (int k = 0; k < p->n; ++k) {
        const int64_t np = static_cast<int64_t>(p->cams[k].width) * p->cams[k].height;
        total += (np + kMapAlignFloats - 1) / kMapAlignFloats * kMapAlignFloats;
    }
    return total;
}

int64_t map_offset(const psfs_plan *p, int view)
{
    int64_t off = 0;
    for (int k = 0; k < view; ++k) {
        const int64_t np = static_cast<int64_t>(p->cams[k].width) * p->cams[k].height;
        off += (np + kMapAlignFloats - 1) / kMapAlignFloats * kMapAlignFloats;
    }
    return off;
}

int64_t nvox(const psfs_grid &g) { return static_cast<int64_t>(g.nx) * g.ny * g.nz; }

int need_cameras(const psfs_plan *p)
{
    if (!p) return fail(PSFS_E_ARG, "plan is NULL");
    if (p->n < 0) return fail(PSFS_E_NOT_READY, "cameras not set");
    return PSFS_OK;
}

int need_backgrounds(const psfs_plan *p)
{
    int rc = need_cameras(p);
    if (rc) return rc;
    for (int k = 0; k < p->n; ++k)
        if (!p->mean[k] || !p->var[k]) return fail(PSFS_E_NOT_READY, "background of view %d not set", k);
    return PSFS_OK;
}

int need_grid(const psfs_plan *p)
{
    int rc = need_cameras(p);
    if (rc) return rc;
    if (!p->has_grid) return fail(PSFS_E_NOT_READY, "grid not set");
    return PSFS_OK;
}

int check_images(const psfs_plan *p, const uint8_t *const *images)
{
    if (p->n > 0 && !images) return fail(PSFS_E_ARG, "images array is NULL");
    for (int k = 0; k < p->n; ++k) {
        if (!images[k]) return fail(PSFS_E_ARG, "image of view %d is NULL", k);
        if (!aligned(images[k], 4)) return fail(PSFS_E_ARG, "image of view %d is not 4-byte aligned", k);
    }
    return PSFS_OK;
}

// Likelihood-kernel arguments for the views of p; returns the largest view's
// pixel count.
int64_t fill_slm(const psfs_plan *p, const uint8_t *const *images, float *lmap, SlmArgs &a, bool use_fg = true)
{
    a.n = p->n;
    a.lmap = lmap;
    a.fg = use_fg ? p->fg : nullptr;
    a.check = p->check;
    a.k0 = a.fg ? static_cast<float>(-1.5 * std::log(2.0 * M_PI))
                : static_cast<float>(-1.5 * std::log(2.0 * M_PI) - static_cast<double>(p->params.log_u));
    int64_t max_np = 0;
    for (int k = 0; k < p->n; ++k) {
        const int64_t np = static_cast<int64_t>(p->cams[k].width) * p->cams[k].height;
        a.view[k] = SlmView{images[k], p->mean[k], p->var[k], np, map_offset(p, k)};
        if (np > max_np) max_np = np;
    }
    return max_np;
}

int enqueue_likelihood(const psfs_plan *p, const uint8_t *const *images, float *lmap, hipStream_t s,
                       bool use_fg = true)
{
    if (p->n == 0) return PSFS_OK;
    int rc = check_device();
    if (rc) return rc;
    SlmArgs a{};
    const int64_t max_np = fill_slm(p, images, lmap, a, use_fg);
    hipError_t e = launch_slm(a, max_np, s);
    if (e != hipSuccess) return hip_fail(e, "likelihood kernel launch");
    return PSFS_OK;
}

void fill_geometry(const psfs_plan *p, int sampling, FuseArgs &a)
{
    a.n = p->n;
    for (int k = 0; k < p->n; ++k) {
        ViewGeom &g = a.view[k];
        const float *P = p->cams[k].P;
        for (int e = 0; e < 12; ++e) g.P[e] = P[e];
        if (sampling == PSFS_NEAREST) {
            // floor((row0 + row2/2).X / row2.X) = floor(u + 1/2)
            for (int c = 0; c < 4; ++c) {
                g.P[c] = static_cast<float>(static_cast<double>(P[c]) + 0.5 * P[8 + c]);
                g.P[4 + c] = static_cast<float>(static_cast<double>(P[4 + c]) + 0.5 * P[8 + c]);
            }
        }
        g.W = p->cams[k].width;
        g.H = p->cams[k].height;
        g.map_off = map_offset(p, k);
    }
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.ox = p->grid.origin[0];
    a.oy = p->grid.origin[1];
    a.oz = p->grid.origin[2];
    a.h = p->grid.voxel;
    const double pr = p->params.prior;
    a.L0 = static_cast<float>(std::log(pr / (1.0 - pr)));
    a.tau = p->params.threshold;
}

int enqueue_fuse(const psfs_plan *p, const float *lmap, float *post, uint8_t *occ, hipStream_t s)
{
    if (nvox(p->grid) == 0) return PSFS_OK;
    int rc = check_device();
    if (rc) return rc;
    FuseArgs a{};
    fill_geometry(p, p->params.sampling, a);
    a.lmap = lmap;
    a.post = post;
    a.occ = occ;
    const int tile = p->tile >= 0 ? p->tile : default_tile();
    hipError_t e = launch_fuse(a, tile, p->params.sampling, s);
    if (e != hipSuccess) return hip_fail(e, "fusion kernel launch");
    return PSFS_OK;
}


// Workspace of the differentiable pass: likelihood maps, adjoint maps, loss
// partials, camera-gradient partials; each region 256-byte aligned.
struct DiffLayout {
    size_t lmap, adj, loss, cam, total;
};

DiffLayout diff_layout(const psfs_plan *p)
{
    DiffLayout L{};
    const size_t maps = static_cast<size_t>(map_floats(p)) * sizeof(float);
    const int64_t nbf = p->has_grid ? diff_fwd_blocks(p->grid.nx, p->grid.ny, p->grid.nz) : 0;
    const int64_t nbb = p->has_grid ? diff_bwd_blocks(p->grid.nx, p->grid.ny, p->grid.nz) : 0;
    L.lmap = 0;
    L.adj = align256(maps);
    L.loss = L.adj + align256(2 * maps);            // int64 adjoint per pixel
    L.cam = L.loss + align256(static_cast<size_t>(nbf) * sizeof(double));
    L.total = L.cam + align256(static_cast<size_t>(nbb) * 12 * (p->n > 0 ? p->n : 0) * sizeof(float));
    return L;
}

int check_region(const psfs_plan *p, const int32_t *sub, int32_t out[6], float *inv_count)
{
    const int32_t dims[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    for (int d = 0; d < 3; ++d) {
        const int32_t lo = sub ? sub[2 * d] : 0, hi = sub ? sub[2 * d + 1] : dims[d];
        if (lo < 0 || hi < lo || hi > dims[d]) return fail(PSFS_E_RANGE, "loss region axis %d [%d,%d) outside [0,%d)", d, lo, hi, dims[d]);
        out[2 * d] = lo;
        out[2 * d + 1] = hi;
    }
    const int64_t cnt = static_cast<int64_t>(out[1] - out[0]) * (out[3] - out[2]) * (out[5] - out[4]);
    *inv_count = cnt > 0 ? static_cast<float>(1.0 / static_cast<double>(cnt)) : 0.0f;
    return PSFS_OK;
}

int prepare_diff(const psfs_plan *p, const uint8_t *const *images, const uint8_t *labels, const int32_t *sub,
                 void *ws, size_t ws_bytes, DiffArgs &a, DiffLayout &L)
{
    int rc = need_backgrounds(p);
    if (rc) return rc;
    if ((rc = need_grid(p))) return rc;
    if ((rc = check_images(p, images))) return rc;
    if (nvox(p->grid) > 0 && !labels) return fail(PSFS_E_ARG, "labels is NULL");
    a = DiffArgs{};
    if ((rc = check_region(p, sub, a.sub, &a.inv_count))) return rc;
    L = diff_layout(p);
    if (!ws || ws_bytes < L.total || !aligned(ws, 256))
        return fail(PSFS_E_WORKSPACE, "differentiable workspace needs %zu bytes, 256-byte aligned (got %zu)", L.total, ws_bytes);
    FuseArgs f{};
    fill_geometry(p, PSFS_BILINEAR, f);
    for (int k = 0; k < p->n; ++k) {
        a.view[k] = f.view[k];
        for (int e = 0; e < 12; ++e) a.Pd[k][e] = static_cast<double>(p->cams[k].P[e]);
    }
    char *base = static_cast<char *>(ws);
    a.lmap = reinterpret_cast<const float *>(base + L.lmap);
    a.adj = reinterpret_cast<float *>(base + L.adj);
    a.loss_part = reinterpret_cast<double *>(base + L.loss);
    a.cam_part = reinterpret_cast<float *>(base + L.cam);
    a.labels = labels;
    a.n = p->n;
    a.nx = p->grid.nx; a.ny = p->grid.ny; a.nz = p->grid.nz;
    a.ox = f.ox; a.oy = f.oy; a.oz = f.oz; a.h = f.h;
    a.L0 = f.L0;
    return PSFS_OK;
}
}  // namespace
}  // namespace psfs

using namespace psfs;
using namespace psfs::host;


// Likelihood maps of psfs_reconstruct_static: one array per GPU, in the code
// object, for callers that cannot allocate. In host code `scratch` names a
// host-side stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) float scratch[PSFS_STATIC_SCRATCH_BYTES / sizeof(float)];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[256] = {};          // device address of `scratch` per device ordinal

// Address of `scratch` on the current device (looked up on its first use there).
int static_scratch(float **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 256) return fail(PSFS_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch array");
        if (!ptr) return fail(PSFS_E_HIP, "hipGetSymbolAddress returned no address for the static scratch array");
        g_scratch_dev[dev] = ptr;
    }
    *out = static_cast<float *>(g_scratch_dev[dev]);
    return PSFS_OK;
}

}  // namespace

extern "C" {

int psfs_version(void) { return PSFS_VERSION; }

const char *psfs_status_str(int status)
{
    switch (status) {
    case PSFS_OK: return "ok";
    case PSFS_E_ARG: return "invalid argument";
    case PSFS_E_RANGE: return "value out of range";
    case PSFS_E_NOT_READY: return "plan not ready";
    case PSFS_E_WORKSPACE: return "workspace too small";
    case PSFS_E_HIP: return "HIP runtime error";
    case PSFS_E_DEVICE: return "unsupported device";
    case PSFS_E_STALE: return "batch shape changed";
    case PSFS_E_INPUT: return "invalid input values";
    default: return "unknown status";
    }
}

const char *psfs_last_error(void) { return psfs::host::g_last_error.c_str(); }

void psfs_default_params(psfs_params *out)
{
    if (!out) return;
    out->prior = 0.5f;
    out->log_u = static_cast<float>(-3.0 * std::log(256.0));
    out->threshold = 0.5f;
    out->sampling = PSFS_NEAREST;
}

int psfs_plan_create(psfs_plan **out)
{
    PSFS_GUARD_BEGIN
    if (!out) return fail(PSFS_E_ARG, "out is NULL");
    psfs_plan *p = new psfs_plan();
    psfs_default_params(&p->params);
    *out = p;
    return PSFS_OK;
    PSFS_GUARD_END
}

void psfs_plan_destroy(psfs_plan *plan) { delete plan; }

int psfs_set_cameras(psfs_plan *plan, int n, const psfs_camera *cams)
{
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (n < 0 || n > PSFS_MAX_VIEWS) return fail(PSFS_E_RANGE, "view count %d outside 0..%d", n, PSFS_MAX_VIEWS);
    if (n > 0 && !cams) return fail(PSFS_E_ARG, "cams is NULL");
    for (int k = 0; k < n; ++k) {
        const psfs_camera &c = cams[k];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535 ||
            static_cast<int64_t>(c.width) * c.height >= (int64_t(1) << 30))
            return fail(PSFS_E_RANGE, "view %d: image size %dx%d out of range", k, c.width, c.height);
        if (!finite_all(c.P, 12)) return fail(PSFS_E_RANGE, "view %d: camera matrix not finite", k);
    }
    plan->n = n;
    for (int k = 0; k < n; ++k) plan->cams[k] = cams[k];
    for (int k = 0; k < PSFS_MAX_VIEWS; ++k) plan->mean[k] = plan->var[k] = nullptr;
    return PSFS_OK;
}

int psfs_set_grid(psfs_plan *plan, const psfs_grid *g)
{
    if (!plan || !g) return fail(PSFS_E_ARG, "plan or grid is NULL");
    if (g->nx < 0 || g->ny < 0 || g->nz < 0 || nvox(*g) >= (int64_t(1) << 31))
        return fail(PSFS_E_RANGE, "grid %dx%dx%d out of range", g->nx, g->ny, g->nz);
    if (!(g->voxel > 0.0f) || !std::isfinite(g->voxel) || !finite_all(g->origin, 3))
        return fail(PSFS_E_RANGE, "grid voxel size or origin invalid");
    plan->grid = *g;
    plan->has_grid = true;
    return PSFS_OK;
}

int psfs_set_params(psfs_plan *plan, const psfs_params *prm)
{
    if (!plan || !prm) return fail(PSFS_E_ARG, "plan or params is NULL");
    if (!(prm->prior > 0.0f && prm->prior < 1.0f)) return fail(PSFS_E_RANGE, "prior must lie in (0,1)");
    if (!std::isfinite(prm->log_u)) return fail(PSFS_E_RANGE, "log_u must be finite");
    if (!(prm->threshold >= 0.0f && prm->threshold <= 1.0f)) return fail(PSFS_E_RANGE, "threshold must lie in [0,1]");
    if (prm->sampling != PSFS_NEAREST && prm->sampling != PSFS_BILINEAR)
        return fail(PSFS_E_ARG, "unknown sampling %d", prm->sampling);
    plan->params = *prm;
    return PSFS_OK;
}

int psfs_set_background(psfs_plan *plan, int view, const float *mean_dev, const float *var_dev)
{
    int rc = need_cameras(plan);
    if (rc) return rc;
    if (view < 0 || view >= plan->n) return fail(PSFS_E_RANGE, "view %d outside 0..%d", view, plan->n - 1);
    if (!mean_dev || !var_dev) return fail(PSFS_E_ARG, "background pointer is NULL");
    if (!aligned(mean_dev, 16) || !aligned(var_dev, 16)) return fail(PSFS_E_ARG, "background pointers must be 16-byte aligned");
    plan->mean[view] = mean_dev;
    plan->var[view] = var_dev;
    return PSFS_OK;
}

int psfs_set_input_check(psfs_plan *plan, uint32_t *flags_dev)
{
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (flags_dev && !aligned(flags_dev, 4)) return fail(PSFS_E_ARG, "flags must be a 4-byte aligned device pointer");
    plan->check = flags_dev;
    return PSFS_OK;
}

int psfs_input_status(psfs_plan *plan)
{
    PSFS_GUARD_BEGIN
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (!plan->check) return fail(PSFS_E_NOT_READY, "no input-check flags set (psfs_set_input_check)");
    uint32_t flags = 0;
    hipError_t e = hipMemcpy(&flags, plan->check, sizeof(flags), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the input-check flags");
    if (flags == 0) return PSFS_OK;
    const uint32_t zero = 0;
    e = hipMemcpy(plan->check, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing the input-check flags");
    std::string views;
    for (int k = 0; k < 32; ++k)
        if (flags & (1u << k)) views += (views.empty() ? "" : ", ") + std::to_string(k);
    return fail(PSFS_E_INPUT, "background model of view(s) %s holds a variance <= 0, NaN or Inf or a non-finite mean",
                views.c_str());
    PSFS_GUARD_END
}

int64_t psfs_lmap_floats(const psfs_plan *plan)
{
    int rc = need_cameras(plan);
    if (rc) return rc;
    return map_floats(plan);
}

int64_t psfs_lmap_offset(const psfs_plan *plan, int view)
{
    int rc = need_cameras(plan);
    if (rc) return rc;
    if (view < 0 || view >= plan->n) return fail(PSFS_E_RANGE, "view %d outside 0..%d", view, plan->n - 1);
    return map_offset(plan, view);
}

size_t psfs_workspace_bytes(const psfs_plan *plan)
{
    if (!plan || plan->n < 0) return 0;
    return static_cast<size_t>(map_floats(plan)) * sizeof(float);
}

int psfs_likelihood(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_backgrounds(plan);
    if (rc) return rc;
    if ((rc = check_images(plan, images_dev))) return rc;
    if (plan->n > 0 && (!lmap_dev || !aligned(lmap_dev, 16))) return fail(PSFS_E_ARG, "lmap must be a 16-byte aligned device pointer");
    return enqueue_likelihood(plan, images_dev, lmap_dev, static_cast<hipStream_t>(stream));
    PSFS_GUARD_END
}

int psfs_fuse(psfs_plan *plan, const float *lmap_dev, float *posterior_dev, uint8_t *occ_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_grid(plan);
    if (rc) return rc;
    if (nvox(plan->grid) > 0) {
        if (!posterior_dev || !aligned(posterior_dev, 16)) return fail(PSFS_E_ARG, "posterior must be a 16-byte aligned device pointer");
        if (plan->n > 0 && (!lmap_dev || !aligned(lmap_dev, 16))) return fail(PSFS_E_ARG, "lmap must be a 16-byte aligned device pointer");
    }
    return enqueue_fuse(plan, lmap_dev, posterior_dev, occ_dev, static_cast<hipStream_t>(stream));
    PSFS_GUARD_END
}

int psfs_reconstruct(psfs_plan *plan, const uint8_t *const *images_dev, float *posterior_dev, uint8_t *occ_dev,
                     void *workspace_dev, size_t workspace_bytes, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_backgrounds(plan);
    if (rc) return rc;
    if ((rc = need_grid(plan))) return rc;
    if ((rc = check_images(plan, images_dev))) return rc;
    if (nvox(plan->grid) > 0 && (!posterior_dev || !aligned(posterior_dev, 16)))
        return fail(PSFS_E_ARG, "posterior must be a 16-byte aligned device pointer");
    const size_t need = psfs_workspace_bytes(plan);
    if (need > 0 && (!workspace_dev || workspace_bytes < need || !aligned(workspace_dev, 16)))
        return fail(PSFS_E_WORKSPACE, "workspace needs %zu bytes, 16-byte aligned (got %zu)", need, workspace_bytes);
    if (nvox(plan->grid) == 0) return PSFS_OK;
    float *lmap = static_cast<float *>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = enqueue_likelihood(plan, images_dev, lmap, s))) return rc;
    return enqueue_fuse(plan, lmap, posterior_dev, occ_dev, s);
    PSFS_GUARD_END
}

int psfs_reconstruct_static(psfs_plan *plan, const uint8_t *const *images_dev, float *posterior_dev,
                            uint8_t *occ_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_backgrounds(plan);
    if (rc) return rc;
    if ((rc = need_grid(plan))) return rc;
    if ((rc = check_images(plan, images_dev))) return rc;
    if (nvox(plan->grid) > 0 && (!posterior_dev || !aligned(posterior_dev, 16)))
        return fail(PSFS_E_ARG, "posterior must be a 16-byte aligned device pointer");
    const size_t need = psfs_workspace_bytes(plan);
    if (need > PSFS_STATIC_SCRATCH_BYTES)
        return fail(PSFS_E_RANGE, "the likelihood maps need %zu bytes; the static scratch holds %zu (use psfs_reconstruct)",
                    need, static_cast<size_t>(PSFS_STATIC_SCRATCH_BYTES));
    if (nvox(plan->grid) == 0) return PSFS_OK;
    if ((rc = check_device())) return rc;
    float *lmap = nullptr;
    if ((rc = static_scratch(&lmap))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = enqueue_likelihood(plan, images_dev, lmap, s))) return rc;
    return enqueue_fuse(plan, lmap, posterior_dev, occ_dev, s);
    PSFS_GUARD_END
}

int psfs_pipeline_step(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap_next_dev,
                       const float *lmap_cur_dev, float *posterior_dev, uint8_t *occ_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_grid(plan);
    if (rc) return rc;
    const bool next = images_dev != nullptr, cur = posterior_dev != nullptr;
    const int64_t maps = map_floats(plan);
    if (next) {
        if ((rc = need_backgrounds(plan))) return rc;
        if ((rc = check_images(plan, images_dev))) return rc;
        if (plan->n > 0 && (!lmap_next_dev || !aligned(lmap_next_dev, 16)))
            return fail(PSFS_E_ARG, "lmap_next must be a 16-byte aligned device pointer");
    }
    if (cur) {
        if (!aligned(posterior_dev, 16)) return fail(PSFS_E_ARG, "posterior must be 16-byte aligned");
        if (plan->n > 0 && (!lmap_cur_dev || !aligned(lmap_cur_dev, 16)))
            return fail(PSFS_E_ARG, "lmap_cur must be a 16-byte aligned device pointer");
    } else if (occ_dev) {
        return fail(PSFS_E_ARG, "occupancy given without a posterior");
    }
    if (next && cur && maps > 0) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(lmap_next_dev), b0 = reinterpret_cast<uintptr_t>(lmap_cur_dev);
        const uintptr_t len = static_cast<uintptr_t>(maps) * sizeof(float);
        if (a0 < b0 + len && b0 < a0 + len) return fail(PSFS_E_ARG, "lmap_next and lmap_cur overlap");
    }
    SlmArgs sa{};
    int64_t max_np = 0;
    if (next && plan->n > 0) max_np = fill_slm(plan, images_dev, lmap_next_dev, sa);
    FuseArgs fa{};
    fill_geometry(plan, plan->params.sampling, fa);
    fa.lmap = lmap_cur_dev;
    fa.post = (cur && nvox(plan->grid) > 0) ? posterior_dev : nullptr;
    fa.occ = fa.post ? occ_dev : nullptr;
    if (sa.n == 0 && !fa.post) return PSFS_OK;
    if ((rc = check_device())) return rc;
    const int tile = plan->tile >= 0 ? plan->tile : default_tile();
    hipError_t e = launch_pipeline(sa, fa, tile, plan->params.sampling, max_np, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pipelined kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_pipeline_step_pair(psfs_plan *plan, const uint8_t *const *images_a_dev, const uint8_t *const *images_b_dev,
                            float *lmap2_next_dev, const float *lmap2_cur_dev, float *posterior_a_dev,
                            uint8_t *occ_a_dev, float *posterior_b_dev, uint8_t *occ_b_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_grid(plan);
    if (rc) return rc;
    if (plan->params.sampling != PSFS_NEAREST) return fail(PSFS_E_ARG, "two-frame steps use nearest sampling");
    const bool next = images_a_dev != nullptr || images_b_dev != nullptr;
    const bool cur = posterior_a_dev != nullptr || posterior_b_dev != nullptr;
    const int64_t maps = map_floats(plan);
    if (next) {
        if (!images_a_dev || !images_b_dev) return fail(PSFS_E_ARG, "both frames' images are needed");
        if ((rc = need_backgrounds(plan))) return rc;
        if ((rc = check_images(plan, images_a_dev))) return rc;
        if ((rc = check_images(plan, images_b_dev))) return rc;
        if (plan->n > 0 && (!lmap2_next_dev || !aligned(lmap2_next_dev, 16)))
            return fail(PSFS_E_ARG, "lmap2_next must be a 16-byte aligned device pointer");
    }
    if (cur) {
        if (!posterior_a_dev || !posterior_b_dev) return fail(PSFS_E_ARG, "both frames' posteriors are needed");
        if (!aligned(posterior_a_dev, 16) || !aligned(posterior_b_dev, 16))
            return fail(PSFS_E_ARG, "posteriors must be 16-byte aligned");
        if (plan->n > 0 && (!lmap2_cur_dev || !aligned(lmap2_cur_dev, 16)))
            return fail(PSFS_E_ARG, "lmap2_cur must be a 16-byte aligned device pointer");
    } else if (occ_a_dev || occ_b_dev) {
        return fail(PSFS_E_ARG, "occupancy given without a posterior");
    }
    if (next && cur && maps > 0) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(lmap2_next_dev), b0 = reinterpret_cast<uintptr_t>(lmap2_cur_dev);
        const uintptr_t len = 2 * static_cast<uintptr_t>(maps) * sizeof(float);
        if (a0 < b0 + len && b0 < a0 + len) return fail(PSFS_E_ARG, "lmap2_next and lmap2_cur overlap");
    }
    SlmArgs sa{};
    PairImages ib{};
    int64_t max_np = 0;
    if (next && plan->n > 0) {
        max_np = fill_slm(plan, images_a_dev, lmap2_next_dev, sa);
        for (int k = 0; k < plan->n; ++k) ib.img[k] = images_b_dev[k];
    }
    FuseArgs fa{};
    fill_geometry(plan, PSFS_NEAREST, fa);
    fa.lmap = lmap2_cur_dev;
    const bool fuse = cur && nvox(plan->grid) > 0;
    fa.post = fuse ? posterior_a_dev : nullptr;
    fa.occ = fuse ? occ_a_dev : nullptr;
    if (sa.n == 0 && !fa.post) return PSFS_OK;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_pipeline_pair(sa, ib, fa, fuse ? posterior_b_dev : nullptr, fuse ? occ_b_dev : nullptr, max_np,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "two-frame pipelined kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_pipeline_step_quad(psfs_plan *plan, const uint8_t *const *images_dev, float *lmap4_next_dev,
                            const float *lmap4_cur_dev, float *const *posterior_dev, uint8_t *const *occ_dev,
                            void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_grid(plan);
    if (rc) return rc;
    if (plan->params.sampling != PSFS_NEAREST) return fail(PSFS_E_ARG, "four-frame steps use nearest sampling");
    for (int k = 0; k < plan->n; ++k)    // quad maps are gathered with 32-bit byte offsets
        if (static_cast<int64_t>(plan->cams[k].width) * plan->cams[k].height >= (int64_t(1) << 28))
            return fail(PSFS_E_RANGE, "view %d: four-frame steps need images below 2^28 pixels", k);
    const bool next = images_dev != nullptr;
    const bool cur = posterior_dev != nullptr;
    const int64_t maps = map_floats(plan);
    const int n = plan->n;
    if (next) {
        if ((rc = need_backgrounds(plan))) return rc;
        for (int f = 0; f < 4; ++f)
            if ((rc = check_images(plan, images_dev + static_cast<ptrdiff_t>(f) * n))) return rc;
        if (n > 0 && (!lmap4_next_dev || !aligned(lmap4_next_dev, 16)))
            return fail(PSFS_E_ARG, "lmap4_next must be a 16-byte aligned device pointer");
    }
    if (cur) {
        for (int f = 0; f < 4; ++f) {
            if (!posterior_dev[f]) return fail(PSFS_E_ARG, "posterior of frame %d is NULL", f);
            if (!aligned(posterior_dev[f], 16)) return fail(PSFS_E_ARG, "posterior of frame %d is not 16-byte aligned", f);
        }
        if (n > 0 && (!lmap4_cur_dev || !aligned(lmap4_cur_dev, 16)))
            return fail(PSFS_E_ARG, "lmap4_cur must be a 16-byte aligned device pointer");
    } else if (occ_dev) {
        return fail(PSFS_E_ARG, "occupancy given without posteriors");
    }
    if (next && cur && maps > 0) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(lmap4_next_dev), b0 = reinterpret_cast<uintptr_t>(lmap4_cur_dev);
        const uintptr_t len = 4 * static_cast<uintptr_t>(maps) * sizeof(float);
        if (a0 < b0 + len && b0 < a0 + len) return fail(PSFS_E_ARG, "lmap4_next and lmap4_cur overlap");
    }
    SlmArgs sa{};
    QuadImages qi{};
    int64_t max_np = 0;
    if (next && n > 0) {
        max_np = fill_slm(plan, images_dev, lmap4_next_dev, sa);
        for (int f = 1; f < 4; ++f)
            for (int k = 0; k < n; ++k) qi.img[f - 1][k] = images_dev[static_cast<ptrdiff_t>(f) * n + k];
    }
    FuseArgs fa{};
    fill_geometry(plan, PSFS_NEAREST, fa);
    fa.lmap = lmap4_cur_dev;
    const bool fuse = cur && nvox(plan->grid) > 0;
    QuadOut qo{};
    if (fuse) {
        fa.post = posterior_dev[0];
        fa.occ = occ_dev ? occ_dev[0] : nullptr;
        for (int f = 1; f < 4; ++f) {
            qo.post[f - 1] = posterior_dev[f];
            qo.occ[f - 1] = occ_dev ? occ_dev[f] : nullptr;
        }
    }
    if (sa.n == 0 && !fa.post) return PSFS_OK;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_pipeline_quad(sa, qi, fa, qo, max_np, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "four-frame pipelined kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_threshold(const float *posterior_dev, int64_t nvox_, float tau, uint8_t *occ_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    if (nvox_ < 0) return fail(PSFS_E_RANGE, "nvox must be >= 0");
    if (!(tau >= 0.0f && tau <= 1.0f)) return fail(PSFS_E_RANGE, "tau must lie in [0,1]");
    if (nvox_ == 0) return PSFS_OK;
    if (!posterior_dev || !occ_dev) return fail(PSFS_E_ARG, "posterior or occ is NULL");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = launch_threshold(posterior_dev, nvox_, tau, occ_dev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "threshold kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

size_t psfs_surface_workspace_bytes(const psfs_plan *plan)
{
    if (!plan || !plan->has_grid) return 0;
    const int64_t V = nvox(plan->grid);
    return align256(static_cast<size_t>(surface_blocks(V)) * sizeof(int32_t)) + align256(static_cast<size_t>(V));
}

int psfs_surface(psfs_plan *plan, const float *posterior_dev, float *smoothed_dev, uint8_t *occ_dev,
                 int32_t *surface_dev, int64_t capacity, int64_t *count_dev, void *workspace_dev,
                 size_t workspace_bytes, void *stream)
{
    PSFS_GUARD_BEGIN
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (!plan->has_grid) return fail(PSFS_E_NOT_READY, "grid not set");
    if (capacity < 0) return fail(PSFS_E_RANGE, "capacity must be >= 0");
    if (!count_dev || !aligned(count_dev, 8)) return fail(PSFS_E_ARG, "count must be an 8-byte aligned device pointer");
    const int64_t V = nvox(plan->grid);
    if (V > 0) {
        if (!posterior_dev || !aligned(posterior_dev, 4)) return fail(PSFS_E_ARG, "posterior must be a 4-byte aligned device pointer");
        if (smoothed_dev && !aligned(smoothed_dev, 4)) return fail(PSFS_E_ARG, "smoothed must be 4-byte aligned");
        if (!occ_dev) return fail(PSFS_E_ARG, "occupancy output is NULL");
        if (capacity > 0 && (!surface_dev || !aligned(surface_dev, 4)))
            return fail(PSFS_E_ARG, "surface must be a 4-byte aligned device pointer");
        const size_t need = psfs_surface_workspace_bytes(plan);
        if (!workspace_dev || workspace_bytes < need || !aligned(workspace_dev, 256))
            return fail(PSFS_E_WORKSPACE, "surface workspace needs %zu bytes, 256-byte aligned (got %zu)", need,
                        workspace_bytes);
    }
    int rc = check_device();
    if (rc) return rc;
    SurfArgs a{};
    a.post = posterior_dev;
    a.smoothed = smoothed_dev;
    a.occ = occ_dev;
    a.out = surface_dev;
    a.capacity = capacity;
    a.count = count_dev;
    a.counts = static_cast<int32_t *>(workspace_dev);
    a.nvox = V;
    a.nblocks = static_cast<int32_t>(surface_blocks(V));
    a.nx = plan->grid.nx;
    a.ny = plan->grid.ny;
    a.nz = plan->grid.nz;
    a.flags = static_cast<uint8_t *>(workspace_dev) + align256(static_cast<size_t>(a.nblocks) * sizeof(int32_t));
    if (V > 0) {
        const int64_t nx = a.nx, ny = a.ny;
        a.step_i = static_cast<int32_t>(256 % nx);
        a.step_j = static_cast<int32_t>((256 / nx) % ny);
        a.step_k = static_cast<int32_t>(256 / (nx * ny));
    }
    a.tau = plan->params.threshold;
    hipError_t e = launch_surface(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "surface kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

size_t psfs_colour_workspace_bytes(const psfs_plan *plan)
{
    if (!plan || plan->n < 0) return 0;
    return static_cast<size_t>(map_floats(plan)) * sizeof(unsigned long long);
}

int psfs_colour(psfs_plan *plan, const uint8_t *const *images_dev, const int32_t *voxels_dev, int64_t count,
                float *colour_dev, int32_t *views_dev, void *workspace_dev, size_t workspace_bytes, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_grid(plan);
    if (rc) return rc;
    if (count < 0 || count >= (int64_t(1) << 31)) return fail(PSFS_E_RANGE, "voxel count %lld out of range", static_cast<long long>(count));
    if ((rc = check_images(plan, images_dev))) return rc;
    if (count > 0) {
        if (!voxels_dev || !aligned(voxels_dev, 4)) return fail(PSFS_E_ARG, "voxel list must be a 4-byte aligned device pointer");
        if (!colour_dev || !aligned(colour_dev, 4)) return fail(PSFS_E_ARG, "colour output must be a 4-byte aligned device pointer");
        if (!views_dev || !aligned(views_dev, 4)) return fail(PSFS_E_ARG, "view-count output must be a 4-byte aligned device pointer");
    }
    const size_t need = psfs_colour_workspace_bytes(plan);
    if (need > 0 && (!workspace_dev || workspace_bytes < need || !aligned(workspace_dev, 8)))
        return fail(PSFS_E_WORKSPACE, "colour workspace needs %zu bytes, 8-byte aligned (got %zu)", need, workspace_bytes);
    if (count == 0) return PSFS_OK;
    if ((rc = check_device())) return rc;
    FuseArgs fa{};
    fill_geometry(plan, PSFS_NEAREST, fa);
    ColourArgs a{};
    for (int k = 0; k < plan->n; ++k) {
        a.view[k] = fa.view[k];
        a.img[k] = images_dev[k];
    }
    a.list = voxels_dev;
    a.nlist = count;
    a.zbuf = static_cast<unsigned long long *>(workspace_dev);
    a.zbuf_len = map_floats(plan);
    a.colour = colour_dev;
    a.views = views_dev;
    a.nvox = nvox(plan->grid);
    a.n = plan->n;
    a.nx = fa.nx;
    a.ny = fa.ny;
    a.ox = fa.ox;
    a.oy = fa.oy;
    a.oz = fa.oz;
    a.h = fa.h;
    hipError_t e = launch_colour(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "colour kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_foreground_model(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *const *masks_dev,
                          const float *lmap_dev, float *log_density_dev, void *workspace_dev, size_t workspace_bytes,
                          void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_cameras(plan);
    if (rc) return rc;
    if ((rc = check_images(plan, images_dev))) return rc;
    if (!log_density_dev || !aligned(log_density_dev, 4))
        return fail(PSFS_E_ARG, "log_density must be a 4-byte aligned device pointer");
    bool need_maps = !masks_dev;
    for (int k = 0; masks_dev && k < plan->n; ++k) need_maps = need_maps || !masks_dev[k];
    if (need_maps && plan->n > 0 && (!lmap_dev || !aligned(lmap_dev, 4)))
        return fail(PSFS_E_ARG, "lmap is needed for views without a mask");
    if (!workspace_dev || workspace_bytes < PSFS_FG_BINS * sizeof(uint32_t) || !aligned(workspace_dev, 4))
        return fail(PSFS_E_WORKSPACE, "foreground workspace needs %zu bytes", static_cast<size_t>(PSFS_FG_BINS * sizeof(uint32_t)));
    if ((rc = check_device())) return rc;
    FgArgs a{};
    a.n = plan->n;
    int64_t max_np = 0;
    for (int k = 0; k < plan->n; ++k) {
        const int64_t np = static_cast<int64_t>(plan->cams[k].width) * plan->cams[k].height;
        a.view[k] = SlmView{images_dev[k], nullptr, nullptr, np, map_offset(plan, k)};
        a.mask[k] = masks_dev ? masks_dev[k] : nullptr;
        if (np > max_np) max_np = np;
    }
    a.lmap = lmap_dev;
    a.counts = static_cast<uint32_t *>(workspace_dev);
    a.logd = log_density_dev;
    hipError_t e = launch_foreground(a, max_np, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "foreground model kernel launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_set_foreground(psfs_plan *plan, const float *log_density_dev)
{
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (log_density_dev && !aligned(log_density_dev, 4)) return fail(PSFS_E_ARG, "log_density must be 4-byte aligned");
    plan->fg = log_density_dev;
    return PSFS_OK;
}

int psfs_particle_weights(psfs_plan *plan, const float *cylinders_dev, int64_t np,
                          const float *const *silhouette_dev, const float *const *edge_dev, double beta,
                          double *log_w_dev, double *weights_dev, double *terms_dev, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = need_cameras(plan);
    if (rc) return rc;
    if (np < 0 || np >= (int64_t(1) << 31)) return fail(PSFS_E_RANGE, "particle count %lld out of range", static_cast<long long>(np));
    if (weights_dev && !(std::isfinite(beta) && beta >= 0.0)) return fail(PSFS_E_RANGE, "beta must be finite and >= 0");
    if (np == 0) return PSFS_OK;
    if (!cylinders_dev || !aligned(cylinders_dev, 16)) return fail(PSFS_E_ARG, "cylinders must be a 16-byte aligned device pointer");
    if (!log_w_dev || !aligned(log_w_dev, 8)) return fail(PSFS_E_ARG, "log_w must be an 8-byte aligned device pointer");
    if (weights_dev && !aligned(weights_dev, 8)) return fail(PSFS_E_ARG, "weights must be 8-byte aligned");
    if (terms_dev && !aligned(terms_dev, 8)) return fail(PSFS_E_ARG, "terms must be 8-byte aligned");
    if (plan->n > 0 && (!silhouette_dev || !edge_dev)) return fail(PSFS_E_ARG, "map arrays are NULL");
    for (int k = 0; k < plan->n; ++k) {
        if (!silhouette_dev[k] || !aligned(silhouette_dev[k], 4)) return fail(PSFS_E_ARG, "silhouette map of view %d must be a 4-byte aligned device pointer", k);
        if (!edge_dev[k] || !aligned(edge_dev[k], 4)) return fail(PSFS_E_ARG, "edge map of view %d must be a 4-byte aligned device pointer", k);
    }
    if ((rc = check_device())) return rc;
    PartArgs a{};
    for (int k = 0; k < plan->n; ++k) {
        a.view[k].sil = silhouette_dev[k];
        a.view[k].edge = edge_dev[k];
        a.view[k].w = plan->cams[k].width;
        a.view[k].h = plan->cams[k].height;
        std::memcpy(a.view[k].P, plan->cams[k].P, sizeof(a.view[k].P));
    }
    a.cyl = cylinders_dev;
    a.logw = log_w_dev;
    a.terms = terms_dev;
    a.np = np;
    a.n = plan->n;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_particle_weights(a, s);
    if (e != hipSuccess) return hip_fail(e, "particle weight kernel launch");
    if (weights_dev) {
        e = launch_particle_normalise(NormArgs{log_w_dev, weights_dev, np, beta}, s);
        if (e != hipSuccess) return hip_fail(e, "particle normalisation kernel launch");
    }
    return PSFS_OK;
    PSFS_GUARD_END
}

size_t psfs_diff_workspace_bytes(const psfs_plan *plan)
{
    if (!plan || plan->n < 0 || !plan->has_grid) return 0;
    return diff_layout(plan).total;
}

int psfs_diff_forward(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *labels_dev,
                      const int32_t *sub, float *logits_dev, float *loss_dev, void *workspace_dev,
                      size_t workspace_bytes, void *stream)
{
    PSFS_GUARD_BEGIN
    DiffArgs a;
    DiffLayout L;
    int rc = prepare_diff(plan, images_dev, labels_dev, sub, workspace_dev, workspace_bytes, a, L);
    if (rc) return rc;
    if (!loss_dev) return fail(PSFS_E_ARG, "loss is NULL");
    if (nvox(plan->grid) > 0 && (!logits_dev || !aligned(logits_dev, 16))) return fail(PSFS_E_ARG, "logits must be a 16-byte aligned device pointer");
    if ((rc = check_device())) return rc;
    a.logits = logits_dev;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the differentiable variant keeps the uniform foreground density (the
    // pixel chain differentiates that form)
    if ((rc = enqueue_likelihood(plan, images_dev, const_cast<float *>(a.lmap), s, false))) return rc;
    hipError_t e = launch_diff_forward(a, loss_dev, s);
    if (e != hipSuccess) return hip_fail(e, "differentiable forward launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_diff_backward(psfs_plan *plan, const uint8_t *const *images_dev, const uint8_t *labels_dev,
                       const int32_t *sub, const float *logits_dev, const float *grad_loss_dev,
                       float *const *gmean_dev, float *const *gvar_dev, float *gP_dev, void *workspace_dev,
                       size_t workspace_bytes, void *stream)
{
    PSFS_GUARD_BEGIN
    DiffArgs a;
    DiffLayout L;
    int rc = prepare_diff(plan, images_dev, labels_dev, sub, workspace_dev, workspace_bytes, a, L);
    if (rc) return rc;
    if (!grad_loss_dev) return fail(PSFS_E_ARG, "grad_loss is NULL");
    if (nvox(plan->grid) > 0 && !logits_dev) return fail(PSFS_E_ARG, "logits is NULL");
    if (plan->n > 0) {
        if (!gmean_dev || !gvar_dev || !gP_dev) return fail(PSFS_E_ARG, "gradient output array is NULL");
        if (!aligned(gP_dev, 4)) return fail(PSFS_E_ARG, "gP must be 4-byte aligned");
        for (int k = 0; k < plan->n; ++k)
            if (!gmean_dev[k] || !gvar_dev[k] || !aligned(gmean_dev[k], 16) || !aligned(gvar_dev[k], 16))
                return fail(PSFS_E_ARG, "gradient outputs of view %d must be 16-byte aligned device pointers", k);
    }
    if ((rc = check_device())) return rc;
    a.logits = const_cast<float *>(logits_dev);
    a.grad_loss = grad_loss_dev;
    ChainArgs c{};
    c.n = plan->n;
    c.adj = a.adj;
    c.grad_loss = grad_loss_dev;
    c.inv_count = a.inv_count;
    c.k0 = static_cast<float>(-1.5 * std::log(2.0 * M_PI) - static_cast<double>(plan->params.log_u));
    int64_t max_np = 0;
    for (int k = 0; k < plan->n; ++k) {
        const int64_t np = static_cast<int64_t>(plan->cams[k].width) * plan->cams[k].height;
        c.view[k] = ChainView{images_dev[k], plan->mean[k], plan->var[k], gmean_dev[k], gvar_dev[k], np, map_offset(plan, k)};
        if (np > max_np) max_np = np;
    }
    hipError_t e = launch_diff_backward(a, c, 2 * map_floats(plan), max_np, gP_dev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "differentiable backward launch");
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_tile_count(void) { return tile_count(); }

int psfs_tile_describe(int tile, int32_t *tx, int32_t *ty, int32_t *kz)
{
    if (tile < 0 || tile >= tile_count()) return fail(PSFS_E_RANGE, "tile %d outside 0..%d", tile, tile_count() - 1);
    const TileCfg &c = tile_cfg(tile);
    if (tx) *tx = c.tx;
    if (ty) *ty = c.ty;
    if (kz) *kz = c.kz;
    return PSFS_OK;
}

int psfs_set_tile(psfs_plan *plan, int tile)
{
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    if (tile < -1 || tile >= tile_count()) return fail(PSFS_E_RANGE, "tile %d outside -1..%d", tile, tile_count() - 1);
    plan->tile = tile;
    return PSFS_OK;
}

int psfs_get_tile(const psfs_plan *plan)
{
    if (!plan) return fail(PSFS_E_ARG, "plan is NULL");
    return plan->tile >= 0 ? plan->tile : default_tile();
}

size_t psfs_tune_workspace_bytes(const psfs_plan *plan)
{
    if (!plan || plan->n < 0 || !plan->has_grid) return 0;
    const size_t v = static_cast<size_t>(nvox(plan->grid));
    return align256(psfs_workspace_bytes(plan)) + align256(4 * v) + align256(v);
}

int psfs_tune(psfs_plan *plan, const uint8_t *const *images_dev, void *workspace_dev, size_t workspace_bytes,
              void *stream, int force, int *best_tile)
{
    PSFS_GUARD_BEGIN
    int rc = need_backgrounds(plan);
    if (rc) return rc;
    if ((rc = need_grid(plan))) return rc;
    if ((rc = check_images(plan, images_dev))) return rc;
    const size_t need = psfs_tune_workspace_bytes(plan);
    if (!workspace_dev || workspace_bytes < need || !aligned(workspace_dev, 256))
        return fail(PSFS_E_WORKSPACE, "tuning workspace needs %zu bytes, 256-byte aligned (got %zu)", need,
                    workspace_bytes);
    // cache key: device, CU count, sampling, grid edge class, view count, image class
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    if ((rc = check_device())) return rc;
    auto log2ceil = [](int64_t x) {
        int c = 0;
        while ((int64_t(1) << c) < x) ++c;
        return c;
    };
    int64_t edge = std::max({plan->grid.nx, plan->grid.ny, plan->grid.nz}), px = 1;
    for (int k = 0; k < plan->n; ++k) px = std::max<int64_t>(px, static_cast<int64_t>(plan->cams[k].width) * plan->cams[k].height);
    char key[160];
    std::snprintf(key, sizeof(key), "gfx950/%dcu/plan/s%d/e%d/n%d/i%d", cus, plan->params.sampling, log2ceil(edge),
                  plan->n, log2ceil(px));
    const std::string path = tune_cache_path();
    if (!force) {
        std::lock_guard<std::mutex> lock(tune_cache_mutex());
        const auto m = read_tune_cache(path);
        const auto it = m.find(key);
        if (it != m.end() && it->second >= 0 && it->second < tile_count()) {
            plan->tile = it->second;
            if (best_tile) *best_tile = it->second;
            return PSFS_OK;
        }
    }
    char *base = static_cast<char *>(workspace_dev);
    float *lmap = reinterpret_cast<float *>(base);
    const size_t v = static_cast<size_t>(nvox(plan->grid));
    float *post = reinterpret_cast<float *>(base + align256(psfs_workspace_bytes(plan)));
    uint8_t *occ = reinterpret_cast<uint8_t *>(base + align256(psfs_workspace_bytes(plan)) + align256(4 * v));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the maps do not depend on the tile: one likelihood pass, then each tile's fusion
    if ((rc = enqueue_likelihood(plan, images_dev, lmap, s))) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    const int keep = plan->tile;
    float best_ms = 1e30f;
    int best = default_tile();
    for (int t = 0; t < tile_count() && rc == PSFS_OK; ++t) {
        plan->tile = t;
        for (int w = 0; w < 2 && rc == PSFS_OK; ++w) rc = enqueue_fuse(plan, lmap, post, occ, s);
        if (rc) break;
        const int reps = 5;
        hipEventRecord(e0, s);
        for (int r = 0; r < reps && rc == PSFS_OK; ++r) rc = enqueue_fuse(plan, lmap, post, occ, s);
        hipEventRecord(e1, s);
        if (rc) break;
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) { rc = hip_fail(e, "hipEventSynchronize"); break; }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) {
        plan->tile = keep;
        return rc;
    }
    plan->tile = best;
    {
        std::lock_guard<std::mutex> lock(tune_cache_mutex());
        auto m = read_tune_cache(path);
        m[key] = best;
        write_tune_cache(path, m);
    }
    if (best_tile) *best_tile = best;
    return PSFS_OK;
    PSFS_GUARD_END
}

}  // extern "C"
