// Host side of the batched pass: frame validation, the launch-chain order,
// the device descriptor table, HIP-graph capture/replay and the tile
// autotuner with its on-disk cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "host_util.h"

using namespace psfs;
using namespace psfs::host;

struct psfs_batch {
    psfs_params params{};
    int device = -1;
    int cus = 0;
    int tile = 0;
    std::vector<psfs_frame> user;           // caller's frame structs (pointers to their arrays not kept)
    std::vector<int> order;                 // order[i] = user frame placed i-th in the chain (chain_order)
    std::vector<psfs_camera> cams;          // all cameras, user frame order
    std::vector<int> cam0;                  // first camera of each user frame
    std::vector<const uint8_t *> imgs;
    std::vector<const float *> means, vars;
    std::vector<BatchView> views;           // device table image (cost order)
    std::vector<BatchFrame> frames;
    std::vector<int64_t> slm_per_view;      // per table frame: likelihood workgroups per view
    std::vector<int64_t> fuse_tiles;        // per table frame: fusion bricks of the current tile
    int64_t map_floats = 0;
    void *dtable = nullptr;
    void *staging = nullptr;                // pinned host image of dtable
    size_t dtable_bytes = 0;
    bool dirty = true;
    hipEvent_t copied = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_ws = nullptr;
    int graph_tile = -1;
};

namespace {

int validate_frame(const psfs_frame &f, int idx)
{
    const psfs_grid &g = f.grid;
    if (g.nx < 0 || g.ny < 0 || g.nz < 0 || static_cast<int64_t>(g.nx) * g.ny * g.nz >= (int64_t(1) << 31))
        return fail(PSFS_E_RANGE, "frame %d: grid %dx%dx%d out of range", idx, g.nx, g.ny, g.nz);
    if (!(g.voxel > 0.0f) || !std::isfinite(g.voxel) || !finite_all(g.origin, 3))
        return fail(PSFS_E_RANGE, "frame %d: voxel size or origin invalid", idx);
    if (f.n < 1 || f.n > PSFS_MAX_VIEWS) return fail(PSFS_E_RANGE, "frame %d: view count %d outside 1..%d", idx, f.n, PSFS_MAX_VIEWS);
    if (!f.cams || !f.images_dev || !f.mean_dev || !f.var_dev) return fail(PSFS_E_ARG, "frame %d: NULL array", idx);
    for (int k = 0; k < f.n; ++k) {
        const psfs_camera &c = f.cams[k];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535 ||
            static_cast<int64_t>(c.width) * c.height >= (int64_t(1) << 30))
            return fail(PSFS_E_RANGE, "frame %d view %d: image size out of range", idx, k);
        if (!finite_all(c.P, 12)) return fail(PSFS_E_RANGE, "frame %d view %d: camera matrix not finite", idx, k);
        if (!f.images_dev[k] || !aligned(f.images_dev[k], 4)) return fail(PSFS_E_ARG, "frame %d view %d: image pointer NULL or misaligned", idx, k);
        if (!f.mean_dev[k] || !f.var_dev[k] || !aligned(f.mean_dev[k], 16) || !aligned(f.var_dev[k], 16))
            return fail(PSFS_E_ARG, "frame %d view %d: background pointers NULL or misaligned", idx, k);
    }
    if (static_cast<int64_t>(g.nx) * g.ny * g.nz > 0 && (!f.posterior_dev || !aligned(f.posterior_dev, 16)))
        return fail(PSFS_E_ARG, "frame %d: posterior must be a 16-byte aligned device pointer", idx);
    return PSFS_OK;
}

bool same_signature(const psfs_frame &a, const psfs_frame &b)
{
    if (a.grid.nx != b.grid.nx || a.grid.ny != b.grid.ny || a.grid.nz != b.grid.nz || a.n != b.n) return false;
    for (int k = 0; k < a.n; ++k)
        if (a.cams[k].width != b.cams[k].width || a.cams[k].height != b.cams[k].height) return false;
    return true;
}

// Order of the frames in the launch chain (launch i runs frame i's likelihood
// beside frame i-1's fusion). Costs in voxel-view units: fusion = voxels x
// views, likelihood = 4.4 per pixel (the measured ratio of likelihood time per
// pixel to fusion time per voxel-view). The chain starts with the cheapest
// likelihood and each next frame is the unplaced one whose likelihood cost is
// closest to the previous frame's fusion cost, so that the two halves of a
// launch are of similar length (2.79 ms instead of 2.85 for the 64 uneven
// frames against decreasing-cost order). Above kGreedyFrames frames (the
// greedy pass is quadratic) the order is decreasing fusion cost.
constexpr int kGreedyFrames = 4096;

void chain_order(const psfs_frame *frames, int nframes, std::vector<int> &order)
{
    std::vector<double> fuse(nframes), lik(nframes);
    for (int f = 0; f < nframes; ++f) {
        fuse[f] = static_cast<double>(frames[f].grid.nx) * frames[f].grid.ny * frames[f].grid.nz * frames[f].n;
        double px = 0.0;
        for (int k = 0; k < frames[f].n; ++k) px += static_cast<double>(frames[f].cams[k].width) * frames[f].cams[k].height;
        lik[f] = 4.4 * px;
    }
    order.resize(nframes);
    std::iota(order.begin(), order.end(), 0);
    if (nframes > kGreedyFrames) {
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return fuse[x] > fuse[y]; });
        return;
    }
    std::vector<char> used(nframes, 0);
    int cur = 0;
    for (int f = 1; f < nframes; ++f)
        if (lik[f] < lik[cur]) cur = f;
    for (int i = 0; i < nframes; ++i) {
        order[i] = cur;
        used[cur] = 1;
        int next = -1;
        for (int f = 0; f < nframes; ++f) {
            if (used[f]) continue;
            if (next < 0 || std::fabs(lik[f] - fuse[cur]) < std::fabs(lik[next] - fuse[cur])) next = f;
        }
        if (next < 0) break;
        cur = next;
    }
}

// Copies the caller's frames (and the arrays they point to) into the batch.
void take_frames(psfs_batch *b, int nframes, const psfs_frame *frames)
{
    b->user.assign(frames, frames + nframes);
    b->cams.clear(); b->cam0.clear(); b->imgs.clear(); b->means.clear(); b->vars.clear();
    for (int f = 0; f < nframes; ++f) {
        b->cam0.push_back(static_cast<int>(b->cams.size()));
        for (int k = 0; k < frames[f].n; ++k) {
            b->cams.push_back(frames[f].cams[k]);
            b->imgs.push_back(frames[f].images_dev[k]);
            b->means.push_back(frames[f].mean_dev[k]);
            b->vars.push_back(frames[f].var_dev[k]);
        }
    }
}

// Builds the descriptor table (and the per-frame launch sizes) for the
// current frames and tile.
void build_table(psfs_batch *b)
{
    const int nf = static_cast<int>(b->user.size());
    const bool nearest = b->params.sampling == PSFS_NEAREST;
    b->views.clear();
    b->frames.clear();
    b->slm_per_view.clear();
    b->fuse_tiles.clear();
    int64_t map_off = 0;
    for (int oi = 0; oi < nf; ++oi) {
        const int f = b->order[oi];
        const psfs_frame &u = b->user[f];
        BatchFrame fr{};
        fr.grid = GridDesc{u.grid.nx, u.grid.ny, u.grid.nz, u.grid.origin[0], u.grid.origin[1], u.grid.origin[2], u.grid.voxel};
        fr.n = u.n;
        fr.view0 = static_cast<int32_t>(b->views.size());
        fr.post = u.posterior_dev;
        fr.occ = u.occ_dev;
        int64_t max_np = 0;
        for (int k = 0; k < u.n; ++k) {
            const int ci = b->cam0[f] + k;
            const psfs_camera &c = b->cams[ci];
            BatchView v{};
            for (int e = 0; e < 12; ++e) v.g.P[e] = c.P[e];
            if (nearest) {
                for (int q = 0; q < 4; ++q) {
                    v.g.P[q] = static_cast<float>(static_cast<double>(c.P[q]) + 0.5 * c.P[8 + q]);
                    v.g.P[4 + q] = static_cast<float>(static_cast<double>(c.P[4 + q]) + 0.5 * c.P[8 + q]);
                }
            }
            v.g.W = c.width;
            v.g.H = c.height;
            v.g.map_off = map_off;
            v.img = b->imgs[ci];
            v.mean = b->means[ci];
            v.var = b->vars[ci];
            v.npix = static_cast<int64_t>(c.width) * c.height;
            max_np = std::max(max_np, v.npix);
            map_off += padded_pixels(c.width, c.height);
            b->views.push_back(v);
        }
        b->frames.push_back(fr);
        b->slm_per_view.push_back(batch_slm_blocks_per_view(max_np));
        b->fuse_tiles.push_back(batch_bricks(u.grid.nx, u.grid.ny, u.grid.nz, b->tile));
    }
    b->map_floats = map_off;
    b->dirty = true;
}

size_t workspace_bytes(const psfs_batch *b)
{
    return std::max<size_t>(256, align256(static_cast<size_t>(b->map_floats) * sizeof(float)));
}

void drop_graph(psfs_batch *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ws = nullptr;
    b->graph_tile = -1;
}

BatchArgs make_args(const psfs_batch *b, void *ws)
{
    BatchArgs a{};
    a.views = static_cast<const BatchView *>(b->dtable);
    a.frames = reinterpret_cast<const BatchFrame *>(static_cast<const char *>(b->dtable) +
                                                     align256(b->views.size() * sizeof(BatchView)));
    a.lmap = static_cast<float *>(ws);
    a.k0 = static_cast<float>(-1.5 * std::log(2.0 * M_PI) - static_cast<double>(b->params.log_u));
    const double pr = b->params.prior;
    a.L0 = static_cast<float>(std::log(pr / (1.0 - pr)));
    a.tau = b->params.threshold;
    return a;
}

int upload_table(psfs_batch *b, hipStream_t s)
{
    if (!b->dirty) return PSFS_OK;
    const size_t vb = align256(b->views.size() * sizeof(BatchView));
    // the previous upload must have finished reading the pinned staging copy
    hipError_t e = hipEventSynchronize(b->copied);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    char *st = static_cast<char *>(b->staging);
    std::memcpy(st, b->views.data(), b->views.size() * sizeof(BatchView));
    std::memcpy(st + vb, b->frames.data(), b->frames.size() * sizeof(BatchFrame));
    e = hipMemcpyAsync(b->dtable, st, b->dtable_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor table upload");
    e = hipEventRecord(b->copied, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    b->dirty = false;
    return PSFS_OK;
}

int check_run_args(psfs_batch *b, void *ws, size_t bytes)
{
    if (!b) return fail(PSFS_E_ARG, "batch is NULL");
    const size_t need = workspace_bytes(b);
    if (!ws || bytes < need || !aligned(ws, 256))
        return fail(PSFS_E_WORKSPACE, "batch workspace needs %zu bytes, 256-byte aligned (got %zu)", need, bytes);
    int rc = check_device();
    if (rc) return rc;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != b->device) return fail(PSFS_E_DEVICE, "batch was created on device %d, current device is %d", b->device, dev);
    return PSFS_OK;
}

// The launches of one run: table frame i's likelihood beside frame i-1's
// fusion, i = 0 .. nframes (one launch per step for tiles of 256 lanes, two
// for the 128-lane tile).
hipError_t enqueue_batch(const psfs_batch *b, void *ws, hipStream_t s)
{
    const BatchArgs a = make_args(b, ws);
    const int nf = static_cast<int>(b->frames.size());
    for (int i = 0; i <= nf; ++i) {
        const int fl = i < nf ? i : -1, ff = i - 1;
        hipError_t e = launch_batch_step(a, b->tile, b->params.sampling, fl, fl >= 0 ? b->slm_per_view[fl] : 0,
                                         fl >= 0 ? b->frames[fl].n : 0, ff, ff >= 0 ? b->fuse_tiles[ff] : 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int run_eager(psfs_batch *b, void *ws, hipStream_t s)
{
    hipError_t e = enqueue_batch(b, ws, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return PSFS_OK;
}

// ------------------------------------------------------------- tuning cache

std::string cache_key(const psfs_batch *b)
{
    // FNV-1a over the shape signature
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= static_cast<uint64_t>((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(static_cast<int64_t>(b->user.size()));
    for (size_t f = 0; f < b->user.size(); ++f) {
        const psfs_frame &u = b->user[f];
        mix(u.grid.nx); mix(u.grid.ny); mix(u.grid.nz); mix(u.n);
        for (int k = 0; k < u.n; ++k) {
            mix(b->cams[b->cam0[f] + k].width);
            mix(b->cams[b->cam0[f] + k].height);
        }
    }
    char buf[128];
    std::snprintf(buf, sizeof(buf), "gfx950/%dcu/chain/s%d/%016llx", b->cus, b->params.sampling,
                  static_cast<unsigned long long>(h));
    return buf;
}


}  // namespace

extern "C" {

int psfs_batch_create(psfs_batch **out, const psfs_params *params, int nframes, const psfs_frame *frames)
{
    PSFS_GUARD_BEGIN
    if (!out || !params) return fail(PSFS_E_ARG, "out or params is NULL");
    *out = nullptr;
    if (nframes < 1 || nframes > 65536) return fail(PSFS_E_RANGE, "frame count %d outside 1..65536", nframes);
    if (!frames) return fail(PSFS_E_ARG, "frames is NULL");
    if (!(params->prior > 0.0f && params->prior < 1.0f) || !std::isfinite(params->log_u) ||
        !(params->threshold >= 0.0f && params->threshold <= 1.0f))
        return fail(PSFS_E_RANGE, "params out of range");
    if (params->sampling != PSFS_NEAREST && params->sampling != PSFS_BILINEAR)
        return fail(PSFS_E_ARG, "unknown sampling %d", params->sampling);
    for (int f = 0; f < nframes; ++f) {
        int rc = validate_frame(frames[f], f);
        if (rc) return rc;
    }
    int rc = check_device();
    if (rc) return rc;
    psfs_batch *b = new psfs_batch();
    b->params = *params;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) { delete b; return hip_fail(e, "device query"); }
    take_frames(b, nframes, frames);
    chain_order(frames, nframes, b->order);
    b->tile = default_tile();
    build_table(b);
    b->dtable_bytes = align256(b->views.size() * sizeof(BatchView)) + align256(b->frames.size() * sizeof(BatchFrame));
    e = hipMalloc(&b->dtable, b->dtable_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&b->staging, b->dtable_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->copied, nullptr);
    if (e != hipSuccess) {
        if (b->dtable) hipFree(b->dtable);
        if (b->staging) hipHostFree(b->staging);
        if (b->copied) hipEventDestroy(b->copied);
        delete b;
        return hip_fail(e, "batch descriptor allocation");
    }
    *out = b;
    return PSFS_OK;
    PSFS_GUARD_END
}

size_t psfs_batch_workspace_bytes(const psfs_batch *batch)
{
    return batch ? workspace_bytes(batch) : 0;
}

int psfs_batch_update(psfs_batch *b, int nframes, const psfs_frame *frames)
{
    PSFS_GUARD_BEGIN
    if (!b || !frames) return fail(PSFS_E_ARG, "batch or frames is NULL");
    if (nframes != static_cast<int>(b->user.size()))
        return fail(PSFS_E_STALE, "frame count %d differs from the batch's %zu", nframes, b->user.size());
    for (int f = 0; f < nframes; ++f) {
        int rc = validate_frame(frames[f], f);
        if (rc) return rc;
        // compare against the stored copies (the caller's earlier arrays may be gone)
        psfs_frame stored = b->user[f];
        stored.cams = b->cams.data() + b->cam0[f];
        if (!same_signature(frames[f], stored)) return fail(PSFS_E_STALE, "frame %d changes the batch shape", f);
    }
    take_frames(b, nframes, frames);
    build_table(b);
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_batch_run(psfs_batch *b, void *workspace_dev, size_t workspace_bytes_, void *stream)
{
    PSFS_GUARD_BEGIN
    int rc = check_run_args(b, workspace_dev, workspace_bytes_);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = upload_table(b, s))) return rc;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    hipError_t e = s ? hipStreamIsCapturing(s, &st) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    // the null stream cannot be captured, and a caller's capture records the launches itself
    if (!s || st != hipStreamCaptureStatusNone) return run_eager(b, workspace_dev, s);
    if (!b->exec || b->graph_ws != workspace_dev || b->graph_tile != b->tile) {
        drop_graph(b);
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = enqueue_batch(b, workspace_dev, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (le != hipSuccess) { if (g) hipGraphDestroy(g); return hip_fail(le, "batch launch during capture"); }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_graph(b); return hip_fail(e, "hipGraphInstantiate"); }
        b->graph_ws = workspace_dev;
        b->graph_tile = b->tile;
    }
    e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return PSFS_OK;
    PSFS_GUARD_END
}

void psfs_batch_destroy(psfs_batch *b)
{
    if (!b) return;
    if (b->copied) {
        hipEventSynchronize(b->copied);
        hipEventDestroy(b->copied);
    }
    drop_graph(b);
    if (b->dtable) {
        hipDeviceSynchronize();
        hipFree(b->dtable);
    }
    if (b->staging) hipHostFree(b->staging);
    delete b;
}

int psfs_batch_set_tile(psfs_batch *b, int tile)
{
    PSFS_GUARD_BEGIN
    if (!b) return fail(PSFS_E_ARG, "batch is NULL");
    if (tile < -1 || tile >= tile_count()) return fail(PSFS_E_RANGE, "tile %d outside -1..%d", tile, tile_count() - 1);
    const int t = tile < 0 ? default_tile() : tile;
    if (t != b->tile) {
        b->tile = t;
        build_table(b);
    }
    return PSFS_OK;
    PSFS_GUARD_END
}

int psfs_batch_get_tile(const psfs_batch *b)
{
    if (!b) return fail(PSFS_E_ARG, "batch is NULL");
    return b->tile;
}

int psfs_batch_tune(psfs_batch *b, void *workspace_dev, size_t workspace_bytes_, void *stream, int force,
                    int *best_tile)
{
    PSFS_GUARD_BEGIN
    int rc = check_run_args(b, workspace_dev, workspace_bytes_);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string key = cache_key(b), path = tune_cache_path();
    if (!force) {
        std::lock_guard<std::mutex> lock(tune_cache_mutex());
        const auto m = read_tune_cache(path);
        const auto it = m.find(key);
        if (it != m.end() && it->second >= 0 && it->second < tile_count()) {
            if ((rc = psfs_batch_set_tile(b, it->second))) return rc;
            if (best_tile) *best_tile = it->second;
            return PSFS_OK;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    float best_ms = 1e30f;
    int best = b->tile;
    for (int t = 0; t < tile_count() && rc == PSFS_OK; ++t) {
        if ((rc = psfs_batch_set_tile(b, t))) break;
        if ((rc = upload_table(b, s))) break;
        for (int w = 0; w < 2 && rc == PSFS_OK; ++w) rc = run_eager(b, workspace_dev, s);
        if (rc) break;
        const int reps = 5;
        hipEventRecord(e0, s);
        for (int r = 0; r < reps && rc == PSFS_OK; ++r) rc = run_eager(b, workspace_dev, s);
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
    if (rc) return rc;
    if ((rc = psfs_batch_set_tile(b, best))) return rc;
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
