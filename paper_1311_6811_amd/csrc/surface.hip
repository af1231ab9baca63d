// The step after the posterior (Sec. 2.2.2, last paragraph; Sec. 3.3.3 steps
// d and e): smoothing of the occupancy probabilities, thresholding, and removal
// of the voxels inside the body, leaving the surface voxels as a compact list.
//   smooth_kernel          3x3x3 mean over the in-grid neighbours and the
//                          threshold in one traversal (the paper merges
//                          smoothing with voxel generation to save a round
//                          trip through memory)
//   surface_flag_kernel    surface flag of every voxel (occupied, with an
//                          unoccupied or out-of-grid face neighbour) and, per
//                          block of kSurfBlock consecutive voxels, their count
//                          (surface_flag_words_kernel: the same, four voxels
//                          per lane, when rows are whole 4-byte words)
//   surface_scan_kernel    (grids of more than kScanMin blocks) the block
//                          offsets: exclusive prefix of the counts, one
//                          workgroup
//   surface_write          the flagged voxels' linear indices at their place
//                          in the ascending list (block offset = sum of the
//                          earlier blocks' counts, summed by each block itself
//                          on smaller grids)
// The paper keeps inner-voxel removal on the CPU; here it is a deterministic
// two-kernel stream compaction over a flag grid.
#include "psfs_internal.h"

namespace psfs {
namespace {

constexpr int kTileY = 2;                           // rows per smoothing wave
constexpr int kTileZ = 2;                           // planes per smoothing wave
constexpr int kSurfBlock = 4096;                    // voxels per compaction block (16 per lane)
constexpr int kPerLane = kSurfBlock / 256;
constexpr int kScanThreads = 1024;
constexpr int kScanMin = 4096;                      // more blocks: offsets from surface_scan_kernel

__device__ __forceinline__ uint32_t byte_at(uint32_t w, int b) { return (w >> (8 * b)) & 0xffu; }

// 3x3x3 mean over the in-grid neighbours and threshold. A wave owns a tile of
// 64 x-columns (one per lane) by kTileY rows by kTileZ planes. Per plane it
// loads the x-windows of the kTileY + 2 rows it needs once (three loads each,
// a contiguous row of the wave per load), forms each row's 3 x 3 window sum
// (rows dy = -1..1, in each row dx = -1..1), and slides a sum of three planes
// along z. Out-of-grid cells are skipped and the sum is divided by the number
// of in-grid cells; every voxel's additions run in one fixed order.
template <int TY, int TZ>
__global__ __launch_bounds__(256) void smooth_kernel(SurfArgs a)
{
    const int nxb = (a.nx + 63) / 64, nyb = (a.ny + TY - 1) / TY;
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= static_cast<int64_t>(nxb) * nyb) return;            // whole waves
    const int y0 = static_cast<int>(tile / nxb) * TY;
    const int x = static_cast<int>(tile % nxb) * 64 + static_cast<int>(threadIdx.x & 63);
    if (x >= a.nx) return;
    const int z0 = static_cast<int>(blockIdx.y) * TZ;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    const bool xl = x > 0, xr = x + 1 < a.nx;
    // sum of the 3 x 3 window of every output row of the tile in plane z
    auto windows = [&](int z, float (&w)[TY]) {
        if (z < 0 || z >= a.nz) {
#pragma unroll
            for (int r = 0; r < TY; ++r) w[r] = 0.0f;
            return;
        }
        float row[TY + 2];
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
            const int y = y0 - 1 + r;
            row[r] = 0.0f;
            if (y < 0 || y >= a.ny) continue;
            const float *p = a.post + z * plane + static_cast<int64_t>(y) * a.nx + x;
            float t = p[0];
            if (xl) t = p[-1] + t;
            if (xr) t = t + p[1];
            row[r] = t;
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const int y = y0 + r;
            float s = 0.0f;
            if (y > 0) s += row[r];
            s += row[r + 1];
            if (y + 1 < a.ny) s += row[r + 2];
            w[r] = s;
        }
    };
    float wa[TY], wb[TY], wc[TY];
    windows(z0 - 1, wa);
    windows(z0, wb);
    const int cx = xl + 1 + xr;
#pragma unroll
    for (int q = 0; q < TZ; ++q) {
        const int z = z0 + q;
        windows(z + 1, wc);
        if (z < a.nz) {
            const int cz = (z > 0) + 1 + (z + 1 < a.nz);
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const int y = y0 + r;
                if (y >= a.ny) break;
                const int c = cx * ((y > 0) + 1 + (y + 1 < a.ny)) * cz;
                const float m = ((wa[r] + wb[r]) + wc[r]) / static_cast<float>(c);
                const int64_t idx = z * plane + static_cast<int64_t>(y) * a.nx + x;
                if (a.smoothed) a.smoothed[idx] = m;
                a.occ[idx] = m > a.tau ? 1 : 0;
            }
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            wa[r] = wb[r];
            wb[r] = wc[r];
        }
    }
}

// Surface flags of one compaction block and its count. Lane l of wave w
// tests voxels base + 256 r + 64 w + l (coalesced neighbour loads); the
// lane's (i, j, k) is divided out once and then advanced by 256 voxels per
// step with the carries the host precomputed.
__global__ __launch_bounds__(256) void surface_flag_kernel(SurfArgs a)
{
    __shared__ int part[4];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSurfBlock;
    const int64_t v0 = base + threadIdx.x;
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    int k = static_cast<int>(v0 / plane);
    const int64_t rem = v0 - static_cast<int64_t>(k) * plane;
    int j = static_cast<int>(rem / a.nx);
    int i = static_cast<int>(rem - static_cast<int64_t>(j) * a.nx);
    int c = 0;
#pragma unroll
    for (int r = 0; r < kPerLane; ++r) {
        const int64_t v = v0 + 256 * r;
        if (v < a.nvox) {
            // all seven loads at in-grid addresses (a face on the grid's border
            // reads the voxel itself, the border test decides there), issued
            // together rather than one after another
            const bool border = (i == 0) | (i + 1 == a.nx) | (j == 0) | (j + 1 == a.ny) | (k == 0) | (k + 1 == a.nz);
            const uint8_t o = a.occ[v];
            const uint8_t xm = a.occ[i > 0 ? v - 1 : v], xp = a.occ[i + 1 < a.nx ? v + 1 : v];
            const uint8_t ym = a.occ[j > 0 ? v - a.nx : v], yp = a.occ[j + 1 < a.ny ? v + a.nx : v];
            const uint8_t zm = a.occ[k > 0 ? v - plane : v], zp = a.occ[k + 1 < a.nz ? v + plane : v];
            const bool hole = (xm == 0) | (xp == 0) | (ym == 0) | (yp == 0) | (zm == 0) | (zp == 0);
            const bool surf = (o != 0) & (border | hole);
            a.flags[v] = surf ? 1 : 0;
            c += surf;
        }
        i += a.step_i;
        if (i >= a.nx) {
            i -= a.nx;
            ++j;
        }
        j += a.step_j;
        if (j >= a.ny) {
            j -= a.ny;
            ++k;
        }
        k += a.step_k;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Surface flags four voxels at a time, when nx is a multiple of 4 and the
// occupancy and flag arrays are 4-byte aligned: lane l of wave w tests the
// four voxels of word g = block * 1024 + 256 r + 64 w + l (one row, one
// plane). Their x-neighbours are in the same word or in the adjacent words of
// the row, their y- and z-neighbours in the words nx / 4 and nx * ny / 4 away;
// seven word loads at clamped in-grid addresses (the border tests decide for
// faces on the grid's border), one word store of four flags.
__global__ __launch_bounds__(256) void surface_flag_words_kernel(SurfArgs a)
{
    __shared__ int part[4];
    const uint32_t *occ = reinterpret_cast<const uint32_t *>(a.occ);
    uint32_t *flags = reinterpret_cast<uint32_t *>(a.flags);
    const int64_t plane = static_cast<int64_t>(a.nx) * a.ny;
    const int64_t nwords = a.nvox / 4, rw = a.nx / 4, pw = plane / 4;
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * (kSurfBlock / 4) + threadIdx.x;
    int c = 0;
#pragma unroll
    for (int r = 0; r < kSurfBlock / 4 / 256; ++r) {
        const int64_t g = g0 + 256 * r;
        if (g < nwords) {
            const int64_t v0 = 4 * g;
            const int k = static_cast<int>(v0 / plane);
            const int64_t rem = v0 - static_cast<int64_t>(k) * plane;
            const int j = static_cast<int>(rem / a.nx), i0 = static_cast<int>(rem - static_cast<int64_t>(j) * a.nx);
            const uint32_t C = occ[g];
            const uint32_t L = occ[i0 > 0 ? g - 1 : g], R = occ[i0 + 4 < a.nx ? g + 1 : g];
            const uint32_t YM = occ[j > 0 ? g - rw : g], YP = occ[j + 1 < a.ny ? g + rw : g];
            const uint32_t ZM = occ[k > 0 ? g - pw : g], ZP = occ[k + 1 < a.nz ? g + pw : g];
            const bool border_yz = (j == 0) | (j + 1 == a.ny) | (k == 0) | (k + 1 == a.nz);
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t o = byte_at(C, b);
                const uint32_t xm = b > 0 ? byte_at(C, b - 1) : byte_at(L, 3);
                const uint32_t xp = b < 3 ? byte_at(C, b + 1) : byte_at(R, 0);
                const bool border = border_yz | (b == 0 && i0 == 0) | (b == 3 && i0 + 4 == a.nx);
                const uint32_t ym = byte_at(YM, b), yp = byte_at(YP, b), zm = byte_at(ZM, b), zp = byte_at(ZP, b);
                const bool hole = (xm == 0) | (xp == 0) | (ym == 0) | (yp == 0) | (zm == 0) | (zp == 0);
                const bool surf = (o != 0) & (border | hole);
                word |= (surf ? 1u : 0u) << (8 * b);
                c += surf;
            }
            flags[g] = word;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Lane l of a compaction block owns its 16 consecutive voxels
// base + 16 l .. base + 16 l + 15 (one 16-byte load of flags).
__device__ __forceinline__ uint32_t lane_flags(const SurfArgs &a, int64_t base)
{
    const int64_t v = base + 16 * static_cast<int64_t>(threadIdx.x);
    uint32_t bits = 0;
    if (v + 16 <= a.nvox) {
        const uint4 w = *reinterpret_cast<const uint4 *>(a.flags + v);
        const uint32_t word[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if ((word[q >> 2] >> (8 * (q & 3))) & 0xffu) bits |= 1u << q;
    } else {
        for (int q = 0; q < 16 && v + q < a.nvox; ++q)
            if (a.flags[v + q]) bits |= 1u << q;
    }
    return bits;
}

// Inclusive sum over the block's 256 lanes in lane order (wave scans + the
// totals of the waves before).
__device__ __forceinline__ int block_inclusive_scan(int x, int *wave_tot)
{
    const int lane = static_cast<int>(threadIdx.x & 63), w = static_cast<int>(threadIdx.x >> 6);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wave_tot[w] = x;
    __syncthreads();
    for (int q = 0; q < w; ++q) x += wave_tot[q];
    return x;
}

// Exclusive prefix of the block counts, written over them as offsets, and the
// total: one workgroup; thread t owns a contiguous range of blocks, so the
// additions run in block order within a range and in thread order across the
// ranges (offsets are below nvox < 2^31).
__global__ __launch_bounds__(kScanThreads) void surface_scan_kernel(SurfArgs a)
{
    __shared__ int64_t part[kScanThreads];
    const int t = static_cast<int>(threadIdx.x);
    const int64_t per = (static_cast<int64_t>(a.nblocks) + kScanThreads - 1) / kScanThreads;
    const int64_t lo = t * per < a.nblocks ? t * per : a.nblocks;
    const int64_t hi = lo + per < a.nblocks ? lo + per : a.nblocks;
    int64_t s = 0;
    for (int64_t q = lo; q < hi; ++q) s += a.counts[q];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t add = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t q = lo; q < hi; ++q) {
        const int32_t c = a.counts[q];
        a.counts[q] = static_cast<int32_t>(run);
        run += c;
    }
    if (t == kScanThreads - 1) *a.count = part[t];
}

// Block b's offset summed by the block itself over the earlier blocks' counts
// (and, in block 0, the total into *count); every thread of the block calls it.
__device__ __forceinline__ int64_t own_block_offset(const SurfArgs &a, int b, int64_t *red)
{
    int64_t s = 0, tot = 0;
    for (int q = static_cast<int>(threadIdx.x); q < a.nblocks; q += 256) {
        if (q < b) s += a.counts[q];
        tot += a.counts[q];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const int64_t off = red[0];
    __syncthreads();
    if (b == 0) {
        red[threadIdx.x] = tot;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.count = red[0];
    }
    return off;
}

// scanned: the counts already hold the block offsets (surface_scan_kernel)
__global__ __launch_bounds__(256) void surface_write_kernel(SurfArgs a, int scanned)
{
    __shared__ int64_t red[256];
    __shared__ int wave_tot[4];
    const int b = static_cast<int>(blockIdx.x);
    const int64_t block_off = scanned ? static_cast<int64_t>(a.counts[b]) : own_block_offset(a, b, red);
    const int64_t base = static_cast<int64_t>(b) * kSurfBlock;
    uint32_t bits = lane_flags(a, base);
    const int c = __popc(bits);
    int64_t pos = block_off + (block_inclusive_scan(c, wave_tot) - c);
    const int64_t v0 = base + 16 * static_cast<int64_t>(threadIdx.x);
    while (bits) {
        const int q = __ffs(bits) - 1;
        bits &= bits - 1;
        if (pos < a.capacity) a.out[pos] = static_cast<int32_t>(v0 + q);
        ++pos;
    }
}

__global__ void zero_count_kernel(int64_t *count)
{
    if (threadIdx.x == 0) *count = 0;
}

}  // namespace

int64_t surface_blocks(int64_t nvox) { return (nvox + kSurfBlock - 1) / kSurfBlock; }

hipError_t launch_surface(const SurfArgs &a, hipStream_t s)
{
    if (a.nvox == 0) {
        hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, a.count);
        return hipGetLastError();
    }
    const int64_t tiles = static_cast<int64_t>((a.nx + 63) / 64) * ((a.ny + kTileY - 1) / kTileY);
    const dim3 sg(static_cast<unsigned>((tiles + 3) / 4), static_cast<unsigned>((a.nz + kTileZ - 1) / kTileZ));
    hipLaunchKernelGGL((smooth_kernel<kTileY, kTileZ>), sg, dim3(256), 0, s, a);
    const bool words = a.nx % 4 == 0 && reinterpret_cast<uintptr_t>(a.occ) % 4 == 0 &&
                       reinterpret_cast<uintptr_t>(a.flags) % 4 == 0;
    if (words)
        hipLaunchKernelGGL(surface_flag_words_kernel, dim3(static_cast<unsigned>(a.nblocks)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(surface_flag_kernel, dim3(static_cast<unsigned>(a.nblocks)), dim3(256), 0, s, a);
    const int scanned = a.nblocks > kScanMin ? 1 : 0;
    if (scanned) hipLaunchKernelGGL(surface_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a);
    hipLaunchKernelGGL(surface_write_kernel, dim3(static_cast<unsigned>(a.nblocks)), dim3(256), 0, s, a, scanned);
    return hipGetLastError();
}

}  // namespace psfs
