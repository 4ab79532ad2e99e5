// bcf_cps.hip -- colored prefix sums on gfx950, the paper's example of how
// shared-memory bank conflicts decide a kernel's runtime (Sitchinava &
// Weichert, Sec. 1.2 and the appendix on colored prefix sums).
//
// out[i] = sum of values[j] over j <= i with colors[j] == colors[i] (inclusive,
// modulo 2^32), for d <= 32 colors, by the paper's three phases:
//   1. every work-group reduces its tile (a contiguous range, processed in
//      pages of 8192 elements) to d per-color sums;
//   2. one work-group per color scans those sums over the tiles: each tile's
//      starting offset per color;
//   3. every work-group scans its tile page by page: each thread counts the
//      32 consecutive elements it owns per color, the counts are scanned over
//      the threads per color (the intra-page offsets), and each thread then
//      walks its elements again with running per-color sums.
// The per-thread, per-color counters live in LDS (their color index is data,
// so they cannot be registers).  CF = false keeps a thread's d counters
// consecutive (word t * d + c): in one step the 32 lanes of a half-wave touch
// words t * d + c_t, whose banks collide more the larger d is -- the layout
// whose runtime grows with d in the paper.  CF = true stores them color-major
// (word c * 256 + t): lane t always hits bank t mod 32, whatever the colors,
// so every counter access is conflict-free, and the scans over threads run in
// registers (DPP row shifts and lane reads) instead of through a transposed
// LDS matrix.  The counters take 256 * d words of dynamic LDS, so small d
// leaves room for more resident work-groups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bcf.h"

namespace {

constexpr int kThreads = 256;  // four waves per work-group
constexpr int kWaves = kThreads / 64;
constexpr int kPerThread = 32;  // consecutive elements a thread owns in a page
constexpr int kPage = kThreads * kPerThread;
constexpr uint32_t kMaxColors = 32;
constexpr uint64_t kMaxTiles = 2048;

template <bool CF>
__device__ __forceinline__ uint32_t slot(uint32_t t, uint32_t c, uint32_t d)
{
    return CF ? c * kThreads + t : t * d + c;
}

__device__ __forceinline__ uint32_t color_of(uint32_t c, uint32_t d) { return c < d ? c : d - 1; }

// The kPerThread elements thread t owns in the page starting at `page` (< hi),
// with 16-byte loads when all are in range (the arrays are 16-byte aligned).
__device__ __forceinline__ void load_chunk(const uint32_t *values, const uint8_t *colors, uint64_t page,
                                           uint64_t hi, uint32_t t, uint32_t (&v)[kPerThread],
                                           uint32_t (&c)[kPerThread], uint32_t &valid)
{
    const uint64_t base = page + (uint64_t)t * kPerThread;
    if (base + kPerThread <= hi) {
        valid = kPerThread;
        const uint4 *vp = reinterpret_cast<const uint4 *>(values + base);
#pragma unroll
        for (int q = 0; q < kPerThread / 4; ++q) {
            const uint4 x = vp[q];
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
        const uint4 *cp = reinterpret_cast<const uint4 *>(colors + base);
#pragma unroll
        for (int q = 0; q < kPerThread / 16; ++q) {
            const uint4 cc = cp[q];
            const uint32_t w[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
            for (int i = 0; i < 16; ++i)
                c[16 * q + i] = (w[i / 4] >> (8 * (i % 4))) & 0xffu;
        }
    } else {
        valid = base < hi ? (uint32_t)(hi - base) : 0u;
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            const bool in = (uint32_t)i < valid;
            v[i] = in ? values[base + i] : 0u;
            c[i] = in ? colors[base + i] : 0u;
        }
    }
}

// Sum of x over the 64 lanes of the wave.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int k = 32; k >= 1; k /= 2)
        x += (uint32_t)__shfl_xor((int)x, k);
    return x;
}

// Inclusive prefix sum of x over the lanes of the wave, without LDS: a
// Kogge-Stone scan inside each row of 16 lanes by DPP row shifts (lanes with
// no source read 0), then each row adds the totals of the rows before it,
// read from lanes 15, 31 and 47.
__device__ __forceinline__ uint32_t wave_scan(uint32_t x, uint32_t lane)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
    const uint32_t row = lane >> 4;
    return x + (row > 0 ? r0 : 0u) + (row > 1 ? r1 : 0u) + (row > 2 ? r2 : 0u);
}

// Phase 1: per-color sums of tile b = [b * tile, min((b + 1) * tile, n)).
template <bool CF>
__global__ __launch_bounds__(kThreads) void k_cps_tile_sums(const uint32_t *values, const uint8_t *colors, uint64_t n,
                                                            uint32_t d, uint64_t tile, uint32_t *sums)
{
    extern __shared__ uint32_t cnt[];  // kThreads * d counters
    __shared__ uint32_t part[kWaves][kMaxColors];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t / 64;
    const uint64_t lo = (uint64_t)blockIdx.x * tile, hi = lo + tile < n ? lo + tile : n;
    for (uint32_t c = 0; c < d; ++c)
        cnt[slot<CF>(t, c, d)] = 0;
    for (uint64_t page = lo; page < hi; page += kPage) {
        uint32_t v[kPerThread], col[kPerThread], valid;
        load_chunk(values, colors, page, hi, t, v, col, valid);
#pragma unroll
        for (int i = 0; i < kPerThread; ++i)
            if ((uint32_t)i < valid)
                cnt[slot<CF>(t, color_of(col[i], d), d)] += v[i];
    }
    for (uint32_t c = 0; c < d; ++c) {
        const uint32_t s = wave_sum(cnt[slot<CF>(t, c, d)]);
        if (lane == 0)
            part[wave][c] = s;
    }
    __syncthreads();
    if (t < d) {
        uint32_t s = 0;
        for (int w = 0; w < kWaves; ++w)
            s += part[w][t];
        sums[(uint64_t)blockIdx.x * d + t] = s;
    }
}

// Phase 2: work-group c turns the tile sums of color c into exclusive offsets.
__global__ __launch_bounds__(kThreads) void k_cps_tile_offsets(const uint32_t *sums, uint32_t *offsets,
                                                               uint32_t tiles, uint32_t d)
{
    __shared__ uint32_t wtot[kWaves];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t / 64, c = blockIdx.x;
    const uint32_t per = (tiles + kThreads - 1) / kThreads;  // consecutive tiles per thread
    const uint32_t b0 = t * per, b1 = b0 + per < tiles ? b0 + per : tiles;
    uint32_t local = 0;
    for (uint32_t b = b0; b < b1; ++b)
        local += sums[(uint64_t)b * d + c];
    const uint32_t incl = wave_scan(local, lane);
    if (lane == 63)
        wtot[wave] = incl;
    __syncthreads();
    uint32_t run = incl - local;
    for (uint32_t w = 0; w < wave; ++w)
        run += wtot[w];
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t s = sums[(uint64_t)b * d + c];
        offsets[(uint64_t)b * d + c] = run;
        run += s;
    }
}

// Phase 3: the colored prefix sums of tile b, seeded with its offsets.
template <bool CF>
__global__ __launch_bounds__(kThreads) void k_cps_scan(const uint32_t *values, const uint8_t *colors, uint32_t *out,
                                                       uint64_t n, uint32_t d, uint64_t tile, const uint32_t *offsets)
{
    extern __shared__ uint32_t cnt[];  // kThreads * d counters
    __shared__ uint32_t wtot[kWaves][kMaxColors];
    __shared__ uint32_t carry[kMaxColors];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t / 64;
    const uint64_t lo = (uint64_t)blockIdx.x * tile, hi = lo + tile < n ? lo + tile : n;
    if (t < d)
        carry[t] = offsets[(uint64_t)blockIdx.x * d + t];
    for (uint64_t page = lo; page < hi; page += kPage) {
        uint32_t v[kPerThread], col[kPerThread], valid;
        load_chunk(values, colors, page, hi, t, v, col, valid);
#pragma unroll
        for (int i = 0; i < kPerThread; ++i)
            col[i] = color_of(col[i], d);
        // this thread's per-color sums of its kPerThread elements
        for (uint32_t c = 0; c < d; ++c)
            cnt[slot<CF>(t, c, d)] = 0;
#pragma unroll
        for (int i = 0; i < kPerThread; ++i)
            if ((uint32_t)i < valid)
                cnt[slot<CF>(t, col[i], d)] += v[i];
        // exclusive scan over the threads, per color: within the wave in
        // registers, then across the four waves
        for (uint32_t c = 0; c < d; ++c) {
            const uint32_t x = cnt[slot<CF>(t, c, d)];
            const uint32_t incl = wave_scan(x, lane);
            cnt[slot<CF>(t, c, d)] = incl - x;
            if (lane == 63)
                wtot[wave][c] = incl;
        }
        __syncthreads();
        for (uint32_t c = 0; c < d; ++c) {
            uint32_t base = carry[c];
            for (uint32_t w = 0; w < wave; ++w)
                base += wtot[w][c];
            cnt[slot<CF>(t, c, d)] += base;
        }
        __syncthreads();
        if (t < d) {
            uint32_t s = 0;
            for (int w = 0; w < kWaves; ++w)
                s += wtot[w][t];
            carry[t] += s;
        }
        // running sums over this thread's elements
        const uint64_t base = page + (uint64_t)t * kPerThread;
        uint32_t r[kPerThread];
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            const uint32_t s = slot<CF>(t, col[i], d);
            const uint32_t x = cnt[s] + v[i];
            if ((uint32_t)i < valid)
                cnt[s] = x;
            r[i] = x;
        }
        if (valid == kPerThread) {
            uint4 *op = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
            for (int q = 0; q < kPerThread / 4; ++q)
                op[q] = make_uint4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
        } else {
#pragma unroll
            for (int i = 0; i < kPerThread; ++i)
                if ((uint32_t)i < valid)
                    out[base + i] = r[i];
        }
        __syncthreads();  // the next page reuses the counters and wtot
    }
}

// Tiles of a call over n > 0 elements: at most kMaxTiles, each a multiple of a
// page (kPage elements).
void tiling(uint64_t n, uint64_t &tiles, uint64_t &tile)
{
    const uint64_t pages = (n + kPage - 1) / kPage;
    const uint64_t per = (pages + kMaxTiles - 1) / kMaxTiles;  // pages per tile
    tile = per * kPage;
    tiles = (n + tile - 1) / tile;
}

}  // namespace

extern "C" bcf_status bcf_colored_prefix_sums(const uint32_t *values, const uint8_t *colors, uint32_t *out,
                                              uint64_t n, uint32_t d, int conflict_free, void *temp,
                                              uint64_t *temp_bytes, void *stream)
{
    if (!temp_bytes || d == 0 || d > kMaxColors || n > 0xffffffffull)
        return BCF_ERR_INVALID;
    if (n == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    uint64_t tiles = 0, tile = 0;
    tiling(n, tiles, tile);
    const uint64_t sums_bytes = (tiles * d * 4 + 255) / 256 * 256;
    const uint64_t need = 2 * sums_bytes;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (!values || !colors || !out)
        return BCF_ERR_INVALID;
    if (((reinterpret_cast<uintptr_t>(values) | reinterpret_cast<uintptr_t>(colors) |
          reinterpret_cast<uintptr_t>(out)) & 15) != 0)
        return BCF_ERR_INVALID;  // 16-byte accesses
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *sums = static_cast<uint32_t *>(temp);
    uint32_t *offsets = reinterpret_cast<uint32_t *>(static_cast<char *>(temp) + sums_bytes);
    const dim3 grid((uint32_t)tiles), block(kThreads);
    const size_t lds = (size_t)kThreads * d * sizeof(uint32_t);
    if (conflict_free)
        hipLaunchKernelGGL(k_cps_tile_sums<true>, grid, block, lds, s, values, colors, n, d, tile, sums);
    else
        hipLaunchKernelGGL(k_cps_tile_sums<false>, grid, block, lds, s, values, colors, n, d, tile, sums);
    hipLaunchKernelGGL(k_cps_tile_offsets, dim3(d), block, 0, s, sums, offsets, (uint32_t)tiles, d);
    if (conflict_free)
        hipLaunchKernelGGL(k_cps_scan<true>, grid, block, lds, s, values, colors, out, n, d, tile, offsets);
    else
        hipLaunchKernelGGL(k_cps_scan<false>, grid, block, lds, s, values, colors, out, n, d, tile, offsets);
    return hipGetLastError() == hipSuccess ? BCF_OK : BCF_ERR_DEVICE;
}
