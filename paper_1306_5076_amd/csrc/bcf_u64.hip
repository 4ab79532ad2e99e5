// bcf_u64.hip -- sort of unsigned 64-bit keys (an extension: the paper sorts
// 32-bit keys) on the same design as the 32-bit sort, with a key held in a
// register pair and compared as one 64-bit integer.
//
// * Block sort (the paper's base case, Sec. 3.1, as the 32-bit wave tiles do
//   it): a wave holds a 64 x 64 tile of keys, 64 per lane.  Each lane sorts
//   its line with Batcher's odd-even merge sort, lines alternating direction,
//   then six bitonic merge rounds turn the 64 lines into one sorted run of
//   4096 keys.  Every compare-exchange is between two registers of one lane;
//   the switches between the STRIDED and BLOCKED layouts go through LDS as
//   two 32-bit halves, each with the conflict-free 68-word rows of the 32-bit
//   tiles.  Above 2^19 keys four waves of a work-group then merge their
//   sorted sub-tiles in two more rounds through the shared CROSS layout (the
//   group tiles of the 32-bit sort), for runs of 16384 keys: two merge passes
//   fewer.
// * Merge passes (Sec. 3.2, binary merging): every wave produces one
//   4096-key output tile of one merge of two runs.  Its two half-waves find
//   the co-ranks of the tile's first and last output (the merge-path split,
//   exact whatever the duplicates), the A piece is loaded ascending and the B
//   piece reversed into one bitonic tile, a half-cleaner network sorts it
//   (register bits of the STRIDED layout, transpose, those of the BLOCKED
//   layout) and the tile is stored coalesced.  Passes ping-pong between the
//   output and temp so that the last one writes the output.
// Keys only: equal keys are indistinguishable, so the order among them needs
// no tie-break.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bcf.h"
#include "bcf_device.hpp"

namespace bcf {

// Host services of bcf_api.hip: a profiling scope around one launch.
void *prof_begin(const char *name, hipStream_t s, double bytes);
void prof_end(void *scope);

namespace {

constexpr uint64_t kMaxN64 = 0xFFFFFFFFull;

// STRIDED tile of `count` keys from src (position p = 64 r + lane), padding
// with the maximum key (never stored).
__device__ __forceinline__ void load_tile64(Lines64 &t, const uint64_t *__restrict__ src, uint32_t count,
                                            uint32_t lane)
{
    if (count >= (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kLine; ++r)
            t.e[r] = src[kWave * r + lane];
        return;
    }
    const uint32_t last = count ? count - 1 : 0;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        const uint64_t k = count ? src[p < count ? p : last] : kMaxKey64;  // clamped: a valid address
        t.e[r] = p < count ? k : kMaxKey64;
    }
}

// Loads and stores of a pass, with the nontemporal hint when the pass
// streams more than the last-level cache holds (below that the next pass
// finds its input there).
template <bool NT>
__device__ __forceinline__ uint64_t ld64(const uint64_t *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void store_tile64(const Lines64 &t, uint64_t *__restrict__ dst, uint32_t count,
                                             uint32_t lane)
{
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        if (p < count) {
            if constexpr (NT)
                __builtin_nontemporal_store(t.e[r], dst + p);
            else
                dst[p] = t.e[r];
        }
    }
}

// Round J (1..6) of the tile sort: pairs of sorted runs of 2^(5+J) positions,
// alternating in direction, become runs of 2^(6+J).  Position bits 5+J..6 are
// register bits in STRIDED layout (direction: register bit J), bits 5..0 in
// BLOCKED layout (direction: lane bit J, applied by complementing).
template <int J>
__device__ __forceinline__ void merge_round64(Lines64 &t, uint32_t *lds, uint32_t lane)
{
    to_strided(t, lds, lane);
    half_clean_lines<(1 << (J - 1)), (J < 6 ? J : -1)>(t);
    to_blocked(t, lds, lane);
    if constexpr (J < 6)
        flip(t, lane >> J);
    half_clean_lines<kLine / 2, -1>(t);
    if constexpr (J < 6)
        flip(t, lane >> J);
}

// Sort a wave tile: on entry as loaded (read as BLOCKED: lane l's line), on
// exit sorted in BLOCKED layout.
__device__ __forceinline__ void sort_tile_blocked64(Lines64 &t, uint32_t *lds, uint32_t lane)
{
    flip(t, lane);  // lines: even lanes ascending, odd lanes descending
    oe_sort_lines<0, kLine - 1>(t);
    flip(t, lane);
    merge_round64<1>(t, lds, lane);
    merge_round64<2>(t, lds, lane);
    merge_round64<3>(t, lds, lane);
    merge_round64<4>(t, lds, lane);
    merge_round64<5>(t, lds, lane);
    merge_round64<6>(t, lds, lane);
}

constexpr int kGroupWaves64 = 4;  // group tiles of 16384 keys
constexpr uint64_t kGroupMinN64 = 1ull << 19;

// One 4096-key tile per wave, one wave per work-group.
template <bool NT>
__global__ __launch_bounds__(kWave) void k_u64_block_sort(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                          uint64_t n)
{
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    const uint32_t lane = threadIdx.x;
    const uint64_t start = (uint64_t)blockIdx.x * kTile;
    if (start >= n)
        return;
    const uint32_t count = n - start < (uint64_t)kTile ? (uint32_t)(n - start) : (uint32_t)kTile;
    Lines64 t;
    load_tile64(t, in + start, count, lane);
    sort_tile_blocked64(t, lds, lane);
    to_strided(t, lds, lane);
    store_tile64<NT>(t, out + start, count, lane);
}

// One group tile of kGroupWaves64 sub-tiles per work-group: each wave sorts
// its sub-tile (odd waves descending, by complementing around the sort), then
// the group rounds merge across the waves.  Every wave of a work-group reaches
// the same barriers: waves whose sub-tile lies past the end hold padding only.
template <bool NT>
__global__ __launch_bounds__(kWave *kGroupWaves64) void k_u64_block_sort_group(const uint64_t *__restrict__ in,
                                                                             uint64_t *__restrict__ out, uint64_t n)
{
    __shared__ __align__(16) uint32_t lds[kGroupWaves64 * kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t gstart = (uint64_t)blockIdx.x * (kGroupWaves64 * kTile);
    if (gstart >= n)
        return;
    const uint64_t start = gstart + (uint64_t)wave * kTile;
    const uint32_t count = start >= n ? 0u : (n - start < (uint64_t)kTile ? (uint32_t)(n - start) : (uint32_t)kTile);
    Lines64 t;
    load_tile64(t, in + start, count, lane);  // count 0: padding only, nothing loaded
    uint32_t *own = lds + kLdsWords * wave;
    flip(t, wave);
    sort_tile_blocked64(t, own, lane);
    flip(t, wave);
    group_rounds<kGroupWaves64, 7>(t, lds, lane, wave);
    to_strided(t, own, lane);
    store_tile64<NT>(t, out + start, count, lane);
}

// Output tile t of a binary pass over runs of `run` keys (a multiple of
// 4096): runs 2s and 2s+1 merge into [2s run, min(2(s+1) run, n)).
template <bool NT>
__global__ __launch_bounds__(kWave) void k_u64_merge(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                                     uint64_t n, uint64_t run)
{
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    const uint32_t lane = threadIdx.x;
    const uint64_t gstart = (uint64_t)blockIdx.x * kTile;
    if (gstart >= n)
        return;
    const uint64_t base = gstart / (2 * run) * (2 * run);
    const uint64_t rem = n - base;
    const uint32_t na = (uint32_t)(rem < run ? rem : run);
    const uint32_t nb = (uint32_t)(rem - na < run ? rem - na : run);
    const uint32_t d0 = (uint32_t)(gstart - base);
    const uint32_t count = na + nb - d0 < (uint32_t)kTile ? na + nb - d0 : (uint32_t)kTile;
    const uint64_t *A = src + base, *B = A + na;
    // lanes 0..31: co-rank of the tile's first output, 32..63: of its end
    const uint32_t d = lane < 32 ? d0 : d0 + count;
    const uint32_t split = corank_halfwave(A, na, B, nb, d, lane);
    const uint32_t a0 = __builtin_amdgcn_readlane(split, 0), a1 = __builtin_amdgcn_readlane(split, 32);
    const uint32_t pa = a1 - a0, pb = count - pa;
    // A piece ascending at [0, pa), B piece reversed at [4096 - pb, 4096):
    // position p reads pA[p] or pA[bend - p], the B piece lying dB keys after
    // the A piece; one 32-bit offset per register, every load issued before
    // any is used
    const uint64_t *pA = A + a0;
    const uint32_t dB = na - a0 + (d0 - a0);
    const uint32_t bend = dB + (kTile - 1);
    const uint32_t bstart = kTile - pb;
    Lines64 t;
    if (count == (uint32_t)kTile) {
        // full tile: every position is in A or in B, no select after a load
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            t.e[r] = ld64<NT>(pA + (p < pa ? p : bend - p));
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            const bool in_a = p < pa, in_b = p >= bstart;
            const uint64_t k = ld64<NT>(pA + (in_a ? p : (in_b ? bend - p : 0u)));
            t.e[r] = (in_a || in_b) ? k : kMaxKey64;
        }
    }
    half_clean_lines<kLine / 2, -1>(t);  // position bits 11..6
    to_blocked(t, lds, lane);
    half_clean_lines<kLine / 2, -1>(t);  // position bits 5..0
    to_strided(t, lds, lane);
    store_tile64<NT>(t, dst + gstart, count, lane);
}

uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }

// Run length after the block sort, and the binary merge passes after it.
uint64_t run0_for(uint64_t n) { return n > kGroupMinN64 ? (uint64_t)kGroupWaves64 * kTile : (uint64_t)kTile; }

uint32_t passes_for(uint64_t n)
{
    uint32_t p = 0;
    const uint64_t run0 = run0_for(n);
    for (uint64_t runs = (n + run0 - 1) / run0; runs > 1; runs = (runs + 1) / 2)
        ++p;
    return p;
}

}  // namespace
}  // namespace bcf

using namespace bcf;

extern "C" bcf_status bcf_sort_u64(const uint64_t *keys_in, uint64_t *keys_out, uint64_t n, void *temp,
                                   uint64_t *temp_bytes, void *stream)
{
    if (!temp_bytes || n > kMaxN64)
        return BCF_ERR_INVALID;
    const uint32_t passes = passes_for(n);
    const uint64_t need = passes ? align256(n * sizeof(uint64_t)) : 0;  // the ping-pong buffer
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (n == 0)
        return BCF_OK;
    if (!keys_in || !keys_out)
        return BCF_ERR_INVALID;
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t *tb = static_cast<uint64_t *>(temp);
    // buffer after pass j: the output when passes - j is even, so the last pass writes it
    auto buf = [&](uint32_t j) { return ((passes - j) % 2 == 0) ? keys_out : tb; };
    const uint32_t tiles = (uint32_t)((n + kTile - 1) / kTile);
    // MI355X's last-level cache holds 256 MiB; a pass reads and writes 16 B per key
    const bool nt = 16.0 * n > 256.0 * 1024 * 1024;
    const uint64_t run0 = run0_for(n);
    void *scope = prof_begin("block_sort_u64", s, 16.0 * n);
    if (run0 > (uint64_t)kTile) {
        const uint32_t groups = (uint32_t)((n + run0 - 1) / run0);
        const dim3 block(kWave * kGroupWaves64);
        if (nt)
            hipLaunchKernelGGL(k_u64_block_sort_group<true>, dim3(groups), block, 0, s, keys_in, buf(0), n);
        else
            hipLaunchKernelGGL(k_u64_block_sort_group<false>, dim3(groups), block, 0, s, keys_in, buf(0), n);
    } else if (nt) {
        hipLaunchKernelGGL(k_u64_block_sort<true>, dim3(tiles), dim3(kWave), 0, s, keys_in, buf(0), n);
    } else {
        hipLaunchKernelGGL(k_u64_block_sort<false>, dim3(tiles), dim3(kWave), 0, s, keys_in, buf(0), n);
    }
    prof_end(scope);
    if (hipGetLastError() != hipSuccess)
        return BCF_ERR_DEVICE;
    uint64_t run = run0;
    for (uint32_t j = 1; j <= passes; ++j, run *= 2) {
        scope = prof_begin("merge_u64", s, 16.0 * n);
        if (nt)
            hipLaunchKernelGGL(k_u64_merge<true>, dim3(tiles), dim3(kWave), 0, s, buf(j - 1), buf(j), n, run);
        else
            hipLaunchKernelGGL(k_u64_merge<false>, dim3(tiles), dim3(kWave), 0, s, buf(j - 1), buf(j), n, run);
        prof_end(scope);
        if (hipGetLastError() != hipSuccess)
            return BCF_ERR_DEVICE;
    }
    return BCF_OK;
}
