// HIP kernels of the bank-conflict-free sort for gfx950.
//
//  k_block_sort  -- base case (paper Sec. 3.1): one wave sorts a 64 x 64 tile
//                   of 4096 keys.  Lines of 64 keys are sorted in registers
//                   with Batcher's network; the 64 sorted lines are then merged
//                   in six rounds of bitonic merging whose compare-exchanges
//                   are all register-local, alternating between the STRIDED
//                   and BLOCKED layouts through conflict-free LDS transposes.
//  k_merge       -- one binary merge pass (paper Sec. 3.2): every wave produces
//                   4096 consecutive outputs of the merge of two sorted runs.
//                   The split of its output range between the runs is found by
//                   a co-rank search (the exact counterpart of the paper's
//                   splitter ranks), the two pieces are loaded coalesced as one
//                   bitonic sequence (A ascending, B reversed) and merged by a
//                   12-step half-cleaner network, again register-local between
//                   two conflict-free transposes; the tile is stored coalesced.
//
// Both kernels come in a keys-only and a stable key/value form, and in a
// "regular" form (all runs of one power-of-two length, positions computed
// arithmetically) and a "table" form (tiles and merge jobs read from
// descriptor arrays planned on the host, used for merging arbitrary runs and
// for segmented sorting).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bcf_device.hpp"
#include "bcf_internal.hpp"

namespace bcf {

// ------------------------------------------------------------------ tile I/O

// Load `count` elements starting at `src` into STRIDED layout (position
// p = 64r + lane); positions >= count become padding (max key, max rank).
// For pairs the tie-break rank is the position in the input order.
template <bool P>
__device__ __forceinline__ void load_tile(Lines<P> &t, const uint32_t *__restrict__ ksrc,
                                          const uint32_t *__restrict__ vsrc, uint32_t count,
                                          uint32_t lane)
{
    const uint32_t *kp = ksrc + lane;
    const uint32_t *vp = P ? vsrc + lane : nullptr;
    if (count >= (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            t.k[r] = kp[kWave * r];
            if constexpr (P) {
                t.i[r] = kWave * r + lane;
                t.v[r] = vp[kWave * r];
            }
        }
    } else {
        const uint32_t last = count ? count - 1 : 0;
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            const uint32_t q = p < count ? p : last;  // clamped: always a valid address
            const uint32_t key = count ? ksrc[q] : kMaxKey;
            t.k[r] = p < count ? key : kMaxKey;
            if constexpr (P) {
                t.i[r] = p < count ? p : kPadIdx;
                t.v[r] = count ? vsrc[q] : 0u;
            }
        }
    }
}

// Store the first `count` positions of a STRIDED tile.
template <bool P>
__device__ __forceinline__ void store_tile(const Lines<P> &t, uint32_t *__restrict__ kdst,
                                           uint32_t *__restrict__ vdst, uint32_t count, uint32_t lane)
{
    uint32_t *kp = kdst + lane;
    uint32_t *vp = P ? vdst + lane : nullptr;
    if (count >= (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            kp[kWave * r] = t.k[r];
            if constexpr (P)
                vp[kWave * r] = t.v[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            if (kWave * r + lane < count) {
                kp[kWave * r] = t.k[r];
                if constexpr (P)
                    vp[kWave * r] = t.v[r];
            }
        }
    }
}

// ----------------------------------------------------------- block sort body

// Round J (1..6) merges pairs of sorted runs of 2^(5+J) positions into runs of
// 2^(6+J).  Runs alternate direction (bit 6+J of the position set: the merged
// run is descending), so each pair is a bitonic sequence and a half-cleaner
// cascade over position bits 5+J .. 0 sorts it.  Bits 5+J .. 6 are register
// bits in STRIDED layout, where the direction bit is register bit J (a
// compile-time constant); bits 5 .. 0 are register bits in BLOCKED layout,
// where the direction bit is lane bit J and is applied by complementing.
template <int J, bool P>
__device__ __forceinline__ void merge_round(Lines<P> &t, uint32_t *lds, uint32_t lane)
{
    to_strided(t, lds, lane);
    half_clean<(1 << (J - 1)), (J < 6 ? J : -1), P>(t);
    to_blocked(t, lds, lane);
    if constexpr (J < 6)
        flip(t, lane >> J);
    half_clean<kLine / 2, -1, P>(t);
    if constexpr (J < 6)
        flip(t, lane >> J);
}

// Sort one wave tile.  On entry the tile is in STRIDED positions as loaded;
// it is re-read as BLOCKED (lane l owns the 64 keys it loaded), which is only
// a renaming of positions: the multiset of the tile, and for pairs the
// tie-break ranks, are what the sort is defined on.  On exit the tile is
// sorted in STRIDED layout.
template <bool P>
__device__ __forceinline__ void sort_tile(Lines<P> &t, uint32_t *lds, uint32_t lane)
{
    // lines: even lanes ascending, odd lanes descending (run direction = bit 6)
    flip(t, lane);
    oe_sort<0, kLine - 1, P>(t);
    flip(t, lane);
    merge_round<1, P>(t, lds, lane);
    merge_round<2, P>(t, lds, lane);
    merge_round<3, P>(t, lds, lane);
    merge_round<4, P>(t, lds, lane);
    merge_round<5, P>(t, lds, lane);
    merge_round<6, P>(t, lds, lane);
    to_strided(t, lds, lane);
}

// --------------------------------------------------------------- merge body

// Merge the A-piece [0, na) and B-piece [0, nb) (na + nb = count <= kTile) of
// a stable merge into one sorted STRIDED tile.  A goes to positions [0, na)
// ascending, B to positions [kTile - nb, kTile) reversed, padding in between,
// which makes the tile bitonic; ranks follow the order A then B so that equal
// keys leave A first.
template <bool P>
__device__ __forceinline__ void merge_tile(Lines<P> &t, const uint32_t *__restrict__ ka,
                                           const uint32_t *__restrict__ va, uint32_t na,
                                           const uint32_t *__restrict__ kb,
                                           const uint32_t *__restrict__ vb, uint32_t nb,
                                           uint32_t *lds, uint32_t lane)
{
    const uint32_t bstart = kTile - nb;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        const bool in_a = p < na;
        const bool in_b = p >= bstart;
        const uint32_t qb = kTile - 1 - p;  // index into B when in_b
        // every lane loads from a valid address; padding lanes re-read A[0] or B[0]
        const uint32_t *kp = in_a ? ka + p : (in_b ? kb + qb : (na ? ka : kb));
        const uint32_t key = (na | nb) ? *kp : kMaxKey;
        t.k[r] = (in_a || in_b) ? key : kMaxKey;
        if constexpr (P) {
            const uint32_t *vp = in_a ? va + p : (in_b ? vb + qb : (na ? va : vb));
            t.v[r] = (na | nb) ? *vp : 0u;
            t.i[r] = in_a ? p : (in_b ? na + qb : kPadIdx);
        }
    }
    half_clean<kLine / 2, -1, P>(t);  // position bits 11..6 (registers, STRIDED)
    to_blocked(t, lds, lane);
    half_clean<kLine / 2, -1, P>(t);  // position bits 5..0 (registers, BLOCKED)
    to_strided(t, lds, lane);
}

// ------------------------------------------------------------------- kernels

template <bool P>
__global__ __launch_bounds__(kWave *kWavesPerGroup) void k_block_sort(const uint32_t *__restrict__ kin,
                                                                      const uint32_t *__restrict__ vin,
                                                                      uint32_t *__restrict__ kout,
                                                                      uint32_t *__restrict__ vout,
                                                                      uint64_t n)
{
    __shared__ uint32_t lds_all[kWavesPerGroup][kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t tile = (uint64_t)blockIdx.x * kWavesPerGroup + wave;
    const uint64_t start = tile * kTile;
    if (start >= n)
        return;
    const uint64_t rem = n - start;
    const uint32_t count = rem < (uint64_t)kTile ? (uint32_t)rem : (uint32_t)kTile;
    Lines<P> t;
    load_tile<P>(t, kin + start, P ? vin + start : nullptr, count, lane);
    sort_tile<P>(t, lds_all[wave], lane);
    store_tile<P>(t, kout + start, P ? vout + start : nullptr, count, lane);
}

template <bool P>
__global__ __launch_bounds__(kWave *kWavesPerGroup) void k_block_sort_table(Bufs kb, Bufs vb,
                                                                            const BlockTile *__restrict__ tiles,
                                                                            uint32_t ntiles)
{
    __shared__ uint32_t lds_all[kWavesPerGroup][kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x * kWavesPerGroup + wave;
    if (tile >= ntiles)
        return;
    const BlockTile d = tiles[tile];
    uint32_t *kdst = d.dst == kBufOut ? kb.out : kb.temp;
    uint32_t *vdst = P ? (d.dst == kBufOut ? vb.out : vb.temp) : nullptr;
    Lines<P> t;
    load_tile<P>(t, kb.in + d.start, P ? vb.in + d.start : nullptr, d.count, lane);
    sort_tile<P>(t, lds_all[wave], lane);
    store_tile<P>(t, kdst + d.start, P ? vdst + d.start : nullptr, d.count, lane);
}

// Shared body of both merge kernels: the wave's output range is
// [d0, d0 + count) of the merge of A (na) and B (nb).
template <bool P>
__device__ __forceinline__ void merge_range(const uint32_t *__restrict__ ka, const uint32_t *__restrict__ va,
                                            uint32_t na, uint32_t nb, uint32_t d0, uint32_t count,
                                            uint32_t *__restrict__ kdst, uint32_t *__restrict__ vdst,
                                            uint32_t *lds, uint32_t lane)
{
    const uint32_t *kbp = ka + na;
    const uint32_t *vbp = P ? va + na : nullptr;
    // lanes 0..31: split at d0; lanes 32..63: split at d0 + count
    const uint32_t d = lane < 32 ? d0 : d0 + count;
    const uint32_t split = corank_halfwave(ka, na, kbp, nb, d, lane);
    const uint32_t a0 = __shfl(split, 0);
    const uint32_t a1 = __shfl(split, 32);
    const uint32_t b0 = d0 - a0;
    const uint32_t pa = a1 - a0;
    const uint32_t pb = count - pa;
    Lines<P> t;
    merge_tile<P>(t, ka + a0, P ? va + a0 : nullptr, pa, kbp + b0, P ? vbp + b0 : nullptr, pb, lds, lane);
    store_tile<P>(t, kdst + d0, P ? vdst + d0 : nullptr, count, lane);
}

// Regular pass: runs of length `run` (a multiple of kTile) cover [0, n);
// runs 2s and 2s+1 are merged into [2s*run, min(2(s+1)*run, n)).
template <bool P>
__global__ __launch_bounds__(kWave *kWavesPerGroup) void k_merge(const uint32_t *__restrict__ ksrc,
                                                                 const uint32_t *__restrict__ vsrc,
                                                                 uint32_t *__restrict__ kdst,
                                                                 uint32_t *__restrict__ vdst, uint64_t n,
                                                                 uint64_t run)
{
    __shared__ uint32_t lds_all[kWavesPerGroup][kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t gstart = ((uint64_t)blockIdx.x * kWavesPerGroup + wave) * kTile;
    if (gstart >= n)
        return;
    const uint64_t base = gstart / (2 * run) * (2 * run);
    const uint64_t rem = n - base;
    const uint32_t na = (uint32_t)(rem < run ? rem : run);
    const uint64_t remb = rem - na;
    const uint32_t nb = (uint32_t)(remb < run ? remb : run);
    const uint32_t d0 = (uint32_t)(gstart - base);
    const uint32_t left = na + nb - d0;
    const uint32_t count = left < (uint32_t)kTile ? left : (uint32_t)kTile;
    merge_range<P>(ksrc + base, P ? vsrc + base : nullptr, na, nb, d0, count, kdst + base,
                   P ? vdst + base : nullptr, lds_all[wave], lane);
}

template <bool P>
__global__ __launch_bounds__(kWave *kWavesPerGroup) void k_merge_table(Bufs kb, Bufs vb,
                                                                       const MergeJob *__restrict__ jobs,
                                                                       const uint32_t *__restrict__ tile_job,
                                                                       uint32_t ntiles)
{
    __shared__ uint32_t lds_all[kWavesPerGroup][kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x * kWavesPerGroup + wave;
    if (tile >= ntiles)
        return;
    const MergeJob j = jobs[tile_job[tile]];
    const uint32_t d0 = (tile - j.first_tile) * (uint32_t)kTile;
    const uint32_t left = j.na + j.nb - d0;
    const uint32_t count = left < (uint32_t)kTile ? left : (uint32_t)kTile;
    const uint32_t *ks = j.src == kBufIn ? kb.in : (j.src == kBufOut ? kb.out : kb.temp);
    uint32_t *kd = j.dst == kBufOut ? kb.out : kb.temp;
    const uint32_t *vs = nullptr;
    uint32_t *vd = nullptr;
    if constexpr (P) {
        vs = j.src == kBufIn ? vb.in : (j.src == kBufOut ? vb.out : vb.temp);
        vd = j.dst == kBufOut ? vb.out : vb.temp;
    }
    merge_range<P>(ks + j.a_start, P ? vs + j.a_start : nullptr, j.na, j.nb, d0, count, kd + j.a_start,
                   P ? vd + j.a_start : nullptr, lds_all[wave], lane);
}

// Sortedness check of the runs of a merge input: sets *flag when some
// keys[i] > keys[i+1] with i+1 not the start of a run.
__global__ void k_check_runs(const uint32_t *__restrict__ keys, const uint64_t *__restrict__ offs, uint32_t k,
                             uint64_t n, uint32_t *flag)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < n; i += stride) {
        if (keys[i] > keys[i + 1]) {
            // is i+1 a run start?  binary search in offs[0..k]
            uint32_t lo = 0, hi = k;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2;
                if (offs[mid] < i + 1)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (offs[lo] != i + 1)
                *flag = 1u;
        }
    }
}

// ------------------------------------------------------------------ launchers

static inline uint32_t groups_for(uint64_t tiles)
{
    return (uint32_t)((tiles + kWavesPerGroup - 1) / kWavesPerGroup);
}

hipError_t launch_block_sort_regular(bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                     uint32_t *vout, uint64_t n, hipStream_t s)
{
    const uint64_t tiles = (n + kTile - 1) / kTile;
    const dim3 grid(groups_for(tiles)), block(kWave * kWavesPerGroup);
    if (pairs)
        hipLaunchKernelGGL(k_block_sort<true>, grid, block, 0, s, kin, vin, kout, vout, n);
    else
        hipLaunchKernelGGL(k_block_sort<false>, grid, block, 0, s, kin, vin, kout, vout, n);
    return hipGetLastError();
}

hipError_t launch_merge_regular(bool pairs, const uint32_t *ksrc, const uint32_t *vsrc, uint32_t *kdst,
                                uint32_t *vdst, uint64_t n, uint64_t run, hipStream_t s)
{
    const uint64_t tiles = (n + kTile - 1) / kTile;
    const dim3 grid(groups_for(tiles)), block(kWave * kWavesPerGroup);
    if (pairs)
        hipLaunchKernelGGL(k_merge<true>, grid, block, 0, s, ksrc, vsrc, kdst, vdst, n, run);
    else
        hipLaunchKernelGGL(k_merge<false>, grid, block, 0, s, ksrc, vsrc, kdst, vdst, n, run);
    return hipGetLastError();
}

hipError_t launch_block_sort_table(bool pairs, Bufs kb, Bufs vb, const BlockTile *tiles, uint32_t ntiles,
                                   hipStream_t s)
{
    const dim3 grid(groups_for(ntiles)), block(kWave * kWavesPerGroup);
    if (pairs)
        hipLaunchKernelGGL(k_block_sort_table<true>, grid, block, 0, s, kb, vb, tiles, ntiles);
    else
        hipLaunchKernelGGL(k_block_sort_table<false>, grid, block, 0, s, kb, vb, tiles, ntiles);
    return hipGetLastError();
}

hipError_t launch_merge_table(bool pairs, Bufs kb, Bufs vb, const MergeJob *jobs, const uint32_t *tile_job,
                              uint32_t ntiles, hipStream_t s)
{
    const dim3 grid(groups_for(ntiles)), block(kWave * kWavesPerGroup);
    if (pairs)
        hipLaunchKernelGGL(k_merge_table<true>, grid, block, 0, s, kb, vb, jobs, tile_job, ntiles);
    else
        hipLaunchKernelGGL(k_merge_table<false>, grid, block, 0, s, kb, vb, jobs, tile_job, ntiles);
    return hipGetLastError();
}

hipError_t launch_check_runs(const uint32_t *keys, const uint64_t *offs_dev, uint32_t k, uint64_t n,
                             uint32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_runs, dim3(1024), dim3(256), 0, s, keys, offs_dev, k, n, flag);
    return hipGetLastError();
}

const char *kname_block_sort(bool pairs, bool table)
{
    return pairs ? (table ? "block_sort_pairs_table" : "block_sort_pairs")
                 : (table ? "block_sort_keys_table" : "block_sort_keys");
}

const char *kname_merge(bool pairs, bool table)
{
    return pairs ? (table ? "merge_pairs_table" : "merge_pairs") : (table ? "merge_keys_table" : "merge_keys");
}

}  // namespace bcf
