// Device building blocks of the bank-conflict-free sort for gfx950 (CDNA4, wave64).
//
// The paper (Sitchinava & Weichert, Sec. 2.1) views a block of shared memory as
// a matrix whose rows are the memory banks, filled column-major, and processes
// it so that every thread of a warp owns one bank row; a conflict-free
// transposition turns columns into rows.  Its sort (Sec. 3.1) keeps one line of
// the w x w tile in registers per thread (Sec. 3.3, "use of registers") and
// sorts lines with Batcher's odd-even merge sort.
//
// Re-derived for gfx950 (measured: 32 banks x 4 bytes; a wave64 b32 LDS
// instruction is serviced as two independent 32-lane halves):
//   * a tile is a 64 x 64 matrix of keys, w = 64 = wave width, so one wave owns
//     w^2 = 4096 keys, 64 per lane, held in registers with compile-time indices;
//   * two register layouts of tile position p in [0, 4096):
//       STRIDED  lane = p mod 64, register = p / 64   (global loads/stores are
//                coalesced: register r of all lanes is 64 consecutive keys)
//       BLOCKED  lane = p / 64,   register = p mod 64 (lane owns a run of 64)
//   * switching layouts goes through LDS with four pad words per 64
//     (address = p + 4 (p/64)): STRIDED accesses are 4-byte reads and writes
//     of word 68r + lane, so every 32-lane half touches 32 distinct banks;
//     BLOCKED accesses move four consecutive registers at once, 16 bytes at
//     word 68 lane + r (r a multiple of 4): lane l's first bank is
//     4l + r mod 32, so any 8 consecutive lanes (one pass of 128 bytes) cover
//     the 32 banks once.  The lane-dependent part of an address is a base
//     register and the register-dependent part an immediate offset;
//   * compare-exchanges only ever happen between two registers of one lane, so
//     the sorting networks themselves issue no LDS traffic at all.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcf {

constexpr int kWave = 64;              // lanes per wavefront (w)
constexpr int kLine = 64;              // keys per lane (one line of the w x w tile)
constexpr int kTile = kWave * kLine;   // 4096 keys per wave tile (w^2)
constexpr int kLdsPad = 4;                   // pad words per 64-word LDS row
constexpr int kLdsStride = kLine + kLdsPad;  // 68 words per LDS row
constexpr int kLdsWords = kWave * kLdsStride;

constexpr uint32_t kMaxKey = 0xFFFFFFFFu;

// A wave's tile in registers.  Keys only: one 32-bit key per position.
//
// Key/value pairs: one 64-bit element per position that orders by (key,
// rank), where the rank is the element's position in the input order of the
// tile; comparing ranks on equal keys makes every network stable.  The
// element is a double in [1, 2) whose mantissa holds key * 2^15 + rank: such
// doubles are finite, normal and positive, so they order exactly as that
// 47-bit integer, and a compare-exchange is one v_min_f64 and one v_max_f64
// (full-rate on CDNA4), the same two instructions as for keys.  Values do not
// travel through the networks: after the last network the rank names the
// input position whose value goes with the key, the value is fetched by it
// (from LDS in the block sort, from global memory in a merge) and the element
// is repacked as key (high half) and value (low half) for the store.
template <bool PAIRS>
struct Lines {
    uint32_t k[kLine];
};
template <>
struct Lines<true> {
    double e[kLine];
};

// Unsigned 64-bit keys: one key per position in a register pair, compared as
// integers (no values, no ranks: equal keys are indistinguishable).
struct Lines64 {
    uint64_t e[kLine];
};
constexpr uint64_t kMaxKey64 = ~0ull;

constexpr uint32_t kRankBits = 15;                    // group tiles of up to 32768 positions
constexpr uint32_t kPadRank = (1u << kRankBits) - 1;  // rank of padding (never a real rank)
constexpr int kRankShift = 52 - 32 - (int)kRankBits;  // payload in mantissa bits 51 .. 5
constexpr uint64_t kElemOne = 0x3FF0000000000000ull;  // sign and exponent of 1.0
constexpr uint64_t kPayloadMask = ((1ull << (32 + kRankBits)) - 1) << kRankShift;

__device__ __forceinline__ uint64_t bits_of(double x) { return __builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ double elem_of(uint64_t b) { return __builtin_bit_cast(double, b); }

__device__ __forceinline__ double make_elem(uint32_t key, uint32_t rank)
{
    return elem_of(kElemOne | ((uint64_t)key << (kRankShift + kRankBits)) | ((uint64_t)rank << kRankShift));
}
__device__ __forceinline__ uint32_t elem_key(double e) { return (uint32_t)(bits_of(e) >> (kRankShift + kRankBits)); }
__device__ __forceinline__ uint32_t elem_rank(double e) { return (uint32_t)(bits_of(e) >> kRankShift) & kPadRank; }

// After the value step: key in the high half, value in the low half.
__device__ __forceinline__ double make_out(uint32_t key, uint32_t value)
{
    return elem_of(((uint64_t)key << 32) | value);
}
__device__ __forceinline__ uint32_t out_key(double e) { return (uint32_t)(bits_of(e) >> 32); }
__device__ __forceinline__ uint32_t out_value(double e) { return (uint32_t)bits_of(e); }

// Key of register r of a tile that is still in element form.
template <bool P>
__device__ __forceinline__ uint32_t key_of(const Lines<P> &t, int r)
{
    if constexpr (P)
        return elem_key(t.e[r]);
    else
        return t.k[r];
}

// ---------------------------------------------------------------- comparators

// Put the smaller element in register a, the larger in register b.
template <bool P>
__device__ __forceinline__ void cx(Lines<P> &t, int a, int b)
{
    if constexpr (!P) {
        const uint32_t x = t.k[a], y = t.k[b];
        t.k[a] = min(x, y);
        t.k[b] = max(x, y);
    } else {
        const double x = t.e[a], y = t.e[b];
        t.e[a] = __builtin_fmin(x, y);
        t.e[b] = __builtin_fmax(x, y);
    }
}

// 64-bit keys: one unsigned 64-bit compare and four 32-bit selects.
__device__ __forceinline__ void cx(Lines64 &t, int a, int b)
{
    const uint64_t x = t.e[a], y = t.e[b];
    const bool lt = x < y;
    t.e[a] = lt ? x : y;
    t.e[b] = lt ? y : x;
}

// Reverse the order of every element of a lane when `bit` is 1: the key (or
// the element's payload) is replaced by its bitwise complement, an
// order-reversing bijection, so an ascending network run on complemented data
// sorts descending.  Used where
// the direction of a merge depends on the lane (BLOCKED layout).
template <bool P>
__device__ __forceinline__ void flip(Lines<P> &t, uint32_t bit)
{
    const uint32_t m = 0u - (bit & 1u);
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        if constexpr (P)  // complement the payload only: the element stays in [1, 2)
            t.e[r] = elem_of(bits_of(t.e[r]) ^ (kPayloadMask & ((uint64_t)m << 32 | m)));
        else
            t.k[r] ^= m;
    }
}

__device__ __forceinline__ void flip(Lines64 &t, uint32_t bit)
{
    const uint64_t m = 0ull - (uint64_t)(bit & 1u);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        t.e[r] ^= m;
}

// ---------------------------------------------------- register-local networks
//
// Written once for any line type L (Lines<false>, Lines<true>, Lines64): the
// compare-exchange cx(t, a, b) is chosen by overload.

// One bitonic half-cleaner step at register distance D: registers r and r+D
// (r with bit D clear) are compare-exchanged, ascending, or descending where
// register bit DB of r is set (DB < 0: ascending everywhere).
template <int D, int DB, class L>
__device__ __forceinline__ void half_clean_step_lines(L &t)
{
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        if (r & D)
            continue;
        if (DB >= 0 && ((r >> (DB < 0 ? 0 : DB)) & 1))
            cx(t, r + D, r);
        else
            cx(t, r, r + D);
    }
}

// Half-cleaner cascade D, D/2, ..., 1: sorts every aligned group of 2D
// registers that holds a bitonic sequence.
template <int D, int DB, class L>
__device__ __forceinline__ void half_clean_lines(L &t)
{
    half_clean_step_lines<D, DB>(t);
    if constexpr (D > 1)
        half_clean_lines<D / 2, DB>(t);
}

// Batcher's odd-even merge of registers LO..HI (inclusive) whose two halves
// are sorted, considering every R-th register (Batcher 1968; the recursive
// formulation in Knuth, TAOCP vol. 3, Sec. 5.3.4).
template <int LO, int HI, int R, class L>
__device__ __forceinline__ void oe_merge_lines(L &t)
{
    constexpr int STEP = 2 * R;
    if constexpr (STEP < HI - LO) {
        oe_merge_lines<LO, HI, STEP>(t);
        oe_merge_lines<LO + R, HI, STEP>(t);
#pragma unroll
        for (int i = LO + R; i < HI - R; i += STEP)
            cx(t, i, i + R);
    } else {
        cx(t, LO, LO + R);
    }
}

// Batcher's odd-even merge sort of registers LO..HI (inclusive), ascending:
// the per-thread line sort of the paper (Sec. 3.1; 543 comparators for 64).
template <int LO, int HI, class L>
__device__ __forceinline__ void oe_sort_lines(L &t)
{
    if constexpr (HI - LO >= 1) {
        constexpr int MID = LO + (HI - LO) / 2;
        oe_sort_lines<LO, MID>(t);
        oe_sort_lines<MID + 1, HI>(t);
        oe_merge_lines<LO, HI, 1>(t);
    }
}

// The same networks for the 32-bit element kinds, named by the pairs flag.
template <int D, int DB, bool P>
__device__ __forceinline__ void half_clean_step(Lines<P> &t)
{
    half_clean_step_lines<D, DB>(t);
}
template <int D, int DB, bool P>
__device__ __forceinline__ void half_clean(Lines<P> &t)
{
    half_clean_lines<D, DB>(t);
}
template <int LO, int HI, int R, bool P>
__device__ __forceinline__ void oe_merge(Lines<P> &t)
{
    oe_merge_lines<LO, HI, R>(t);
}
template <int LO, int HI, bool P>
__device__ __forceinline__ void oe_sort(Lines<P> &t)
{
    oe_sort_lines<LO, HI>(t);
}

// ------------------------------------------------------------ LDS transposes

// Orders this wave's LDS accesses in the compiler: a wave's LDS instructions
// execute in issue order, so no hardware wait is needed between a lane's
// write and another lane's later read of the same word.
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x[r] -> w[S*r] for r = 0..63.  With S = 1 (the BLOCKED side: a lane's
// registers are consecutive words and the row starts 16-byte aligned) the
// compiler merges every four registers into one 16-byte store.
template <int S>
__device__ __forceinline__ void lds_put(uint32_t *w, const uint32_t (&x)[kLine])
{
    if constexpr (S == 1)
        w = static_cast<uint32_t *>(__builtin_assume_aligned(w, 16));
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        w[S * r] = x[r];
}

// x[r] <- rd[S*r] for r = 0..63 (S = 1: 16-byte loads).
template <int S>
__device__ __forceinline__ void lds_get(uint32_t (&x)[kLine], const uint32_t *rd)
{
    if constexpr (S == 1)
        rd = static_cast<const uint32_t *>(__builtin_assume_aligned(rd, 16));
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        x[r] = rd[S * r];
}

// x[r] -> lds[wbase + WS*r], then x[r] <- lds[rbase + RS*r].
template <int WS, int RS>
__device__ __forceinline__ void exchange(uint32_t (&x)[kLine], uint32_t *lds, uint32_t wbase,
                                         uint32_t rbase)
{
    lds_put<WS>(lds + wbase, x);
    wave_lds_fence();
    lds_get<RS>(x, lds + rbase);
    wave_lds_fence();
}

// The 32-bit halves of 64-bit elements.
__device__ __forceinline__ void split_halves(const double (&x)[kLine], uint32_t (&hi)[kLine], uint32_t (&lo)[kLine])
{
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        hi[r] = (uint32_t)(bits_of(x[r]) >> 32);
        lo[r] = (uint32_t)bits_of(x[r]);
    }
}

// The same for 64-bit elements, one 32-bit half at a time (each half keeps the
// conflict-free word pattern of the 32-bit exchange).
template <int WS, int RS>
__device__ __forceinline__ void exchange(double (&x)[kLine], uint32_t *lds, uint32_t wbase, uint32_t rbase)
{
    uint32_t hi[kLine], lo[kLine];
    split_halves(x, hi, lo);
    exchange<WS, RS>(hi, lds, wbase, rbase);
    exchange<WS, RS>(lo, lds, wbase, rbase);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        x[r] = elem_of(((uint64_t)hi[r] << 32) | lo[r]);
}

// The same for 64-bit keys.
template <int WS, int RS>
__device__ __forceinline__ void exchange(uint64_t (&x)[kLine], uint32_t *lds, uint32_t wbase, uint32_t rbase)
{
    uint32_t hi[kLine], lo[kLine];
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        hi[r] = (uint32_t)(x[r] >> 32);
        lo[r] = (uint32_t)x[r];
    }
    exchange<WS, RS>(hi, lds, wbase, rbase);
    exchange<WS, RS>(lo, lds, wbase, rbase);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        x[r] = ((uint64_t)hi[r] << 32) | lo[r];
}

__device__ __forceinline__ uint64_t (&elems(Lines64 &t))[kLine] { return t.e; }

template <bool P>
__device__ __forceinline__ auto &elems(Lines<P> &t)
{
    if constexpr (P)
        return t.e;
    else
        return t.k;
}

// STRIDED -> BLOCKED: write word 68r + lane, read word 68 lane + r.
template <class L>
__device__ __forceinline__ void to_blocked(L &t, uint32_t *lds, uint32_t lane)
{
    exchange<kLdsStride, 1>(elems(t), lds, lane, kLdsStride * lane);
}

// BLOCKED -> STRIDED: write word 68 lane + r, read word 68r + lane.  Afterwards
// LDS word 68q + r holds tile position 64q + r.
template <class L>
__device__ __forceinline__ void to_strided(L &t, uint32_t *lds, uint32_t lane)
{
    exchange<1, kLdsStride>(elems(t), lds, kLdsStride * lane, lane);
}

// BLOCKED -> STRIDED with the positions reversed (position p of the result
// holds position 4095 - p): write word 68 lane + r, read word
// 68(63 - r) + 63 - lane (consecutive lanes, consecutive words).
__device__ __forceinline__ void to_strided_reversed(Lines<false> &t, uint32_t *lds, uint32_t lane)
{
    exchange<1, -kLdsStride>(t.k, lds, kLdsStride * lane, kLdsStride * (kLine - 1) + (kWave - 1) - lane);
}

// ------------------------------------------ half-width transposes (9 KiB LDS)
//
// The same STRIDED <-> BLOCKED transposes with half the LDS: view the tile as
// the 64 x 64 matrix M[register][lane].  v_permlane32_swap on registers r and
// r + 32 (r < 32) exchanges the upper half-wave of register r with the lower
// half-wave of register r + 32, which swaps the off-diagonal 32 x 32 quadrants
// of M; afterwards each half-wave holds two 32 x 32 blocks (registers 0..31
// and 32..63) that only need transposing inside the half-wave.  Each block
// goes through a 32-row LDS matrix per half-wave (rows of 36 words), one
// block after the other, so a wave needs 2 x 32 x 36 words instead of
// 64 x 68.  Accesses stay conflict-free on the measured geometry: 4-byte
// writes / reads of word 36r + l' (32 consecutive words per half-wave), and
// 16-byte reads / writes of word 36l' + c, c a multiple of 4 (36 = 4 mod 32:
// any 8 consecutive lanes cover the 32 banks once).
constexpr int kHalfRows = 32;
constexpr int kHalfStride = 36;
constexpr int kHalfLdsWords = 2 * kHalfRows * kHalfStride;  // per wave: 9 KiB

// Exchange the upper half-wave of register r with the lower half-wave of
// register r + 32, for r = 0..31.
__device__ __forceinline__ void swap_quadrants(uint32_t (&x)[kLine])
{
#pragma unroll
    for (int r = 0; r < kLine / 2; ++r) {
        const auto p = __builtin_amdgcn_permlane32_swap(x[r], x[r + kLine / 2], false, false);
        x[r] = p[0];
        x[r + kLine / 2] = p[1];
    }
}

// This half-wave's 32 x 36-word LDS matrix.
__device__ __forceinline__ uint32_t *half_matrix(uint32_t *lds, uint32_t lane)
{
    return lds + (lane >> 5) * (kHalfRows * kHalfStride);
}

// Transpose the 32 x 32 block in registers R0..R0+31 inside each half-wave:
// the STRIDED side (register r, lane l') at word 36r + l', the BLOCKED side
// (lane l', register c) at word 36l' + c.  S2B: STRIDED side in, BLOCKED
// side out; else the reverse.
template <int R0, bool S2B>
__device__ __forceinline__ void half_block_transpose(uint32_t (&x)[kLine], uint32_t *lds, uint32_t lane)
{
    uint32_t *m = half_matrix(lds, lane);
    const uint32_t l = lane & 31;
    uint32_t *row = static_cast<uint32_t *>(__builtin_assume_aligned(m + kHalfStride * l, 16));
    if constexpr (S2B) {
#pragma unroll
        for (int r = 0; r < kHalfRows; ++r)
            m[kHalfStride * r + l] = x[R0 + r];
        wave_lds_fence();
#pragma unroll
        for (int c = 0; c < kHalfRows; ++c)
            x[R0 + c] = row[c];
    } else {
#pragma unroll
        for (int c = 0; c < kHalfRows; ++c)
            row[c] = x[R0 + c];
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < kHalfRows; ++r)
            x[R0 + r] = m[kHalfStride * r + l];
    }
    wave_lds_fence();
}

// STRIDED -> BLOCKED (keys) through the half-width matrices.
__device__ __forceinline__ void to_blocked_half(Lines<false> &t, uint32_t *lds, uint32_t lane)
{
    swap_quadrants(t.k);
    half_block_transpose<0, true>(t.k, lds, lane);
    half_block_transpose<kLine / 2, true>(t.k, lds, lane);
}

// BLOCKED -> STRIDED (keys) through the half-width matrices.
__device__ __forceinline__ void to_strided_half(Lines<false> &t, uint32_t *lds, uint32_t lane)
{
    half_block_transpose<0, false>(t.k, lds, lane);
    half_block_transpose<kLine / 2, false>(t.k, lds, lane);
    swap_quadrants(t.k);
}

// The same two transposes for 64-bit elements, one 32-bit half after the
// other through the same matrices.
__device__ __forceinline__ void to_blocked_half(Lines<true> &t, uint32_t *lds, uint32_t lane)
{
    uint32_t hi[kLine], lo[kLine];
    split_halves(t.e, hi, lo);
    swap_quadrants(hi);
    half_block_transpose<0, true>(hi, lds, lane);
    half_block_transpose<kLine / 2, true>(hi, lds, lane);
    swap_quadrants(lo);
    half_block_transpose<0, true>(lo, lds, lane);
    half_block_transpose<kLine / 2, true>(lo, lds, lane);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        t.e[r] = elem_of(((uint64_t)hi[r] << 32) | lo[r]);
}

__device__ __forceinline__ void to_strided_half(Lines<true> &t, uint32_t *lds, uint32_t lane)
{
    uint32_t hi[kLine], lo[kLine];
    split_halves(t.e, hi, lo);
    half_block_transpose<0, false>(hi, lds, lane);
    half_block_transpose<kLine / 2, false>(hi, lds, lane);
    swap_quadrants(hi);
    half_block_transpose<0, false>(lo, lds, lane);
    half_block_transpose<kLine / 2, false>(lo, lds, lane);
    swap_quadrants(lo);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        t.e[r] = elem_of(((uint64_t)hi[r] << 32) | lo[r]);
}

// ------------------------------------------------------ group (multi-wave) sort
//
// NW waves of a work-group (NW = 2^LW) sort a group tile of NW * 4096 keys:
// every wave sorts its 4096-key sub-tile (odd waves descending, by
// complementing around the wave sort), then LW more bitonic rounds
// (J = 7 .. 6+LW) merge across waves.  Wave w holds group positions with
// bits 12.. equal to w.  A third layout brings the wave bits into registers:
//   CROSS  lane = p bits 0..5, wave = p bits 6..5+LW, register = p bits 6+LW..11+LW
// Round J: BLOCKED -> CROSS (shared LDS, barriers), stages on bits 5+J..6+LW
// in registers, CROSS -> STRIDED, stages on bits 5+LW..6, STRIDED -> BLOCKED
// (the wave's own LDS slice), stages on bits 5..0.  The LDS word of position
// p is p + 4 (p/64) in all three layouts, so every access keeps the 68-word
// rows of the single-wave transposes: lane-consecutive 4-byte accesses (CROSS,
// STRIDED) touch 32 distinct banks per 32-lane half, and BLOCKED accesses are
// 16-byte, four registers at a time, 8 lanes covering the 32 banks.

// x[r] -> lds[wbase + WS*r]; barrier; x[r] <- lds[rbase + RS*r]; barrier.
template <int WS, int RS>
__device__ __forceinline__ void group_exchange(uint32_t (&x)[kLine], uint32_t *lds, uint32_t wbase,
                                               uint32_t rbase)
{
    lds_put<WS>(lds + wbase, x);
    __syncthreads();
    lds_get<RS>(x, lds + rbase);
    __syncthreads();
}

// The same for 64-bit elements, one 32-bit half at a time.
template <int WS, int RS>
__device__ __forceinline__ void group_exchange(double (&x)[kLine], uint32_t *lds, uint32_t wbase, uint32_t rbase)
{
    uint32_t hi[kLine], lo[kLine];
    split_halves(x, hi, lo);
    group_exchange<WS, RS>(hi, lds, wbase, rbase);
    group_exchange<WS, RS>(lo, lds, wbase, rbase);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        x[r] = elem_of(((uint64_t)hi[r] << 32) | lo[r]);
}

// The same for 64-bit keys.
template <int WS, int RS>
__device__ __forceinline__ void group_exchange(uint64_t (&x)[kLine], uint32_t *lds, uint32_t wbase, uint32_t rbase)
{
    uint32_t hi[kLine], lo[kLine];
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        hi[r] = (uint32_t)(x[r] >> 32);
        lo[r] = (uint32_t)x[r];
    }
    group_exchange<WS, RS>(hi, lds, wbase, rbase);
    group_exchange<WS, RS>(lo, lds, wbase, rbase);
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        x[r] = ((uint64_t)hi[r] << 32) | lo[r];
}

// BLOCKED p = 4096w + 64 lane + r  ->  CROSS p = lane + 64w + 64*NW*r
template <int NW, class L>
__device__ __forceinline__ void blocked_to_cross(L &t, uint32_t *lds, uint32_t lane, uint32_t wave)
{
    const uint32_t wb = kLdsStride * (kWave * wave + lane), rb = kLdsStride * wave + lane;
    group_exchange<1, kLdsStride * NW>(elems(t), lds, wb, rb);
}

// CROSS p = lane + 64w + 64*NW*r  ->  STRIDED p = 4096w + 64r + lane
template <int NW, class L>
__device__ __forceinline__ void cross_to_strided(L &t, uint32_t *lds, uint32_t lane, uint32_t wave)
{
    const uint32_t wb = kLdsStride * wave + lane, rb = kLdsStride * kWave * wave + lane;
    group_exchange<kLdsStride * NW, kLdsStride>(elems(t), lds, wb, rb);
}

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }

// Round J (7 .. 6+LW) of the group sort; on entry and exit the tile is
// BLOCKED and every run of 2^(6+J) positions is sorted, descending where bit
// 6+J is set (the last round sorts ascending).
template <int NW, int J, class L>
__device__ __forceinline__ void group_round(L &t, uint32_t *lds, uint32_t lane, uint32_t wave)
{
    constexpr int LW = log2i(NW);
    constexpr bool last = J == 6 + LW;
    blocked_to_cross<NW>(t, lds, lane, wave);
    // bits 5+J .. 6+LW = CROSS register bits J-1-LW .. 0; direction bit 6+J = register bit J-LW
    half_clean_lines<(1 << (J - 1 - LW)), (last ? -1 : J - LW)>(t);
    cross_to_strided<NW>(t, lds, lane, wave);
    // bits 5+LW .. 6 = STRIDED register bits LW-1 .. 0; direction bit 6+J = wave bit J-6
    if constexpr (!last)
        flip(t, wave >> (J - 6));
    half_clean_lines<(1 << (LW - 1)), -1>(t);
    to_blocked(t, lds + kLdsWords * wave, lane);
    half_clean_lines<kLine / 2, -1>(t);
    if constexpr (!last)
        flip(t, wave >> (J - 6));
}

// Rounds J .. 6 + log2(NW) of a group tile (any line type).
template <int NW, int J, class L>
__device__ __forceinline__ void group_rounds(L &t, uint32_t *lds, uint32_t lane, uint32_t wave)
{
    group_round<NW, J>(t, lds, lane, wave);
    if constexpr (J < 6 + log2i(NW))
        group_rounds<NW, J + 1>(t, lds, lane, wave);
}

// ---------------------------------------------------------------- wave utils

// The value of x, hidden from the optimiser.  Persistent kernels re-derive
// their lane index through this at the top of every tile so that the 64
// per-register address constants computed from it are not hoisted out of the
// tile loop (which would keep them all live in registers).
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Co-rank (merge-path split) of the stable merge of sorted A and B: the number
// of elements of A among the first d outputs when equal keys take A first.
// It is the smallest i in [max(0, d-nb), min(d, na)] with A[i] > B[d-1-i].
// Lanes 0..31 search for diagonal d of their half-wave, lanes 32..63 for
// theirs; each round probes 32 evenly spaced candidates per half and keeps
// the bracket between the last failing and the first passing probe, so a
// search over 2^25 candidates takes 5 rounds of loads.
template <class K>
__device__ __forceinline__ uint32_t corank_halfwave(const K *__restrict__ A, uint32_t na, const K *__restrict__ B,
                                                    uint32_t nb, uint32_t d, uint32_t lane)
{
    const uint32_t k = lane & 31;
    const uint32_t shift = lane & 32;  // 0 or 32: position of this half in the ballot
    uint32_t lo = d > nb ? d - nb : 0;
    uint32_t hi = d < na ? d : na;
    while (true) {
        const uint32_t span = hi - lo;
        if (ballot(span != 0) == 0)
            break;
        // probe k of this half: lo + floor(span * k / 32) < hi when span > 0
        const uint32_t i = lo + (uint32_t)(((uint64_t)span * k) >> 5);
        bool pass = true;
        if (span != 0)
            pass = A[i] > B[d - 1 - i];
        const uint32_t fails = (uint32_t)(ballot(!pass && span != 0) >> shift);
        const uint32_t c = __popc(fails);  // probes 0..c-1 fail (the predicate is monotone)
        if (span != 0) {
            if (c == 0) {
                hi = lo;
            } else {
                const uint32_t plast = lo + (uint32_t)(((uint64_t)span * (c - 1)) >> 5);
                const uint32_t pnext = c < 32 ? lo + (uint32_t)(((uint64_t)span * c) >> 5) : hi;
                lo = plast + 1;
                hi = pnext;
            }
        }
    }
    return lo;
}

}  // namespace bcf
