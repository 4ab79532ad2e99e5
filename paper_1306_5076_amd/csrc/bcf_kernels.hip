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

#include <algorithm>
#include <type_traits>

#include "bcf_device.hpp"
#include "bcf_internal.hpp"

namespace bcf {

// ------------------------------------------------------------------ tile I/O

// Global load / store, optionally with the nontemporal hint (streamed data
// that is not re-read by this launch).
template <bool NT>
__device__ __forceinline__ uint32_t ld(const uint32_t *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT>
__device__ __forceinline__ void st(uint32_t *p, uint32_t v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Order-preserving maps between other 32-bit key types and u32: signed
// integers flip the sign bit; IEEE binary32 floats flip the sign bit of a
// non-negative value and every bit of a negative one, which orders the bit
// patterns by IEEE 754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf
// < +NaN).  With (sign, rest) = (0x80000000, 0) for i32 and (0x80000000,
// 0x7fffffff) for f32 the map is x ^ (sign | (x >> 31 arithmetic) & rest) and
// its inverse t ^ (sign | (~t >> 31 arithmetic) & rest).
__device__ __forceinline__ uint32_t map_key(uint32_t x, uint32_t sign, uint32_t rest, uint32_t inverse)
{
    const uint32_t s = (uint32_t)((int32_t)(inverse ? ~x : x) >> 31);
    return x ^ (sign | (s & rest));
}

KeyMap key_map(int kind, bool inverse)
{
    KeyMap m;
    if (kind == 1 || kind == 2) {
        m.sign = 0x80000000u;
        m.rest = kind == 2 ? 0x7fffffffu : 0u;
        m.inverse = inverse ? 1u : 0u;
    }
    return m;
}

// Load `count` keys starting at `ksrc` into STRIDED layout (position
// p = 64r + lane); positions >= count become padding (key `pad`, max rank).
// For pairs the element's rank is rank0 + p, its position in the input order;
// values are not loaded here (see permute_values_lds / gather_values).  The
// pad is the maximum key, or for keys that go through a key map the key that
// the map sends to the maximum, so that the map applies to every position.
template <bool P>
__device__ __forceinline__ void load_tile(Lines<P> &t, const uint32_t *__restrict__ ksrc, uint32_t count,
                                          uint32_t lane, uint32_t rank0 = 0, uint32_t pad = kMaxKey)
{
    const uint32_t *kp = ksrc + lane;
    if constexpr (P) {
        // all 64 loads first, then the conversions: left to itself the
        // scheduler converts each key right after its load and so waits for
        // the loads one at a time.  With count == 0 (a group tile's sub-tile
        // past the end of its input; ksrc may point past the end of the
        // array) nothing is loaded and every position is padding.
        uint32_t key[kLine] = {};
        if (count != 0) {
            const uint32_t last = count - 1;
#pragma unroll
            for (int r = 0; r < kLine; ++r) {
                const uint32_t p = kWave * r + lane;
                key[r] = ksrc[p < count ? p : last];  // clamped: always a valid address
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            t.e[r] = p < count ? make_elem(key[r], rank0 + p) : make_elem(pad, kPadRank);
        }
    } else if (count >= (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kLine; ++r)
            t.k[r] = kp[kWave * r];
    } else {
        const uint32_t last = count ? count - 1 : 0;
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            const uint32_t q = p < count ? p : last;  // clamped: always a valid address
            const uint32_t key = count ? ksrc[q] : pad;
            t.k[r] = p < count ? key : pad;
        }
    }
}

// Store the first `count` positions of a STRIDED tile.  A pairs tile is in
// output form (key and value halves) by now, after its value step.
template <bool P, bool NT = false>
__device__ __forceinline__ void store_tile(const Lines<P> &t, uint32_t *__restrict__ kdst,
                                           uint32_t *__restrict__ vdst, uint32_t count, uint32_t lane)
{
    uint32_t *kp = kdst + lane;
    uint32_t *vp = P ? vdst + lane : nullptr;
    if (count >= (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            if constexpr (P) {
                st<NT>(kp + kWave * r, out_key(t.e[r]));
                st<NT>(vp + kWave * r, out_value(t.e[r]));
            } else {
                st<NT>(kp + kWave * r, t.k[r]);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            if (kWave * r + lane < count) {
                if constexpr (P) {
                    st<NT>(kp + kWave * r, out_key(t.e[r]));
                    st<NT>(vp + kWave * r, out_value(t.e[r]));
                } else {
                    st<NT>(kp + kWave * r, t.k[r]);
                }
            }
        }
    }
}

// A work source whose keys go through a key map: the forward map as the block
// sort loads them, the inverse as the pass that writes the output stores
// them.  A separate type so that sources of u32 sorts compile without the
// map (kMapped = false): a run-time test alone costs the kernels registers.
template <class Base>
struct Mapped : Base {
    static constexpr bool kMapped = true;
    KeyMap in_map, out_map;
};

// The forward key map on a freshly loaded STRIDED tile, every position: the
// tile was padded with pad_key(src), which the map sends to the maximum key.
template <bool P>
__device__ __forceinline__ void map_tile_in(Lines<P> &t, const KeyMap &m);

template <bool P, class Src>
__device__ __forceinline__ void map_tile_in(Lines<P> &t, const Src &src)
{
    if constexpr (Src::kMapped)
        map_tile_in<P>(t, src.in_map);
}

// The padding key of a block-sort tile: the maximum, or its preimage under
// the source's forward key map.
template <class Src>
__device__ __forceinline__ uint32_t pad_key(const Src &src)
{
    if constexpr (Src::kMapped)
        return map_key(kMaxKey, src.in_map.sign, src.in_map.rest, 1u - src.in_map.inverse);
    else
        return kMaxKey;
}

template <bool P>
__device__ __forceinline__ void map_tile_in(Lines<P> &t, const KeyMap &m)
{
    if (m.sign == 0)
        return;
    // one register at a time (the scheduling barrier keeps the compiler from
    // computing every register's map before storing any: 64 temporaries)
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        if constexpr (P)
            t.e[r] = make_elem(map_key(elem_key(t.e[r]), m.sign, m.rest, m.inverse), elem_rank(t.e[r]));
        else
            t.k[r] = map_key(t.k[r], m.sign, m.rest, m.inverse);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The inverse key map on a tile about to be stored (pairs: in output form,
// key in the high half).  Padding positions are never stored.
template <bool P>
__device__ __forceinline__ void map_tile_out(Lines<P> &t, const KeyMap &m);

template <bool P, class Src>
__device__ __forceinline__ void map_tile_out(Lines<P> &t, const Src &src)
{
    if constexpr (Src::kMapped)
        map_tile_out<P>(t, src.out_map);
}

template <bool P>
__device__ __forceinline__ void map_tile_out(Lines<P> &t, const KeyMap &m)
{
    if (m.sign == 0)
        return;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        if constexpr (P)
            t.e[r] = make_out(map_key(out_key(t.e[r]), m.sign, m.rest, m.inverse), out_value(t.e[r]));
        else
            t.k[r] = map_key(t.k[r], m.sign, m.rest, m.inverse);
        __builtin_amdgcn_sched_barrier(0);
    }
}

typedef __attribute__((address_space(1))) const void global_cvoid;
typedef __attribute__((address_space(3))) void lds_void;

// Value step of a block sort (pairs): the tile is sorted, in STRIDED layout,
// and every element's rank is its input position in [0, count) (padding
// ranks are larger).  The values of those `count` input positions are staged
// in LDS (`vals`, coalesced global reads, conflict-free consecutive LDS
// words) and each element is repacked as its key and the value read from LDS
// at its rank.  Callers separate this from other LDS use by the fence or
// barrier `sync`.
template <class Sync>
__device__ __forceinline__ void permute_values_lds(Lines<true> &t, const uint32_t *__restrict__ vsrc,
                                                   uint32_t count, uint32_t *vals, uint32_t stage_off,
                                                   uint32_t stage_count, uint32_t lane, const Sync &sync)
{
    // stage input positions [stage_off, stage_off + stage_count) of this wave
    // with direct global-to-LDS loads (lanes past the end re-read the first
    // position; their LDS words are never read).  A wave with nothing to
    // stage (a group tile's sub-tile past the end of the input, where src
    // points past the end of the array) issues no load.
    const uint32_t *src = vsrc + stage_off;
    if (stage_count != 0) {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            __builtin_amdgcn_global_load_lds((global_cvoid *)(src + (p < stage_count ? p : 0u)),
                                             (lds_void *)(vals + stage_off + kWave * r), 4, 0, 0);
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    sync();
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t rank = elem_rank(t.e[r]);
        const uint32_t v = rank < count ? vals[rank] : 0u;
        t.e[r] = make_out(elem_key(t.e[r]), v);
    }
    sync();
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
__device__ __forceinline__ void sort_tile_blocked(Lines<P> &t, uint32_t *lds, uint32_t lane)
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
}

template <bool P>
__device__ __forceinline__ void sort_tile(Lines<P> &t, uint32_t *lds, uint32_t lane)
{
    sort_tile_blocked<P>(t, lds, lane);
    to_strided(t, lds, lane);
}

// The paper's base case (Sec. 3.1, Algorithm 1): ShearSort of the 64 x 64
// tile, kept as an alternative to the merge rounds.  The grid's rows are the
// lines lanes hold in BLOCKED layout, its columns the lines they hold in
// STRIDED layout, so every line sort is Batcher's network on one lane's
// registers and every switch between rows and columns is one conflict-free
// transpose.  log2(64) = 6 iterations of (rows in snake order: odd rows
// descending, by complementing; columns ascending) leave the grid sorted in
// snake order except inside rows; a last ascending row sort then orders it
// row-major.  13 line sorts of 543 comparators and 12 transposes, against
// 8.5 line sorts' worth of comparators and 12 transposes for the merge rounds.
// Entry: the loaded STRIDED registers re-read as BLOCKED; exit: BLOCKED.
template <bool P>
__device__ __forceinline__ void shear_sort_blocked(Lines<P> &t, uint32_t *lds, uint32_t lane)
{
#pragma unroll 1
    for (int it = 0; it < 6; ++it) {
        flip(t, lane);
        oe_sort<0, kLine - 1, P>(t);
        flip(t, lane);
        to_strided(t, lds, lane);
        oe_sort<0, kLine - 1, P>(t);
        to_blocked(t, lds, lane);
    }
    oe_sort<0, kLine - 1, P>(t);
}

// --------------------------------------------------------------- merge body

// The inputs of one merge work item: the A-piece [0, pa) and B-piece [0, pb)
// (pa + pb = count <= kTile) that produce `count` consecutive outputs.
template <bool P>
struct MergeTask {
    const uint32_t *ka, *va, *kb, *vb;
    uint32_t *kd, *vd;
    uint64_t gpos;  // array position of the first output
    uint32_t pa, pb, count;
};

// Load a merge work item as one bitonic STRIDED tile: A goes to positions
// [0, pa) ascending, B to positions [kTile - pb, kTile) reversed, padding in
// between.  For pairs the rank of A[j] is j and that of B[j] is pa + j, so
// equal keys leave A first and the rank also names the element's source.
// Every lane computes a 32-bit element offset from the A-piece (the B-piece
// lies dB elements after it in the same array) and issues one unconditional
// load per register row, so all 64 loads of a tile are in flight together;
// padding lanes re-read element 0, which is always valid.
template <bool P, bool NT = false>
__device__ __forceinline__ void merge_load(Lines<P> &t, const MergeTask<P> &m, uint32_t lane)
{
    const uint32_t na = m.pa, nb = m.pb;
    const uint32_t bstart = kTile - nb;
    const uint32_t dB = (uint32_t)(m.kb - m.ka);   // B-piece start relative to the A-piece
    const uint32_t bend = dB + (kTile - 1);        // offset of position p in B is bend - p
    if constexpr (P) {
        // all 64 loads first, then the conversions to (key, rank) elements
        uint32_t key[kLine];
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            key[r] = ld<NT>(m.ka + (p < na ? p : (p >= bstart ? bend - p : 0u)));
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            const bool in_a = p < na, in_b = p >= bstart;
            t.e[r] = (in_a || in_b) ? make_elem(key[r], in_a ? p : na + (kTile - 1 - p)) : make_elem(kMaxKey, kPadRank);
        }
    } else if (m.count == (uint32_t)kTile) {
        // full tile: every position is in A or in B and no register needs a
        // select after its load (such selects make the compiler wait for the
        // loads one by one)
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            t.k[r] = ld<NT>(m.ka + (p < na ? p : bend - p));
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLine; ++r) {
            const uint32_t p = kWave * r + lane;
            const bool in_a = p < na;
            const bool in_b = p >= bstart;
            const uint32_t off = in_a ? p : (in_b ? bend - p : 0u);
            const uint32_t key = ld<NT>(m.ka + off);
            t.k[r] = (in_a || in_b) ? key : kMaxKey;
        }
    }
}

// Values of a merge work item (pairs), staged in LDS in the tile's position
// order (word p holds the value of the element merge_load put at position p)
// by direct global-to-LDS loads: they take no registers and are in flight
// together with the key loads, while the keys go through the network.
__device__ __forceinline__ void stage_merge_values(const MergeTask<true> &m, uint32_t *vals, uint32_t lane)
{
    const uint32_t na = m.pa, nb = m.pb;
    const uint32_t bstart = kTile - nb;
    const uint32_t bend = (uint32_t)(m.vb - m.va) + (kTile - 1);
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        const uint32_t off = p < na ? p : (p >= bstart ? bend - p : 0u);
        __builtin_amdgcn_global_load_lds((global_cvoid *)(m.va + off), (lds_void *)(vals + kWave * r), 4, 0, 0);
    }
}

// Value step of a merge (pairs): the merged tile is in STRIDED layout and each
// of its first `count` elements has a rank r (r < pa: A[r], loaded at
// position r; else B[r - pa], loaded at position 4095 - (r - pa)).  Repack it
// as its key and the value staged in LDS at that position.
__device__ __forceinline__ void gather_values(Lines<true> &t, const MergeTask<true> &m, const uint32_t *vals,
                                              uint32_t lane)
{
    // the staged values have landed in LDS once this wave's loads are done
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const uint32_t na = m.pa;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        const uint32_t rank = elem_rank(t.e[r]);
        const uint32_t pos = rank < na ? rank : (kTile - 1) - (rank - na);
        const uint32_t v = p < m.count ? vals[pos] : 0u;
        t.e[r] = make_out(elem_key(t.e[r]), v);
    }
}

template <bool P>
__device__ __forceinline__ void write_samples(const Lines<P> &t, const SampleSet &s, uint64_t gpos, uint32_t count,
                                              uint32_t lane);

// Sort a bitonic STRIDED tile: half-cleaners on position bits 11..6 (register
// bits in STRIDED layout), transpose, bits 5..0 (register bits in BLOCKED
// layout), transpose back.  In BLOCKED layout the sorted tile's samples are
// written (when `smp` has any).
template <bool P>
__device__ __forceinline__ void merge_network(Lines<P> &t, uint32_t *lds, uint32_t lane, const SampleSet &smp,
                                              uint64_t gpos, uint32_t count)
{
    half_clean<kLine / 2, -1, P>(t);
    to_blocked(t, lds, lane);
    half_clean<kLine / 2, -1, P>(t);
    write_samples<P>(t, smp, gpos, count, lane);
    to_strided(t, lds, lane);
}

// Samples of a sorted tile in BLOCKED layout starting at global position gpos
// (a multiple of 4096): lane l holds positions 64l .. 64l + 63, so register 0
// and register 63 of all lanes are the tile's 64-block samples (one coalesced
// store each); lane 0 / lane 63 hold the tile's first / last key.
template <bool P>
__device__ __forceinline__ void write_samples(const Lines<P> &t, const SampleSet &s, uint64_t gpos, uint32_t count,
                                              uint32_t lane)
{
    if (s.f == nullptr || count == 0)
        return;
    const uint64_t b = gpos / kLine + lane;
    if (lane * kLine < count) {
        s.f[b] = key_of(t, 0);
        s.l[b] = key_of(t, kLine - 1);
    }
    if (s.cf == nullptr)
        return;
    const uint64_t c = gpos / kTile;
    if (lane == 0)
        s.cf[c] = key_of(t, 0);
    if (lane == kWave - 1)
        s.cl[c] = key_of(t, kLine - 1);
}

// ----------------------------------------------------------- work sources
//
// A work source maps a tile number of a launch to the data it covers.
// "Regular" sources compute it arithmetically for a sort of n keys; "table"
// sources read host-planned descriptors.

struct SortItem {
    const uint32_t *ks, *vs;
    uint32_t *kd, *vd;
    uint32_t count;
};

struct RegularSortSrc {
    __device__ void resolve() {}
    const uint32_t *kin, *vin;
    uint32_t *kout, *vout;
    uint64_t n;
    uint32_t ntiles;
    SampleSet out_smp;
    static constexpr bool kMapped = false;
    __device__ uint64_t pos(uint32_t t) const { return (uint64_t)t * kTile; }
    __device__ SortItem get(uint32_t t) const
    {
        const uint64_t start = (uint64_t)t * kTile;
        const uint64_t rem = n - start;
        SortItem it;
        it.ks = kin + start;
        it.vs = vin ? vin + start : nullptr;
        it.kd = kout + start;
        it.vd = vout ? vout + start : nullptr;
        it.count = rem < (uint64_t)kTile ? (uint32_t)rem : (uint32_t)kTile;
        return it;
    }
};

// Table sources take their tile count from the launch (ntiles, the most the
// grid covers) and, when count_dev is set, from device memory (the count a
// device planner wrote; at most ntiles).
__device__ __forceinline__ uint32_t resolved_count(uint32_t bound, const uint32_t *count_dev)
{
    if (count_dev == nullptr)
        return bound;
    const uint32_t c = __builtin_amdgcn_readfirstlane(*count_dev);
    return c < bound ? c : bound;
}

struct TableSortSrc {
    Bufs kb, vb;
    const BlockTile *tiles;
    uint32_t ntiles;
    SampleSet out_smp;  // always empty: table tiles start anywhere
    const uint32_t *count_dev;
    static constexpr bool kMapped = false;
    __device__ void resolve() { ntiles = resolved_count(ntiles, count_dev); }
    __device__ uint64_t pos(uint32_t) const { return 0; }
    __device__ SortItem get(uint32_t t) const
    {
        const BlockTile d = tiles[t];
        SortItem it;
        it.ks = kb.in + d.start;
        it.vs = vb.in ? vb.in + d.start : nullptr;
        it.kd = (d.dst == kBufOut ? kb.out : kb.temp) + d.start;
        it.vd = vb.out ? (d.dst == kBufOut ? vb.out : vb.temp) + d.start : nullptr;
        it.count = d.count;
        return it;
    }
};

// One merge work item before splitting: runs A = ka[0, na) and
// B = ka[na, na + nb); outputs [d0, d0 + count) of their merge go to kd + d0.
struct MergeItem {
    const uint32_t *ka, *va;
    uint32_t *kd, *vd;
    uint64_t base;  // array position of A[0]
    uint32_t na, nb, d0, count;
};

// Runs of length `run` (a multiple of kTile) cover [0, n); runs 2s and 2s+1
// are merged into [2s*run, min(2(s+1)*run, n)).
struct RegularMergeSrc {
    __device__ void resolve() {}
    const uint32_t *ksrc, *vsrc;
    uint32_t *kdst, *vdst;
    uint64_t n, run;
    uint32_t ntiles;
    SampleSet in_smp, out_smp;
    static constexpr bool kMapped = false;
    __device__ MergeItem get(uint32_t t) const
    {
        const uint64_t gstart = (uint64_t)t * kTile;
        const uint64_t base = gstart / (2 * run) * (2 * run);
        const uint64_t rem = n - base;
        MergeItem m;
        m.na = (uint32_t)(rem < run ? rem : run);
        const uint64_t remb = rem - m.na;
        m.nb = (uint32_t)(remb < run ? remb : run);
        m.d0 = (uint32_t)(gstart - base);
        const uint32_t left = m.na + m.nb - m.d0;
        m.count = left < (uint32_t)kTile ? left : (uint32_t)kTile;
        m.base = base;
        m.ka = ksrc + base;
        m.va = vsrc ? vsrc + base : nullptr;
        m.kd = kdst + base;
        m.vd = vdst ? vdst + base : nullptr;
        return m;
    }
};

struct TableMergeSrc {
    Bufs kb, vb;
    const MergeJob *jobs;
    const uint32_t *tile_job;
    uint32_t ntiles;
    SampleSet out_smp;  // always empty: table runs start anywhere
    const uint32_t *count_dev;
    static constexpr bool kMapped = false;
    __device__ void resolve() { ntiles = resolved_count(ntiles, count_dev); }

    __device__ MergeItem get(uint32_t t) const
    {
        const MergeJob j = jobs[tile_job[t]];
        MergeItem m;
        m.na = j.na;
        m.nb = j.nb;
        m.d0 = (t - j.first_tile) * (uint32_t)kTile;
        const uint32_t left = j.na + j.nb - m.d0;
        m.count = left < (uint32_t)kTile ? left : (uint32_t)kTile;
        m.base = j.a_start;
        m.ka = (j.src == kBufIn ? kb.in : (j.src == kBufOut ? kb.out : kb.temp)) + j.a_start;
        m.kd = (j.dst == kBufOut ? kb.out : kb.temp) + j.a_start;
        m.va = nullptr;
        m.vd = nullptr;
        if (vb.out) {
            m.va = (j.src == kBufIn ? vb.in : (j.src == kBufOut ? vb.out : vb.temp)) + j.a_start;
            m.vd = (j.dst == kBufOut ? vb.out : vb.temp) + j.a_start;
        }
        return m;
    }
};

// The A/B pieces of tile t from its split (co-rank at d0, computed by
// k_partition) and the next tile's split, or the end of A when the tile ends
// its merge.
template <bool P>
__device__ __forceinline__ MergeTask<P> merge_task_at(const MergeItem &m, uint32_t a0, uint32_t a1)
{
    const uint32_t b0 = m.d0 - a0;
    MergeTask<P> k;
    k.pa = a1 - a0;
    k.pb = m.count - k.pa;
    k.count = m.count;
    k.ka = m.ka + a0;
    k.kb = m.ka + m.na + b0;
    k.kd = m.kd + m.d0;
    k.gpos = m.base + m.d0;
    k.va = P ? m.va + a0 : nullptr;
    k.vb = P ? m.va + m.na + b0 : nullptr;
    k.vd = P ? m.vd + m.d0 : nullptr;
    return k;
}

template <bool P, class Src>
__device__ __forceinline__ MergeTask<P> merge_task(const Src &src, const uint32_t *__restrict__ splits, uint32_t t)
{
    const MergeItem m = src.get(t);
    const uint32_t a0 = splits[t];
    const uint32_t a1 = (m.d0 + m.count == m.na + m.nb) ? m.na : splits[t + 1];
    return merge_task_at<P>(m, a0, a1);
}

// ------------------------------------------------------------------- kernels
//
// The sort and merge kernels are persistent: wave g of G handles tiles
// g, g + G, g + 2G, ...  For keys, the loads of the next tile are issued
// before the current tile is sorted/merged, so a wave's memory traffic
// overlaps its own arithmetic (two tiles of registers are live; a pairs tile
// holds 64-bit elements, twice the registers, so pairs process one tile at a
// time).

// Everything of a wave tile after it is in registers: sort (merge rounds, or
// the paper's ShearSort when SHEAR), samples, values, store.
template <bool P, bool SHEAR, class Src>
__device__ __forceinline__ void wave_tile(Lines<P> &a, const SortItem &it, const Src &src, uint32_t t, uint32_t *lds,
                                          uint32_t lane)
{
    map_tile_in<P>(a, src);
    if constexpr (SHEAR)
        shear_sort_blocked<P>(a, lds, lane);
    else
        sort_tile_blocked<P>(a, lds, lane);
    write_samples<P>(a, src.out_smp, src.pos(t), it.count, lane);
    to_strided(a, lds, lane);
    if constexpr (P)
        permute_values_lds(a, it.vs, it.count, lds, 0, it.count, lane, wave_lds_fence);
    map_tile_out<P>(a, src);
    store_tile<P>(a, it.kd, it.vd, it.count, lane);
}

template <bool P, class Src, bool SHEAR = false>
__global__ __launch_bounds__(kWave *kWavesPerGroup) void k_block_sort(Src src)
{
    src.resolve();
    __shared__ __align__(16) uint32_t lds_all[kWavesPerGroup][kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t *lds = lds_all[wave];
    const uint32_t G = gridDim.x * kWavesPerGroup;
    uint32_t t = blockIdx.x * kWavesPerGroup + wave;
    if (t >= src.ntiles)
        return;
    if constexpr (P) {
        for (; t < src.ntiles; t += G) {
            const uint32_t ln = opaque(lane);
            const SortItem it = src.get(t);
            Lines<P> a;
            load_tile<P>(a, it.ks, it.count, ln, 0, pad_key(src));
            wave_tile<P, SHEAR>(a, it, src, t, lds, ln);
        }
    } else {
        Lines<P> a, b;
        SortItem ia = src.get(t), ib;
        load_tile<P>(a, ia.ks, ia.count, lane, 0, pad_key(src));
        for (;;) {
            uint32_t ln = opaque(lane);
            const uint32_t tb = t + G;
            const bool hb = tb < src.ntiles;
            if (hb) {
                ib = src.get(tb);
                load_tile<P>(b, ib.ks, ib.count, ln, 0, pad_key(src));
            }
            wave_tile<P, SHEAR>(a, ia, src, t, lds, ln);
            if (!hb)
                break;
            ln = opaque(lane);
            t = tb + G;
            const bool ha = t < src.ntiles;
            if (ha) {
                ia = src.get(t);
                load_tile<P>(a, ia.ks, ia.count, ln, 0, pad_key(src));
            }
            wave_tile<P, SHEAR>(b, ib, src, tb, lds, ln);
            if (!ha)
                break;
        }
    }
}

struct RegularGroupSrc {
    __device__ void resolve() {}
    const uint32_t *kin, *vin;
    uint32_t *kout, *vout;
    uint64_t n;
    uint32_t ngroups;
    uint32_t group_keys;
    SampleSet out_smp;
    static constexpr bool kMapped = false;
    __device__ uint64_t pos(uint32_t g, uint32_t w) const { return (uint64_t)g * group_keys + (uint64_t)w * kTile; }
    __device__ uint32_t group_count(uint32_t g) const
    {
        const uint64_t rem = n - (uint64_t)g * group_keys;
        return rem < group_keys ? (uint32_t)rem : group_keys;
    }
    // sub-tile of wave w of group g (count 0 past the end of the input)
    __device__ SortItem get(uint32_t g, uint32_t w) const
    {
        const uint64_t start = (uint64_t)g * group_keys + (uint64_t)w * kTile;
        const uint64_t rem = start < n ? n - start : 0;
        SortItem it;
        it.ks = kin + start;
        it.vs = vin ? vin + start : nullptr;
        it.kd = kout + start;
        it.vd = vout ? vout + start : nullptr;
        it.count = rem < (uint64_t)kTile ? (uint32_t)rem : (uint32_t)kTile;
        return it;
    }
};

// Group tiles of a table launch: tiles[g] covers `count` (<= NW * 4096) keys.
struct TableGroupSrc {
    Bufs kb, vb;
    const BlockTile *tiles;
    uint32_t ngroups;
    SampleSet out_smp;  // always empty
    const uint32_t *count_dev;
    static constexpr bool kMapped = false;
    __device__ void resolve() { ngroups = resolved_count(ngroups, count_dev); }
    __device__ uint64_t pos(uint32_t, uint32_t) const { return 0; }
    __device__ uint32_t group_count(uint32_t g) const { return tiles[g].count; }
    __device__ SortItem get(uint32_t g, uint32_t w) const
    {
        const BlockTile d = tiles[g];
        const uint64_t off = (uint64_t)w * kTile;
        const uint64_t rem = off < d.count ? d.count - off : 0;
        const uint64_t start = d.start + off;
        SortItem it;
        it.ks = kb.in + start;
        it.vs = vb.in ? vb.in + start : nullptr;
        it.kd = (d.dst == kBufOut ? kb.out : kb.temp) + start;
        it.vd = vb.out ? (d.dst == kBufOut ? vb.out : vb.temp) + start : nullptr;
        it.count = rem < (uint64_t)kTile ? (uint32_t)rem : (uint32_t)kTile;
        return it;
    }
};

// Everything of a group tile after its wave's sub-tile is in registers.
template <int NW, bool P, class Src>
__device__ __forceinline__ void group_tile(Lines<P> &t, const SortItem &it, const Src &src, uint32_t g,
                                           uint32_t *lds, uint32_t lane, uint32_t wave)
{
    uint32_t *own = lds + kLdsWords * wave;
    map_tile_in<P>(t, src);
    flip(t, wave);  // odd sub-tiles descending
    sort_tile_blocked<P>(t, own, lane);
    flip(t, wave);
    group_rounds<NW, 7>(t, lds, lane, wave);
    write_samples<P>(t, src.out_smp, src.pos(g, wave), it.count, lane);
    to_strided(t, own, lane);
    if constexpr (P) {
        // group ranks are 4096 * wave + position; wave w stages the values of
        // its own sub-tile, the LDS is shared by all waves of the group
        const SortItem i0 = src.get(g, 0);
        __syncthreads();
        permute_values_lds(t, i0.vs, src.group_count(g), lds, kTile * wave, it.count, lane,
                           [] { __syncthreads(); });
    }
    map_tile_out<P>(t, src);
    store_tile<P>(t, it.kd, it.vd, it.count, lane);
}

// Persistent over group tiles (block b handles groups b, b + grid, ...).  For
// keys the next group's sub-tile is loaded before the current group is
// sorted (two tiles of registers); a pairs tile is twice as large, so pairs
// take one group at a time.  Whether a next group exists is the same for all
// waves of the block, so every wave reaches the same barriers.
template <int NW, bool P, class Src>
__global__ __launch_bounds__(kWave *NW) void k_block_sort_group(Src src)
{
    src.resolve();
    __shared__ __align__(16) uint32_t lds[NW * kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t g = blockIdx.x;
    if (g >= src.ngroups)
        return;
    if constexpr (P) {
        for (; g < src.ngroups; g += gridDim.x) {
            const uint32_t ln = opaque(lane);
            const SortItem it = src.get(g, wave);
            Lines<P> t;
            load_tile<P>(t, it.ks, it.count, ln, wave * kTile, pad_key(src));
            group_tile<NW, P>(t, it, src, g, lds, ln, wave);
        }
    } else {
        Lines<P> a, b;
        SortItem ia = src.get(g, wave), ib;
        load_tile<P>(a, ia.ks, ia.count, lane, 0, pad_key(src));
        for (;;) {
            uint32_t ln = opaque(lane);
            const uint32_t gb = g + gridDim.x;
            const bool hb = gb < src.ngroups;
            if (hb) {
                ib = src.get(gb, wave);
                load_tile<P>(b, ib.ks, ib.count, ln, 0, pad_key(src));
            }
            group_tile<NW, P>(a, ia, src, g, lds, ln, wave);
            if (!hb)
                break;
            ln = opaque(lane);
            g = gb + gridDim.x;
            const bool ha = g < src.ngroups;
            if (ha) {
                ia = src.get(g, wave);
                load_tile<P>(a, ia.ks, ia.count, ln, 0, pad_key(src));
            }
            group_tile<NW, P>(b, ib, src, gb, lds, ln, wave);
            if (!ha)
                break;
        }
    }
}

// ------------------------------------------------ long ShearSort (h waves)
//
// The paper's extension of its base case to M = w^2 h keys sorted by h waves
// (Sec. 3.1, the ShearSort of a w x wh matrix), kept as a block-sort ablation
// against the merge rounds of the group sort.  NW waves hold a grid of 64
// rows and 64 NW columns: lane l of wave v holds, in BLOCKED layout, the
// segment of row l in columns 64v .. 64v + 63, and after the in-wave
// transpose, in STRIDED layout, column 64v + l.  Columns are one lane's
// registers, sorted by Batcher's network.  Rows span the waves: each segment
// is sorted in registers, then a bitonic network over the NW segments of a
// row runs with merge-splits in place of comparators (a lane keeps the lower
// or upper 64 of its own and its partner wave's segment: the elementwise min
// or max against the partner's reversed segment, then an in-lane bitonic
// merge), which sorts blocks by the same argument as the 0-1 principle.  Odd
// rows descend by complementing.  log2(64) = 6 rounds of (rows in snake
// order, columns) and a last ascending row sort leave the grid sorted
// row-major; the paper gathers a row into adjacent columns of one wave and
// sorts it by a segmented ShearSort, here the row stays spread over the waves
// and meets through LDS.  A line permutation then turns row-major grid order
// into the BLOCKED sub-tiles the rest of the group sort expects.

constexpr uint32_t kShearPitch = 4100;  // words per source wave in the line permutation

// Sort 64 registers that form a bitonic sequence, ascending.
__device__ __forceinline__ void bitonic_merge_line(Lines<false> &t)
{
#pragma unroll
    for (int d = kLine / 2; d >= 1; d /= 2)
#pragma unroll
        for (int i = 0; i < kLine; ++i)
            if ((i & d) == 0)
                cx<false>(t, i, i + d);
}

// Every row's NW sorted segments (lane l of each wave) into one sorted row,
// segment v in wave v.  Each step writes the wave's segment to its own LDS
// slice and reads the partner's (lane-consecutive words, conflict-free).
template <int NW>
__device__ __forceinline__ void merge_rows_across_waves(Lines<false> &t, uint32_t *lds, uint32_t lane,
                                                        uint32_t wave)
{
    uint32_t *own = lds + kLdsWords * wave;
#pragma unroll 1
    for (int k = 1; k < NW; k *= 2) {
#pragma unroll 1
        for (int j = k; j >= 1; j /= 2) {
            const uint32_t q = wave ^ (uint32_t)j;
            const bool asc = (wave & (uint32_t)(2 * k)) == 0;
            const bool keep_low = (wave < q) == asc;
#pragma unroll
            for (int r = 0; r < kLine; ++r)
                own[r * kWave + lane] = t.k[r];
            __syncthreads();
            const uint32_t *other = lds + kLdsWords * q;
#pragma unroll
            for (int r = 0; r < kLine; ++r) {
                const uint32_t b = other[(kLine - 1 - r) * kWave + lane];
                t.k[r] = keep_low ? min(t.k[r], b) : max(t.k[r], b);
            }
            __syncthreads();
            bitonic_merge_line(t);
        }
    }
}

template <int NW>
__device__ __forceinline__ void shear_rows(Lines<false> &t, uint32_t *lds, uint32_t lane, uint32_t wave, bool snake)
{
    if (snake)
        flip(t, lane);
    oe_sort<0, kLine - 1, false>(t);
    merge_rows_across_waves<NW>(t, lds, lane, wave);
    if (snake)
        flip(t, lane);
}

// Entry: any registers (the loaded STRIDED tile read as row segments); exit:
// BLOCKED sub-tiles of the sorted group (wave v, lane l, register r holds
// group position 4096 v + 64 l + r).
template <int NW>
__device__ __forceinline__ void long_shear_sort(Lines<false> &t, uint32_t *lds, uint32_t lane, uint32_t wave)
{
    static_assert(NW >= 2 && NW <= 8 && (NW & (NW - 1)) == 0, "NW waves, a power of two dividing 64");
    uint32_t *own = lds + kLdsWords * wave;
#pragma unroll 1
    for (int it = 0; it < 6; ++it) {
        shear_rows<NW>(t, lds, lane, wave, true);
        to_strided(t, own, lane);
        oe_sort<0, kLine - 1, false>(t);
        to_blocked(t, own, lane);
    }
    shear_rows<NW>(t, lds, lane, wave, false);
    // grid position l * 64 NW + 64 v + r is line L = l NW + v of the group;
    // line L goes to lane L mod 64 of wave L / 64.  Source lines are written
    // lane-consecutively, 4100 words per wave, so that the gathering reads
    // (line L = 64 v' + l' from wave L mod NW, lane L / NW) hit 32 banks.
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        lds[kShearPitch * wave + r * kWave + lane] = t.k[r];
    __syncthreads();
    const uint32_t line = kWave * wave + lane, sv = line % NW, sl = line / NW;
#pragma unroll
    for (int r = 0; r < kLine; ++r)
        t.k[r] = lds[kShearPitch * sv + r * kWave + sl];
    __syncthreads();
}

// One group of NW * 4096 keys per work-group: load, long ShearSort, samples, store.
template <int NW, class Src>
__global__ __launch_bounds__(kWave *NW) void k_block_sort_shear_group(Src src)
{
    static_assert(kShearPitch * (NW - 1) + kTile <= (uint32_t)(NW * kLdsWords), "permutation fits the LDS");
    __shared__ __align__(16) uint32_t lds[NW * kLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t g = blockIdx.x;
    if (g >= src.ngroups)
        return;  // the whole work-group: every wave reaches the same barriers
    const SortItem it = src.get(g, wave);
    Lines<false> t;
    load_tile<false>(t, it.ks, it.count, lane);
    long_shear_sort<NW>(t, lds, lane, wave);
    write_samples<false>(t, src.out_smp, src.pos(g, wave), it.count, lane);
    to_strided(t, lds + kLdsWords * wave, lane);
    store_tile<false>(t, it.kd, nullptr, it.count, lane);
}

// Split of every merge tile: splits[t] = co-rank of the tile's first output
// diagonal in its merge (paper Sec. 3.2: the rank of a splitter in each run,
// here computed exactly for every tile boundary).  One half-wave per tile.
template <class Src>
__global__ __launch_bounds__(256) void k_partition(Src src, uint32_t *__restrict__ splits)
{
    src.resolve();
    if (blockIdx.x * 2 * (256 / kWave) >= src.ntiles)
        return;  // no tile of this block (the grid covers the most a planner allows)
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t t = (blockIdx.x * (256 / kWave) + threadIdx.x / kWave) * 2 + (lane >> 5);
    const bool valid = t < src.ntiles;
    MergeItem m = src.get(valid ? t : src.ntiles - 1);
    if (!valid)
        m.na = m.nb = m.d0 = 0;
    const uint32_t split = corank_halfwave(m.ka, m.na, m.ka + m.na, m.nb, m.d0, lane);
    if (valid && (lane & 31) == 0)
        splits[t] = split;
}

// MODE 0: persistent waves, next tile's loads issued before the current tile
//         is merged (keys only; pairs fall back to MODE 1);
// MODE 1: persistent waves, one tile at a time;
// MODE 2: one tile per wave (grid covers every tile).
// One level of the co-rank search: the answer i* (smallest i in [lo, hi] with
// A[i] > B[d-1-i], hi counting as true) is narrowed to a bracket of width
// at most G by a 64-ary search over the candidates i = G*c in [lo, hi).
// pred(i) evaluates the predicate for such a candidate.
template <uint32_t G, class Pred>
__device__ __forceinline__ void corank_level(uint32_t &lo, uint32_t &hi, uint32_t lane, const Pred &pred)
{
    uint32_t c0 = (lo + G - 1) / G;                // first candidate
    uint32_t c1 = hi > 0 ? (hi - 1) / G + 1 : 0;   // one past the last
    while (c0 < c1) {
        const uint32_t span = c1 - c0;
        const uint32_t c = c0 + (uint32_t)(((uint64_t)span * lane) >> 6);  // probe of this lane
        const bool fail = !pred(G * c);
        const uint64_t fails = __ballot(fail);
        const uint32_t cnt = __popcll(fails);  // probes 0..cnt-1 fail (monotone)
        if (cnt == 0) {
            hi = min(hi, G * c0);
            break;
        }
        const uint32_t cf = c0 + (uint32_t)(((uint64_t)span * (cnt - 1)) >> 6);
        lo = max(lo, G * cf + 1);
        if (cnt < 64) {
            const uint32_t cn = c0 + (uint32_t)(((uint64_t)span * cnt) >> 6);
            hi = min(hi, G * cn);
            c1 = cn;
        }
        c0 = cf + 1;
    }
}

// corank_level for a half-wave: lanes 0..31 and 32..63 each narrow their own
// bracket (two independent searches per wave) with 32 probes per round.
template <uint32_t G, class Pred>
__device__ __forceinline__ void corank_level_half(uint32_t &lo, uint32_t &hi, uint32_t lane, const Pred &pred)
{
    const uint32_t k = lane & 31;
    const uint32_t shift = lane & 32;
    uint32_t c0 = (lo + G - 1) / G;
    uint32_t c1 = hi > 0 ? (hi - 1) / G + 1 : 0;
    while (__ballot(c0 < c1) != 0) {
        const bool act = c0 < c1;
        const uint32_t span = act ? c1 - c0 : 0;
        const uint32_t c = c0 + (uint32_t)(((uint64_t)span * k) >> 5);  // probe of this lane
        const bool fail = act && !pred(G * c);
        const uint32_t cnt = __popc((uint32_t)(__ballot(fail) >> shift));  // probes 0..cnt-1 fail
        if (act) {
            if (cnt == 0) {
                hi = min(hi, G * c0);
                c1 = c0;
            } else {
                const uint32_t cf = c0 + (uint32_t)(((uint64_t)span * (cnt - 1)) >> 5);
                lo = max(lo, G * cf + 1);
                if (cnt < 32) {
                    const uint32_t cn = c0 + (uint32_t)(((uint64_t)span * cnt) >> 5);
                    hi = min(hi, G * cn);
                    c1 = cn;
                }
                c0 = cf + 1;
            }
        }
    }
}

// Three-level sampled co-rank search of diagonal d of merge item m by a
// half-wave (see k_partition_sampled); [lo, hi] is the initial bracket.
__device__ __forceinline__ void corank_sampled_half(const SampleSet &sm, const MergeItem &m, uint32_t d,
                                                    uint32_t lane, uint32_t &lo, uint32_t &hi)
{
    const uint32_t na = m.na;
    const uint64_t apos = m.base, bpos = m.base + na;
    const uint32_t *A = m.ka, *B = m.ka + na;
    auto tile_pred = [&](uint32_t i) { return sm.cf[(apos + i) / kTile] > sm.cl[(bpos + d - 1 - i) / kTile]; };
    auto block_pred = [&](uint32_t i) { return sm.f[(apos + i) / kLine] > sm.l[(bpos + d - 1 - i) / kLine]; };
    auto key_pred = [&](uint32_t i) { return A[i] > B[d - 1 - i]; };
    if (sm.cf != nullptr)
        corank_level_half<kTile>(lo, hi, lane, tile_pred);
    else  // tile samples are every 64th block sample
        corank_level_half<kTile>(lo, hi, lane, block_pred);
    corank_level_half<kLine>(lo, hi, lane, block_pred);
    corank_level_half<1>(lo, hi, lane, key_pred);
}

// Co-rank of every merge tile of a regular pass from the samples the
// previous launch wrote: three exact levels (tile samples, 64-block samples,
// keys), by one wave per tile (HALF = false: 64 probes per round) or by one
// half-wave per tile (HALF = true: 32 probes per round, half the waves, so a
// launch's searches are all resident at once).  Tile diagonals are multiples
// of 4096 and runs start at multiples of 4096, so for a candidate i that is a
// multiple of 64 (4096), A[i] is a first-of-block sample and B[d-1-i] a
// last-of-block sample.
template <bool HALF>
__global__ __launch_bounds__(256) void k_partition_sampled(RegularMergeSrc src, uint32_t *__restrict__ splits)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t w = __builtin_amdgcn_readfirstlane(blockIdx.x * (256 / kWave) + threadIdx.x / kWave);
    const uint32_t t = HALF ? 2 * w + (lane >> 5) : w;
    if ((HALF ? 2 * w : w) >= src.ntiles)
        return;  // the whole wave is past the last tile
    const bool valid = t < src.ntiles;
    const MergeItem m = src.get(valid ? t : src.ntiles - 1);
    const uint32_t d = m.d0, na = m.na, nb = m.nb;
    uint32_t lo = d > nb ? d - nb : 0;
    uint32_t hi = d < na ? d : na;
    if (!valid)
        lo = hi = 0;  // no search in this half
    const uint64_t apos = m.base, bpos = m.base + na;
    const SampleSet &sm = src.in_smp;
    const uint32_t *A = m.ka, *B = m.ka + na;
    auto tile_pred = [&](uint32_t i) { return sm.cf[(apos + i) / kTile] > sm.cl[(bpos + d - 1 - i) / kTile]; };
    auto block_pred = [&](uint32_t i) { return sm.f[(apos + i) / kLine] > sm.l[(bpos + d - 1 - i) / kLine]; };
    auto key_pred = [&](uint32_t i) { return A[i] > B[d - 1 - i]; };
    if constexpr (HALF) {
        corank_sampled_half(sm, m, d, lane, lo, hi);
        if (valid && (lane & 31) == 0)
            splits[t] = lo;
    } else {
        if (sm.cf != nullptr)
            corank_level<kTile>(lo, hi, lane, tile_pred);
        else
            corank_level<kTile>(lo, hi, lane, block_pred);
        corank_level<kLine>(lo, hi, lane, block_pred);
        corank_level<1>(lo, hi, lane, key_pred);
        if (lane == 0)
            splits[t] = lo;
    }
}

// The split of merge tile t computed in the merge kernel itself from the
// samples of its input (regular passes): lanes 0..31 search the tile's first
// diagonal, lanes 32..63 its end, at the same time.
__device__ __forceinline__ void fused_splits(const RegularMergeSrc &src, const MergeItem &m, uint32_t lane,
                                             uint32_t &a0, uint32_t &a1)
{
    const uint32_t d = lane < 32 ? m.d0 : m.d0 + m.count;
    uint32_t lo = d > m.nb ? d - m.nb : 0;
    uint32_t hi = d < m.na ? d : m.na;
    corank_sampled_half(src.in_smp, m, d, lane, lo, hi);
    a0 = __builtin_amdgcn_readlane(lo, 0);
    a1 = __builtin_amdgcn_readlane(lo, 32);
}

// Other sources (tables) never fuse; a regular source that carries a key map
// (derived from RegularMergeSrc) searches like its base.
template <class Src>
__device__ __forceinline__ void fused_splits(const Src &src, const MergeItem &m, uint32_t lane, uint32_t &a0,
                                             uint32_t &a1)
{
    if constexpr (std::is_base_of_v<RegularMergeSrc, Src>)
        fused_splits(static_cast<const RegularMergeSrc &>(src), m, lane, a0, a1);
}

// Work-groups of the one-tile-per-wave merge (MODE 2) hold a single wave: the
// LDS of a wave (its transpose area) is then the unit of residency, and a CU
// keeps nine such waves instead of eight in groups of two (measured: 102 vs
// 107 us per binary pass at 2^26 keys).
constexpr int kMergeTileWaves = 1;

template <int MODE>
constexpr int merge_group_waves() { return MODE == 2 ? kMergeTileWaves : kWavesPerGroup; }

template <bool P, class Src, int MODE, bool NT = false, bool FUSED = false>
__global__ __launch_bounds__(kWave *merge_group_waves<MODE>()) void k_merge(Src src, const uint32_t *__restrict__ splits)
{
    src.resolve();
    constexpr int W = merge_group_waves<MODE>();  // waves per work-group
    // per wave: the transpose area, then (pairs) the tile's staged values
    constexpr int kWaveWords = kLdsWords + (P ? kTile : 0);
    __shared__ __align__(16) uint32_t lds_all[W][kWaveWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t *lds = lds_all[wave];
    uint32_t *vals = lds + kLdsWords;
    const uint32_t G = gridDim.x * W;
    uint32_t t = blockIdx.x * W + wave;
    if (t >= src.ntiles)
        return;
    if constexpr (MODE == 2) {
        MergeTask<P> m;
        if constexpr (FUSED) {
            const MergeItem mi = src.get(t);
            uint32_t a0, a1;
            fused_splits(src, mi, lane, a0, a1);
            m = merge_task_at<P>(mi, a0, a1);
        } else {
            m = merge_task<P>(src, splits, t);
        }
        Lines<P> a;
        merge_load<P, NT>(a, m, lane);
        if constexpr (P)
            stage_merge_values(m, vals, lane);
        merge_network<P>(a, lds, lane, src.out_smp, m.gpos, m.count);
        if constexpr (P)
            gather_values(a, m, vals, lane);
        map_tile_out<P>(a, src);
        store_tile<P, NT>(a, m.kd, m.vd, m.count, lane);
    } else if constexpr (P || MODE == 1) {
        for (; t < src.ntiles; t += G) {
            const uint32_t ln = opaque(lane);
            const MergeTask<P> m = merge_task<P>(src, splits, t);
            Lines<P> a;
            merge_load<P, NT>(a, m, ln);
            if constexpr (P)
                stage_merge_values(m, vals, ln);
            merge_network<P>(a, lds, ln, src.out_smp, m.gpos, m.count);
            if constexpr (P)
                gather_values(a, m, vals, ln);
            map_tile_out<P>(a, src);
            store_tile<P, NT>(a, m.kd, m.vd, m.count, ln);
        }
    } else {
        Lines<P> a, b;
        MergeTask<P> ma = merge_task<P>(src, splits, t), mb;
        merge_load<P>(a, ma, lane);
        for (;;) {
            uint32_t ln = opaque(lane);
            const uint32_t tb = t + G;
            const bool hb = tb < src.ntiles;
            if (hb) {
                mb = merge_task<P>(src, splits, tb);
                merge_load<P>(b, mb, ln);
            }
            merge_network<P>(a, lds, ln, src.out_smp, ma.gpos, ma.count);
            map_tile_out<P>(a, src);
            store_tile<P>(a, ma.kd, ma.vd, ma.count, ln);
            if (!hb)
                break;
            ln = opaque(lane);
            t = tb + G;
            const bool ha = t < src.ntiles;
            if (ha) {
                ma = merge_task<P>(src, splits, t);
                merge_load<P>(a, ma, ln);
            }
            merge_network<P>(b, lds, ln, src.out_smp, mb.gpos, mb.count);
            map_tile_out<P>(b, src);
            store_tile<P>(b, mb.kd, mb.vd, mb.count, ln);
            if (!ha)
                break;
        }
    }
}

// ------------------------------------------------ fan-in 4 merge passes
//
// A fan-in 4 pass merges groups of four consecutive runs A, B, C, D of
// length L (a multiple of 4096) into runs of 4L: two levels of the paper's
// binary merging (Sec. 3.2; AB = merge(A, B), CD = merge(C, D), then
// merge(AB, CD), equal keys in run order) for one read and one write of the
// data instead of two of each.  Neither AB nor CD is ever written.
//
// Work split.  Point (x, y) of a group's four-way merge path is the moment
// when x elements of AB and y of CD have been output.  The path is cut
//   * at every AB position x = kAbStep j (an AB cut: the binary co-rank of A
//     and B at x gives the A/B split, the key k = AB[x] is read, and y counts
//     the C and D keys below k, which come after it), and
//   * at every CD position y = kCdStep m (a CD cut: the same with the roles
//     swapped; A and B keys equal to its key come before it).
// Both kinds need only searches in single sorted runs, none inside a virtual
// sequence.  Consecutive AB cuts bound a segment: kAbStep elements of AB (the
// last one fewer) and any number of CD.  A segment whose CD side holds at most
// kCdStep keys is one merge item; a longer segment is cut again at the CD
// cuts strictly inside it.  So every item holds at most kAbStep keys of AB and
// kCdStep of CD and fits one tile, AB in its lower half and CD in its upper
// half (two networks), and where the runs interleave evenly a segment is one
// item of about 2 kAbStep outputs however far the path strays from the
// diagonal.  A CD cut that does not lie strictly inside a long segment starts
// no item.

constexpr uint32_t kHalfTile = kTile / 2;
static_assert(kAbStep % kLine == 0 && kCdStep % kLine == 0 && kAbStep <= kHalfTile && kCdStep <= kHalfTile,
              "cut steps");

// The runs of group g of a fan-in 4 pass over n keys with runs of L.
struct Group4 {
    uint64_t start;  // array position of A[0]
    uint32_t n[4];   // lengths of A, B, C, D (runs past the end are empty)
    uint32_t J, M;   // AB segments, interior CD cuts
    __device__ Group4() {}
    __device__ Group4(uint64_t nkeys, uint64_t L, uint32_t g)
    {
        start = (uint64_t)g * 4 * L;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint64_t s = start + r * L;
            const uint64_t rem = nkeys > s ? nkeys - s : 0;
            n[r] = (uint32_t)(rem < L ? rem : L);
        }
        J = ab_segments((uint64_t)n[0] + n[1]);
        M = cd_cuts((uint64_t)n[2] + n[3]);
    }
};

// Cut list of a pass: per group, the AB cuts P[0..jfull] (P[0] = nothing
// taken, P[J] = everything) followed by the CD cuts Q[0..mfull] (Q[0] unused),
// each as the counts (a, b, c, d) taken from A, B, C and D before the cut.
struct Merge4Src {
    const uint32_t *ksrc;
    uint32_t *kdst;
    uint64_t n, run;
    uint32_t groups;
    uint32_t jfull, mfull;  // AB segments and interior CD cuts of a full group
    uint4 *cuts;
    SampleSet in_smp, out_smp;
    KeyMap out_map;
    const uint32_t *vsrc = nullptr;  // key/value passes: the values, laid out like the keys
    uint32_t *vdst = nullptr;
    __host__ __device__ uint32_t stride() const { return jfull + mfull + 2; }
};

// One level of a monotone search by groups of 2^LOGP lanes, each group with
// its own bracket and predicate: the smallest i in [lo, hi] with pred(i)
// (hi counting as true) is narrowed to a bracket of width at most G by
// 2^LOGP-ary rounds over the candidates i = G*c in [lo, hi).
template <uint32_t G, int LOGP, class Pred>
__device__ __forceinline__ void search_level(uint32_t &lo, uint32_t &hi, uint32_t lane, const Pred &pred)
{
    constexpr uint32_t P = 1u << LOGP;
    constexpr uint64_t kMask = P == 64 ? ~0ull : ((1ull << P) - 1);
    const uint32_t k = lane & (P - 1);
    const uint32_t shift = lane & ~(P - 1);
    uint32_t c0 = (lo + G - 1) / G;
    uint32_t c1 = hi > 0 ? (hi - 1) / G + 1 : 0;
    while (__ballot(c0 < c1) != 0) {
        const bool act = c0 < c1;
        const uint32_t span = act ? c1 - c0 : 0;
        const uint32_t c = c0 + (uint32_t)(((uint64_t)span * k) >> LOGP);  // probe of this lane
        const bool fail = act && !pred(G * c);
        const uint32_t cnt = __popcll((__ballot(fail) >> shift) & kMask);  // probes 0..cnt-1 fail
        if (act) {
            if (cnt == 0) {
                hi = min(hi, G * c0);
                c1 = c0;
            } else {
                const uint32_t cf = c0 + (uint32_t)(((uint64_t)span * (cnt - 1)) >> LOGP);
                lo = max(lo, G * cf + 1);
                if (cnt < P) {
                    const uint32_t cn = c0 + (uint32_t)(((uint64_t)span * cnt) >> LOGP);
                    hi = min(hi, G * cn);
                    c1 = cn;
                }
                c0 = cf + 1;
            }
        }
    }
}

// The same partition by persistent waves, for launches whose tile count is
// only known on the device (the binary steps of device-planned segmented
// sorts and run merges): each split is searched on the keys by four lanes
// (4-ary rounds, sixteen searches per wave), which fetch fewer lines per
// round than a half-wave's 32 probes, as for the table cut searches.
constexpr int kPartLanesLog = 2;
constexpr uint32_t kPartsPerWave = kWave >> kPartLanesLog;

template <class Src>
__global__ __launch_bounds__(256) void k_partition_persist(Src src, uint32_t *__restrict__ splits)
{
    src.resolve();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t stride = gridDim.x * (256 / kWave) * kPartsPerWave;
    for (uint32_t t0 = (blockIdx.x * (256 / kWave) + threadIdx.x / kWave) * kPartsPerWave; t0 < src.ntiles;
         t0 += stride) {
        const uint32_t t = t0 + (lane >> kPartLanesLog);
        const bool valid = t < src.ntiles;
        MergeItem m = src.get(valid ? t : src.ntiles - 1);
        if (!valid)
            m.na = m.nb = m.d0 = 0;
        const uint32_t *A = m.ka, *B = m.ka + m.na;
        const uint32_t d = m.d0;
        uint32_t lo = d > m.nb ? d - m.nb : 0, hi = d < m.na ? d : m.na;
        search_level<1, kPartLanesLog>(lo, hi, lane, [&](uint32_t i) { return A[i] > B[d - 1 - i]; });
        if (valid && (lane & ((1u << kPartLanesLog) - 1)) == 0)
            splits[t] = lo;
    }
}

// Cut searches, eight per wave: the 8-lane part q of wave w takes task
// 8w + q; task t of group g is AB cut t + 1 (t < jfull - 1) or CD cut
// t - jfull + 2.  A part first finds the binary split of its cut's own side
// (three sampled levels, 8 probes per round; the cut position is a multiple
// of 64, so the first two levels read block samples), reads the cut's key,
// then counts that key in the other side's two runs with one 4-lane group
// per run at the same time.  Task 0 of a group also writes the group's end
// points P[0] and P[J].  The searches are bound by how many are in flight
// more than by their rounds: measured at 2^26 keys, eight searches per wave
// take 12-21 us per launch, four (16 lanes each) 13-24 us, two 18-32 us, one
// (64-lane rounds) 28-41 us, sixteen (4 lanes each) between eight and four.
constexpr int kCutLanesLog = 3;                     // 8 lanes per search
constexpr uint32_t kCutLanes = 1u << kCutLanesLog;
constexpr uint32_t kCutsPerWave = kWave / kCutLanes;

__global__ __launch_bounds__(256) void k_cuts4(Merge4Src src)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t part = lane / kCutLanes;  // this search's lanes: kCutLanes part .. + kCutLanes - 1
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (256 / kWave) + threadIdx.x / kWave);
    const uint32_t per = src.jfull - 1 + src.mfull;  // cut searches of a full group
    const uint32_t task = kCutsPerWave * wave + part;
    const uint32_t g = task / per, t = task % per;
    const bool in_range = g < src.groups;
    const Group4 G(src.n, src.run, in_range ? g : 0);
    uint4 *cuts = src.cuts + (uint64_t)(in_range ? g : 0) * src.stride();
    if (in_range && t == 0 && (lane & (kCutLanes - 1)) == 0) {
        cuts[0] = make_uint4(0, 0, 0, 0);
        cuts[G.J] = make_uint4(G.n[0], G.n[1], G.n[2], G.n[3]);
    }
    const bool ab = t + 1 < src.jfull;
    const uint32_t idx = ab ? t + 1 : t + 2 - src.jfull;  // AB cut j or CD cut m
    const bool valid = in_range && (ab ? idx < G.J : idx <= G.M);
    if (__ballot(valid) == 0)
        return;
    const uint64_t L = src.run;
    const SampleSet &sm = src.in_smp;
    const uint32_t r0 = ab ? 0 : 2;  // first run of the cut's own side
    const uint32_t n0 = ab ? G.n[0] : G.n[2], n1 = ab ? G.n[1] : G.n[3];
    const uint32_t d = ab ? idx * kAbStep : idx * kCdStep;
    const uint64_t apos = G.start + r0 * L, bpos = apos + n0;
    const uint32_t *A = src.ksrc + apos, *B = A + n0;
    uint32_t lo = d > n1 ? d - n1 : 0, hi = d < n0 ? d : n0;
    if (!valid)
        lo = hi = 0;
    auto block_pred = [&](uint32_t i) { return sm.f[(apos + i) / kLine] > sm.l[(bpos + d - 1 - i) / kLine]; };
    search_level<kTile, kCutLanesLog>(lo, hi, lane, block_pred);  // 4096 candidates apart
    search_level<kLine, kCutLanesLog>(lo, hi, lane, block_pred);
    search_level<1, kCutLanesLog>(lo, hi, lane, [&](uint32_t i) { return A[i] > B[d - 1 - i]; });
    const uint32_t s0 = lo, s1 = d - s0;
    uint32_t k = 0;
    if (valid)
        k = (s0 < n0 && (s1 >= n1 || A[s0] <= B[s1])) ? A[s0] : B[s1];
    // the other side: the upper half of a search's lanes counts in its second
    // run.  An AB cut counts keys below k (C and D keys equal to k follow it),
    // a CD cut keys at most k (A and B keys equal to k precede it).
    const uint32_t ro = (ab ? 2 : 0) + ((lane / (kCutLanes / 2)) & 1);
    const uint32_t nr = valid ? (ro == 0 ? G.n[0] : ro == 1 ? G.n[1] : ro == 2 ? G.n[2] : G.n[3]) : 0;
    const uint64_t rpos = G.start + ro * L;
    const uint32_t *R = src.ksrc + rpos;
    const bool strict = !ab;
    auto above = [&](uint32_t v) { return strict ? v > k : v >= k; };
    uint32_t rlo = 0, rhi = nr;
    search_level<kTile, kCutLanesLog - 1>(rlo, rhi, lane, [&](uint32_t i) {
        return sm.cf != nullptr ? above(sm.cf[(rpos + i) / kTile]) : above(sm.f[(rpos + i) / kLine]);
    });
    search_level<kLine, kCutLanesLog - 1>(rlo, rhi, lane, [&](uint32_t i) { return above(sm.f[(rpos + i) / kLine]); });
    search_level<1, kCutLanesLog - 1>(rlo, rhi, lane, [&](uint32_t i) { return above(R[i]); });
    // the counts of this search's two groups (its first lane and the one half
    // way up), fetched from those lanes
    const uint32_t first = lane & ~(kCutLanes - 1);
    const uint32_t o0 = __shfl(rlo, first), o1 = __shfl(rlo, first + kCutLanes / 2);
    if (!valid || (lane & (kCutLanes - 1)) != 0)
        return;
    if (ab)
        cuts[idx] = make_uint4(s0, s1, o0, o1);
    else
        cuts[src.jfull + 1 + idx] = make_uint4(o0, o1, s0, s1);
}

// The four-way merge works with the half-width transposes (9 KiB of LDS per
// wave, see to_blocked_half): with its registers held to 128 four waves fit
// per SIMD, so loads of some items overlap the networks of others.

// Half-cleaners on position bits 11..6 of a STRIDED tile (register bits),
// then the transpose to BLOCKED and bits 5..0: a bitonic tile ends sorted in
// BLOCKED layout.
__device__ __forceinline__ void merge4_network(Lines<false> &t, uint32_t *lds, uint32_t lane)
{
    half_clean<kLine / 2, -1, false>(t);
    to_blocked_half(t, lds, lane);
    half_clean<kLine / 2, -1, false>(t);
}

// Store the first `count` positions of a STRIDED tile (count <= 4096) at dst
// through a raw buffer resource whose range is those count keys: the memory
// system drops every store past the range, so no lane is masked per
// register.  The whole offset of a register (lane + 64 r keys) is passed in the
// vector offset, the part of the address that the range check covers.
template <bool NT>
__device__ __forceinline__ void store_bounded(const uint32_t (&x)[kLine], uint32_t *dst, uint32_t count,
                                              uint32_t lane)
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)(count * 4u), 0x00020000);
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        if ((uint32_t)(kWave * r) >= count)
            break;  // wave-uniform: rows past the end hold padding only
        const uint32_t off = opaque(4u * (kWave * r + lane));
        __builtin_amdgcn_raw_buffer_store_b32(x[r], rs, (int)off, 0, NT ? 2 : 0);
    }
}
template <bool NT>
__device__ __forceinline__ void store_bounded(const Lines<false> &t, uint32_t *dst, uint32_t count, uint32_t lane)
{
    store_bounded<NT>(t.k, dst, count, lane);
}

// Word i (0..3) of the 16 bytes at LDS word w (w a multiple of 4), for a
// wave-uniform i.  The read is volatile so that the compiler keeps it one
// 16-byte read: narrowed to the one 4-byte word, lanes 36 words apart would
// meet 4-way in the banks.
__device__ __forceinline__ uint32_t lds_word_of_quad(const uint32_t *w, uint32_t i)
{
    typedef uint32_t quad __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) const volatile quad lds_quad;
    const quad v = *(lds_quad *)w;
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// A sorted BLOCKED tile to the array: back to STRIDED through the half-width
// matrices, then `count` keys stored at array position gpos, with the samples
// of the output that fall inside it (first and last key of every 64-key block
// and every 4096-key tile of the array).  Tile position bf + 64k starts a
// block of the array and bl + 64k ends one (bf = -gpos mod 64, bl = bf - 1
// mod 64): in BLOCKED layout that is register bf (bl) of lane k, read back
// from the LDS matrix while it holds the lane's registers (16-byte reads, one
// per sample: no bank conflicts).
template <bool NT, bool MAP>
__device__ __forceinline__ void emit_blocked(Lines<false> &t, uint32_t *lds, uint32_t *kdst, uint64_t gpos,
                                             uint32_t count, const SampleSet &smp, const KeyMap &km, uint32_t lane)
{
    const uint32_t bf = (uint32_t)((kLine - gpos % kLine) % kLine);
    const uint32_t bl = (bf + kLine - 1) % kLine;
    uint32_t *m = half_matrix(lds, lane);
    const uint32_t li = lane & 31;
    uint32_t *row = static_cast<uint32_t *>(__builtin_assume_aligned(m + kHalfStride * li, 16));
    const bool want = smp.f != nullptr;
    uint32_t f = 0, l = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        constexpr int H = kLine / 2;
#pragma unroll
        for (int c = 0; c < H; ++c)
            row[c] = t.k[h * H + c];
        wave_lds_fence();
        if (want && bf / H == (uint32_t)h)
            f = lds_word_of_quad(row + (bf % H) / 4 * 4, bf % 4);
        if (want && bl / H == (uint32_t)h)
            l = lds_word_of_quad(row + (bl % H) / 4 * 4, bl % 4);
#pragma unroll
        for (int r = 0; r < H; ++r)
            t.k[h * H + r] = m[kHalfStride * r + li];
        wave_lds_fence();
    }
    swap_quadrants(t.k);
    lane = opaque(lane);
    if (want) {
        const uint32_t pf = bf + kLine * lane, pl = bl + kLine * lane;
        if (pf < count) {
            const uint64_t gp = gpos + pf;
            smp.f[gp / kLine] = f;
            if (smp.cf != nullptr && gp % kTile == 0)
                smp.cf[gp / kTile] = f;
        }
        if (pl < count) {
            const uint64_t gp = gpos + pl;
            smp.l[gp / kLine] = l;
            if (smp.cf != nullptr && gp % kTile == kTile - 1)
                smp.cl[gp / kTile] = l;
        }
    }
    if constexpr (MAP)
        map_tile_out<false>(t, km);
    store_bounded<NT>(t, kdst + gpos, count, lane);
}

// An item of one piece (count <= 2048 keys, already sorted) copied to array
// position gpos with the samples that fall inside it, by coalesced loads and
// stores: every lane moves the elements lane + 64 k.
template <bool NT, bool MAP>
__device__ __forceinline__ void copy4(const uint32_t *x, uint32_t *kdst, uint64_t gpos, uint32_t count,
                                      const SampleSet &smp, const KeyMap &km, uint32_t lane)
{
    constexpr int kRows = kHalfTile / kWave;
    uint32_t v[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const uint32_t i = kWave * k + lane;
        v[k] = ld<false>(x + (i < count ? i : count - 1));  // clamped: always inside the piece
    }
    if constexpr (MAP) {
#pragma unroll
        for (int k = 0; k < kRows; ++k)
            v[k] = map_key(v[k], km.sign, km.rest, km.inverse);
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const uint32_t i = kWave * k + lane;
        if (i < count) {
            const uint64_t gp = gpos + i;
            st<NT>(kdst + gp, v[k]);
            if (smp.f != nullptr) {
                if (gp % kLine == 0)
                    smp.f[gp / kLine] = v[k];
                if (gp % kLine == kLine - 1)
                    smp.l[gp / kLine] = v[k];
                if (smp.cf != nullptr && gp % kTile == 0)
                    smp.cf[gp / kTile] = v[k];
                if (smp.cf != nullptr && gp % kTile == kTile - 1)
                    smp.cl[gp / kTile] = v[k];
            }
        }
    }
}

// Keys that padding positions load: every one the maximum key.
__device__ const uint32_t kPadKeys[kWave] = {
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey,
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey,
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey,
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey,
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey,
    kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey, kMaxKey};

// A merge item's tile: each half of 2048 positions takes a front piece
// (front[h], fn[h] keys, ascending at positions [0, fn)) and a back piece
// (bn[h] keys, reversed at [2048 - bn, 2048): position q reads element
// bend[h] - q), with padding (the maximum key) between; offsets count from
// the group's first key.  The upper half is XORed with xm (0, or ~0 to
// complement it: an order-reversing bijection that turns padding into 0).
struct HalfPieces {
    uint32_t front[2], fn[2], bend[2], bn[2];
    uint32_t xm;
};

// Load an item's tile in STRIDED layout.  Every lane computes one address
// per register, from the pieces or from kPadKeys, and issues every load
// before any of them is used (branch-free: one select of two addresses).
template <bool NT>
__device__ __forceinline__ void load_item(Lines<false> &t, const uint32_t *K, const HalfPieces &hp, uint32_t lane)
{
    typedef __attribute__((address_space(1))) const uint32_t gkey;
    const uint32_t ln = opaque(lane);  // positions are not kept for the stores
    gkey *kg = (gkey *)K, *pad = (gkey *)kPadKeys + ln;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const int h = r / (kLine / 2);
        const uint32_t q = kWave * (r % (kLine / 2)) + ln;  // position in the half
        const bool in_f = q < hp.fn[h], in_b = q >= kHalfTile - hp.bn[h];
        const uint32_t off = in_f ? hp.front[h] + q : hp.bend[h] - q;
        gkey *a = (in_f || in_b) ? kg + off : pad;
        if constexpr (NT)
            t.k[r] = __builtin_nontemporal_load(a);
        else
            t.k[r] = *a;
        // each address right before its load: only the loaded keys stay live
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = kLine / 2; r < kLine; ++r)
        t.k[r] ^= hp.xm;
}

// Both halves of a packed item merged at once (the network without its top
// stage: position bits 10..0), back to STRIDED, and the CD half complemented
// back: AB ascending followed by CD descending, one bitonic sequence.
__device__ __forceinline__ void packed_network(Lines<false> &t, uint32_t *lds, uint32_t lane)
{
    half_clean<kLine / 4, -1, false>(t);
    to_blocked_half(t, lds, lane);
    half_clean<kLine / 2, -1, false>(t);
    to_strided_half(t, lds, lane);
#pragma unroll
    for (int r = kLine / 2; r < kLine; ++r)
        t.k[r] = ~t.k[r];
}

constexpr int kMerge4Waves = 1;  // one wave per work-group (see kMergeTileWaves)

// The cuts that bound item slot i of a group (AB items in slots
// 0 .. abslots - 1, then CD items), read as scalars: false when the slot holds
// no item.  P: the AB cuts P[0..J], Q: the CD cuts Q[0..M] (Q[0] unused).
__device__ __forceinline__ bool item_cuts(const uint4 *P, const uint4 *Q, const Group4 &G, uint32_t i,
                                          uint32_t abslots, uint4 &c0, uint4 &c1)
{
    // a cut is the same in every lane: scalar values, so that every branch
    // below is a scalar one
    auto cut = [](const uint4 *p) {
        const uint4 c = *p;
        return make_uint4(__builtin_amdgcn_readfirstlane(c.x), __builtin_amdgcn_readfirstlane(c.y),
                          __builtin_amdgcn_readfirstlane(c.z), __builtin_amdgcn_readfirstlane(c.w));
    };
    if (i < abslots) {
        if (i >= G.J)
            return false;
        c0 = cut(P + i);
        const uint4 pe = cut(P + i + 1);
        const uint32_t y0 = c0.z + c0.w, y1 = pe.z + pe.w;
        if (y1 < y0)
            return false;
        c1 = y1 - y0 > kCdStep ? cut(Q + y0 / kCdStep + 1) : pe;
    } else {
        const uint32_t m = i - abslots + 1;
        if (m > G.M)
            return false;
        c0 = cut(Q + m);
        const uint4 qn = cut(Q + (m < G.M ? m + 1 : m));
        const uint32_t xq = c0.x + c0.y, gm = kCdStep * m;
        // the segment holding Q[m]: jc, or jc - 1 when P[jc] sits at Q[m]'s AB
        // position but after it (more CD taken)
        const uint32_t jc = min(G.J - 1, xq / kAbStep);
        const uint4 pm = cut(P + (jc > 0 ? jc - 1 : 0)), pc = cut(P + jc), pn = cut(P + jc + 1);
        const bool before = jc > 0 && pc.x + pc.y == xq && pc.z + pc.w > gm;
        const uint4 p0 = before ? pm : pc, p1 = before ? pc : pn;
        const uint32_t y0 = p0.z + p0.w, y1 = p1.z + p1.w;
        if (!(y1 > y0 + kCdStep && y0 < gm && gm < y1))
            return false;  // not inside a long segment: the AB item covers it
        c1 = (m < G.M && kCdStep * (m + 1) < y1) ? qn : p1;
    }
    // every piece inside its run, each side within its half tile (holds for
    // cuts written by the cut search; checked so that no cut can move a load
    // or a store outside the group)
    if (c0.x > c1.x || c0.y > c1.y || c0.z > c1.z || c0.w > c1.w || c1.x > G.n[0] || c1.y > G.n[1] ||
        c1.z > G.n[2] || c1.w > G.n[3])
        return false;
    return true;
}

// Merge one item: the keys between cuts c0 and c1 of group G, whose runs B,
// C and D start ob, oc and od keys after A[0] = K[0]; written to kdst at the
// group's output position.  NT marks the stores nontemporal, never the
// loads (measured at 2^26 keys over the five distributions: 116.8 us per
// launch with nontemporal stores only, 119.9 with both, 125.1 with loads only).
template <bool NT, bool MAP>
__device__ __forceinline__ void merge4_item(const Group4 &G, const uint4 &c0, const uint4 &c1, const uint32_t *K,
                                            uint32_t ob0, uint32_t oc0, uint32_t od0, uint32_t *kdst,
                                            const SampleSet &out_smp, const KeyMap &km, uint32_t *lds, uint32_t lane)
{
    const uint32_t pa = c1.x - c0.x, pb = c1.y - c0.y, pc = c1.z - c0.z, pd = c1.w - c0.w;
    const uint32_t sx = pa + pb, sy = pc + pd, count = sx + sy;
    if (count == 0 || sx > kHalfTile || sy > kHalfTile)
        return;
    const uint64_t gpos = G.start + c0.x + c0.y + c0.z + c0.w;
    const uint32_t pieces = (pa != 0) + (pb != 0) + (pc != 0) + (pd != 0);
    // offsets from A[0] of the four pieces' first keys
    const uint32_t oa = c0.x, ob = ob0 + c0.y, oc = oc0 + c0.z, od = od0 + c0.w;
    if (pieces == 1) {
        // one piece: already sorted, copied as it is (no network, no LDS)
        copy4<NT, MAP>(K + (pa ? oa : pb ? ob : pc ? oc : od), kdst, gpos, count, out_smp, km, lane);
        return;
    }
    HalfPieces hp;
    if (pieces >= 3) {
        // A ascending and B reversed in the lower half, C and D likewise in
        // the upper half, complemented
        hp = HalfPieces{{oa, oc}, {pa, pc}, {ob + kHalfTile - 1, od + kHalfTile - 1}, {pb, pd}, ~0u};
    } else {
        // the first nonempty piece X ascending at the front of the lower half,
        // the second one Y (if any) reversed at the back of the upper half
        const uint32_t ox = pa ? oa : pb ? ob : pc ? oc : od;
        const uint32_t nx = pa ? pa : pb ? pb : pc ? pc : pd;
        const uint32_t oy = (pa && pb) ? ob : ((pa || pb) && pc) ? oc : od;
        const uint32_t ny = pieces == 2 ? count - nx : 0;
        hp = HalfPieces{{ox, 0}, {nx, 0}, {0, oy + kHalfTile - 1}, {0, ny}, 0u};
    }
    Lines<false> t;
    load_item<false>(t, K, hp, lane);
    if (pieces >= 3)
        packed_network(t, lds, lane);
    merge4_network(t, lds, lane);
    emit_blocked<NT, MAP>(t, lds, kdst, gpos, count, out_smp, km, lane);
}

// One wave per merge item (at most kAbStep keys of AB and kCdStep of CD).
// Items of three or four pieces load AB into the lower and CD into the upper
// half of one tile and take two networks (both halves merged at once, then
// the whole tile); items of one or two pieces load the first piece ascending
// at the front and the second reversed at the back (one bitonic tile, already
// sorted for one piece) and take the second network only; items of one piece
// are copied (copy4).  The tile code has one branch (around the first
// network), so the kernel fits 110 registers: four waves per SIMD, as many as
// the 9 KiB of LDS per wave allow.  Keys only:
// equal keys are indistinguishable, so only the cuts (exact counts) decide
// which keys an item holds.
template <bool NT, bool MAP = false>
__global__ __launch_bounds__(kWave *kMerge4Waves) __attribute__((amdgpu_waves_per_eu(4))) void k_merge4(
    Merge4Src src)
{
    __shared__ __align__(16) uint32_t lds[kHalfLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t per = src.jfull + src.mfull;  // item slots of a full group
    const uint32_t g = __builtin_amdgcn_readfirstlane(blockIdx.x / per);
    const uint32_t i = __builtin_amdgcn_readfirstlane(blockIdx.x % per);
    if (g >= src.groups)
        return;
    Group4 G(src.n, src.run, g);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        G.n[r] = __builtin_amdgcn_readfirstlane(G.n[r]);
    G.J = __builtin_amdgcn_readfirstlane(G.J);
    G.M = __builtin_amdgcn_readfirstlane(G.M);
    const uint4 *P = src.cuts + (uint64_t)g * src.stride();
    const uint4 *Q = P + src.jfull + 1;
    uint4 c0, c1;
    if (!item_cuts(P, Q, G, i, src.jfull, c0, c1))
        return;
    const uint32_t L = (uint32_t)src.run;
    merge4_item<NT, MAP>(G, c0, c1, src.ksrc + G.start, L, 2 * L, 3 * L, src.kdst, src.out_smp, src.out_map, lds,
                         lane);
}

// ---------------------------------------------- fan-in 4 passes, key/value
//
// The same pass for stable key/value sorts.  Cuts and items are those of the
// keys-only pass (the cuts count exact stable positions: equal keys of A and
// B before those of C and D, and the binary splits keep A before B, C before
// D), and an item's tile holds (key, rank) elements in the keys' places.  The
// rank is the element's place in the item's input taken run after run (A,
// then B, C, D), so ties leave in run order and the rank names the element's
// source.  After the networks (on 64-bit elements, each transpose one 32-bit
// half at a time) the tile is back in STRIDED layout, where neighbouring
// lanes hold neighbouring outputs; every output fetches its value from the
// input by its rank (reads spread over at most four runs), and keys and
// values are stored.  The tile takes 128 registers, the kernel 230: two
// waves per SIMD.

// Rank layout of an item's pieces: piece q holds ranks [s[q], s[q + 1]) and
// starts o[q] keys after the group's first key (s[4] = 4096: no rank reaches
// it).
struct ItemRanks {
    uint32_t s[4], o[4];
};

__device__ __forceinline__ uint32_t rank_offset(const ItemRanks &ir, uint32_t rank)
{
    return rank < ir.s[1] ? ir.o[0] + rank
                          : rank < ir.s[2] ? ir.o[1] + (rank - ir.s[1])
                                           : rank < ir.s[3] ? ir.o[2] + (rank - ir.s[2]) : ir.o[3] + (rank - ir.s[3]);
}

// Load an item's tile as (key, rank) elements in STRIDED layout, keys placed
// as load_item places them; the front piece of half h has ranks from rf[h],
// the back piece (read backwards) from rb[h].  All 64 loads are issued before
// any is used; the upper half is complemented when hp.xm is set.  (Values
// are fetched after the networks, by rank: staging them in LDS beside the
// keys measured slower, 1.86 against 1.71 ms per pass of 2^28 pairs.)
__device__ __forceinline__ void load_item_pairs(Lines<true> &t, const uint32_t *K, const HalfPieces &hp,
                                                const uint32_t (&rf)[2], const uint32_t (&rb)[2], uint32_t lane)
{
    typedef __attribute__((address_space(1))) const uint32_t gkey;
    const uint32_t ln = opaque(lane);
    gkey *kg = (gkey *)K, *pad = (gkey *)kPadKeys + ln;
    uint32_t key[kLine];
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const int h = r / (kLine / 2);
        const uint32_t q = kWave * (r % (kLine / 2)) + ln;
        const bool in_f = q < hp.fn[h], in_b = q >= kHalfTile - hp.bn[h];
        const uint32_t off = in_f ? hp.front[h] + q : hp.bend[h] - q;
        key[r] = *((in_f || in_b) ? kg + off : pad);
        __builtin_amdgcn_sched_barrier(0);
    }
    const uint64_t cm = hp.xm ? kPayloadMask : 0ull;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const int h = r / (kLine / 2);
        const uint32_t q = kWave * (r % (kLine / 2)) + ln;
        const bool in_f = q < hp.fn[h], in_b = q >= kHalfTile - hp.bn[h];
        const uint32_t rank = in_f ? rf[h] + q : (in_b ? rb[h] + (kHalfTile - 1 - q) : kPadRank);
        const double e = make_elem(key[r], rank);
        t.e[r] = h ? elem_of(bits_of(e) ^ cm) : e;
    }
}

// Lane k receives register k of lane `src` (a wave-uniform lane).
__device__ __forceinline__ uint32_t column_of_lane(const uint32_t (&x)[kLine], uint32_t src, uint32_t lane)
{
    uint32_t v = 0;
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t s = __builtin_amdgcn_readlane(x[r], src);
        v = lane == (uint32_t)r ? s : v;
    }
    return v;
}

template <bool NT, bool MAP>
__device__ __forceinline__ void merge4_item_pairs(const Group4 &G, const uint4 &c0, const uint4 &c1, const uint32_t *K,
                                                  const uint32_t *V, uint32_t ob0, uint32_t oc0, uint32_t od0,
                                                  uint32_t *kdst, uint32_t *vdst, const SampleSet &out_smp,
                                                  const KeyMap &km, uint32_t *lds, uint32_t lane)
{
    const uint32_t pa = c1.x - c0.x, pb = c1.y - c0.y, pc = c1.z - c0.z, pd = c1.w - c0.w;
    const uint32_t sx = pa + pb, sy = pc + pd, count = sx + sy;
    if (count == 0 || sx > kHalfTile || sy > kHalfTile)
        return;
    const uint64_t gpos = G.start + c0.x + c0.y + c0.z + c0.w;
    const uint32_t pieces = (pa != 0) + (pb != 0) + (pc != 0) + (pd != 0);
    const uint32_t oa = c0.x, ob = ob0 + c0.y, oc = oc0 + c0.z, od = od0 + c0.w;
    if (pieces == 1) {
        const uint32_t o = pa ? oa : pb ? ob : pc ? oc : od;
        const SampleSet none{nullptr, nullptr, nullptr, nullptr};
        copy4<NT, MAP>(K + o, kdst, gpos, count, out_smp, km, lane);
        copy4<NT, false>(V + o, vdst, gpos, count, none, KeyMap{}, lane);
        return;
    }
    // every item of two or more pieces takes the four-piece layout and both
    // networks (empty pieces are padding): one code path, which keeps the
    // kernel at 256 registers, two waves per SIMD (a separate two-piece path
    // without the first network spilled at that bound)
    const HalfPieces hp{{oa, oc}, {pa, pc}, {ob + kHalfTile - 1, od + kHalfTile - 1}, {pb, pd}, ~0u};
    const ItemRanks ir{{0, pa, pa + pb, pa + pb + pc}, {pa ? oa : ob, ob, oc, od}};
    const uint32_t rf[2] = {0, pa + pb}, rb[2] = {pa, pa + pb + pc};
    Lines<true> t;
    load_item_pairs(t, K, hp, rf, rb, lane);
    // both halves merged at once, back to STRIDED, the CD half complemented back
    half_clean<kLine / 4, -1, true>(t);
    to_blocked_half(t, lds, lane);
    half_clean<kLine / 2, -1, true>(t);
    to_strided_half(t, lds, lane);
#pragma unroll
    for (int r = kLine / 2; r < kLine; ++r)
        t.e[r] = elem_of(bits_of(t.e[r]) ^ kPayloadMask);
    half_clean<kLine / 2, -1, true>(t);
    to_blocked_half(t, lds, lane);
    half_clean<kLine / 2, -1, true>(t);
    to_strided_half(t, lds, lane);
    // keys, and values fetched by rank (positions past the item read its first value)
    typedef __attribute__((address_space(1))) const uint32_t gval;
    gval *vg = (gval *)V;
    uint32_t kk[kLine], vv[kLine];
#pragma unroll
    for (int r = 0; r < kLine; ++r) {
        const uint32_t p = kWave * r + lane;
        kk[r] = elem_key(t.e[r]);
        const uint32_t off = p < count ? rank_offset(ir, elem_rank(t.e[r])) : ir.o[0];
        vv[r] = vg[off];
    }
    if (out_smp.f != nullptr) {
        // the first and last key of every 64-key block of the array inside the
        // item: positions bf + 64k and bl + 64k, register k of lanes bf and bl
        const uint32_t bf = (uint32_t)((kLine - gpos % kLine) % kLine);
        const uint32_t bl = (bf + kLine - 1) % kLine;
        const uint32_t f = column_of_lane(kk, bf, lane), l = column_of_lane(kk, bl, lane);
        const uint32_t pf = bf + kLine * lane, pl = bl + kLine * lane;
        if (pf < count) {
            const uint64_t gp = gpos + pf;
            out_smp.f[gp / kLine] = f;
            if (out_smp.cf != nullptr && gp % kTile == 0)
                out_smp.cf[gp / kTile] = f;
        }
        if (pl < count) {
            const uint64_t gp = gpos + pl;
            out_smp.l[gp / kLine] = l;
            if (out_smp.cf != nullptr && gp % kTile == kTile - 1)
                out_smp.cl[gp / kTile] = l;
        }
    }
    if constexpr (MAP) {
#pragma unroll
        for (int r = 0; r < kLine; ++r)
            kk[r] = map_key(kk[r], km.sign, km.rest, km.inverse);
    }
    const uint32_t ln = opaque(lane);
    store_bounded<NT>(kk, kdst + gpos, count, ln);
    store_bounded<NT>(vv, vdst + gpos, count, ln);
}

// One wave per merge item, as k_merge4.
template <bool NT, bool MAP = false>
__global__ __launch_bounds__(kWave *kMerge4Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_merge4_pairs(
    Merge4Src src)
{
    __shared__ __align__(16) uint32_t lds[kHalfLdsWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t per = src.jfull + src.mfull;
    const uint32_t g = __builtin_amdgcn_readfirstlane(blockIdx.x / per);
    const uint32_t i = __builtin_amdgcn_readfirstlane(blockIdx.x % per);
    if (g >= src.groups)
        return;
    Group4 G(src.n, src.run, g);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        G.n[r] = __builtin_amdgcn_readfirstlane(G.n[r]);
    G.J = __builtin_amdgcn_readfirstlane(G.J);
    G.M = __builtin_amdgcn_readfirstlane(G.M);
    const uint4 *P = src.cuts + (uint64_t)g * src.stride();
    const uint4 *Q = P + src.jfull + 1;
    uint4 c0, c1;
    if (!item_cuts(P, Q, G, i, src.jfull, c0, c1))
        return;
    const uint32_t L = (uint32_t)src.run;
    merge4_item_pairs<NT, MAP>(G, c0, c1, src.ksrc + G.start, src.vsrc + G.start, L, 2 * L, 3 * L, src.kdst,
                               src.vdst, src.out_smp, src.out_map, lds, lane);
}

// ------------------------------------------ fan-in 4 passes over job tables
//
// The same two launches for the merges of a table-driven pass (the segmented
// sort's segments, each with its own runs): a job is one group of four runs
// anywhere in one of the three buffers, with its own cut records, item slots
// and cut searches (task_job / item_job map a search or an item slot to its
// job).  Runs start at any position, so no samples exist: the cut searches
// read the keys themselves (32-ary rounds for the binary split, 16-ary for
// the counts).

struct Merge4Table {
    Bufs kb;
    const Merge4Job *jobs;
    uint32_t *task_job, *item_job;
    uint32_t njobs, tasks, items;  // bounds when counts is set
    uint4 *cuts;
    const uint32_t *counts;        // device words (jobs, searches, item slots), or nullptr
    Bufs vb;                       // key/value jobs: the values' buffers (vb.in == nullptr for keys)
    // the counts of a plan made on the device, never past the bounds the grid covers
    __device__ void resolve()
    {
        if (counts != nullptr) {
            njobs = min(njobs, counts[0]);
            tasks = min(tasks, counts[1]);
            items = min(items, counts[2]);
        }
    }
};

__device__ __forceinline__ const uint32_t *buf_in(const Bufs &b, uint32_t sel)
{
    return sel == kBufIn ? b.in : (sel == kBufOut ? b.out : b.temp);
}
__device__ __forceinline__ uint32_t *buf_out(const Bufs &b, uint32_t sel) { return sel == kBufOut ? b.out : b.temp; }

__device__ __forceinline__ Group4 group_of_job(const Merge4Job &j)
{
    Group4 G;
    G.start = j.start;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        G.n[r] = j.n[r];
    G.J = ab_segments((uint64_t)j.n[0] + j.n[1]);
    G.M = cd_cuts((uint64_t)j.n[2] + j.n[3]);
    return G;
}

// The maps of a table pass: search t and item slot i to the job whose range
// (task_off, item_off; ascending, every job has at least one of each) holds
// them, by binary search over the job list.
__global__ __launch_bounds__(256) void k_map4_table(Merge4Table src)
{
    src.resolve();
    const uint32_t njobs = src.njobs;
    auto owner = [&](uint32_t x, bool items) {
        uint32_t lo = 0, hi = njobs;  // the job's first index <= x, in [lo, hi)
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if ((items ? src.jobs[mid].item_off : src.jobs[mid].task_off) <= x)
                lo = mid;
            else
                hi = mid;
        }
        return lo;
    };
    const uint32_t most = src.items > src.tasks ? src.items : src.tasks;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < most; i += gridDim.x * 256) {
        if (i < src.items)
            src.item_job[i] = owner(i, true);
        if (i < src.tasks)
            src.task_job[i] = owner(i, false);
    }
}

// Searches of a table pass read the keys themselves (no samples), so every
// deep round fetches its own lines: four lanes per search (4-ary rounds on the
// cut's side, binary counts in each run of the other) fetch fewer lines per
// round and keep sixteen searches in flight per wave.  Measured over the
// table passes of a 1.01e9-key segmented sort: 16 lanes 1.21 ms, 8 lanes
// 0.94-0.97 ms, 4 lanes 0.86 ms.
constexpr int kTableCutLanesLog = 2;
constexpr uint32_t kTableCutLanes = 1u << kTableCutLanesLog;
constexpr uint32_t kTableCutsPerWave = kWave / kTableCutLanes;

// Cut searches of a table pass, kTableCutsPerWave per wave: task t
// of its job is AB cut t + 1 (t < J - 1) or CD cut t + 2 - J; the job's task
// 0 also writes its records P[0] and P[J] (a job with no cut to search has
// one task for that alone).
__device__ __forceinline__ void cut4_table_task(const Merge4Table &src, uint32_t task, uint32_t lane, uint32_t part)
{
    const bool in_range = task < src.tasks;
    const Merge4Job jb = src.jobs[src.task_job[in_range ? task : 0]];
    const Group4 G = group_of_job(jb);
    const uint32_t t = in_range ? task - jb.task_off : 0;
    const bool ab = t + 1 < G.J;
    const uint32_t idx = ab ? t + 1 : t + 2 - G.J;  // AB cut j or CD cut m
    const bool valid = in_range && (ab ? idx < G.J : (idx >= 1 && idx <= G.M));
    if (in_range && t == 0 && (lane & (kTableCutLanes - 1)) == 0) {
        uint4 *P = src.cuts + jb.cut_off;
        P[0] = make_uint4(0, 0, 0, 0);
        P[G.J] = make_uint4(G.n[0], G.n[1], G.n[2], G.n[3]);
    }
    if (__ballot(valid) == 0)
        return;
    const uint32_t *K = buf_in(src.kb, jb.src) + jb.start;
    const uint32_t n0 = ab ? G.n[0] : G.n[2], n1 = ab ? G.n[1] : G.n[3];
    const uint32_t *A = K + (ab ? 0u : G.n[0] + G.n[1]), *B = A + n0;
    const uint32_t d = ab ? idx * kAbStep : idx * kCdStep;
    uint32_t lo = d > n1 ? d - n1 : 0, hi = d < n0 ? d : n0;
    if (!valid)
        lo = hi = 0;
    search_level<1, kTableCutLanesLog>(lo, hi, lane, [&](uint32_t i) { return A[i] > B[d - 1 - i]; });
    const uint32_t s0 = lo, s1 = d - s0;
    uint32_t k = 0;
    if (valid)
        k = (s0 < n0 && (s1 >= n1 || A[s0] <= B[s1])) ? A[s0] : B[s1];
    // the other side: the upper half of a search's lanes counts in its second
    // run.  An AB cut counts keys below k, a CD cut keys at most k.
    const uint32_t second = (lane / (kTableCutLanes / 2)) & 1;
    const uint32_t nr = !valid ? 0 : (ab ? (second ? G.n[3] : G.n[2]) : (second ? G.n[1] : G.n[0]));
    const uint32_t ro = ab ? G.n[0] + G.n[1] + (second ? G.n[2] : 0) : (second ? G.n[0] : 0);
    const uint32_t *R = K + ro;
    const bool strict = !ab;
    uint32_t rlo = 0, rhi = nr;
    search_level<1, kTableCutLanesLog - 1>(rlo, rhi, lane, [&](uint32_t i) { return strict ? R[i] > k : R[i] >= k; });
    const uint32_t first = lane & ~(kTableCutLanes - 1);
    const uint32_t o0 = __shfl(rlo, first), o1 = __shfl(rlo, first + kTableCutLanes / 2);
    if (!valid || (lane & (kTableCutLanes - 1)) != 0)
        return;
    uint4 *P = src.cuts + jb.cut_off;
    if (ab)
        P[idx] = make_uint4(s0, s1, o0, o1);
    else
        P[G.J + 1 + idx] = make_uint4(o0, o1, s0, s1);
}

__global__ __launch_bounds__(256) void k_cuts4_table(Merge4Table src)
{
    src.resolve();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t part = lane / kTableCutLanes;
    const uint32_t waves = gridDim.x * (256 / kWave);
    for (uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (256 / kWave) + threadIdx.x / kWave);
         kTableCutsPerWave * wave < src.tasks; wave += waves)
        cut4_table_task(src, kTableCutsPerWave * wave + part, lane, part);
}

// One item slot of a table pass.
template <bool NT>
__device__ __forceinline__ void merge4_table_item(const Merge4Table &src, uint32_t item, uint32_t *lds,
                                                  uint32_t lane)
{
    const uint32_t jid = __builtin_amdgcn_readfirstlane(src.item_job[item]);
    const Merge4Job &jr = src.jobs[jid];
    Merge4Job jb;
    jb.start = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(jr.start >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)jr.start);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        jb.n[r] = __builtin_amdgcn_readfirstlane(jr.n[r]);
    jb.cut_off = __builtin_amdgcn_readfirstlane(jr.cut_off);
    jb.item_off = __builtin_amdgcn_readfirstlane(jr.item_off);
    const uint32_t sel = __builtin_amdgcn_readfirstlane(((uint32_t)jr.dst << 16) | jr.src);
    const Group4 G = group_of_job(jb);
    const uint4 *P = src.cuts + jb.cut_off;
    const uint4 *Q = P + G.J + 1;
    uint4 c0, c1;
    if (!item_cuts(P, Q, G, item - jb.item_off, G.J, c0, c1))
        return;
    const uint32_t n01 = G.n[0] + G.n[1];
    const SampleSet none{nullptr, nullptr, nullptr, nullptr};
    merge4_item<NT, false>(G, c0, c1, buf_in(src.kb, sel & 0xffff) + G.start, G.n[0], n01, n01 + G.n[2],
                           buf_out(src.kb, sel >> 16), none, KeyMap{}, lds, lane);
}

// One item slot of a key/value table pass (values in src.vb, laid out like
// the keys).
template <bool NT>
__device__ __forceinline__ void merge4_table_item_pairs(const Merge4Table &src, uint32_t item, uint32_t *lds,
                                                        uint32_t lane)
{
    const uint32_t jid = __builtin_amdgcn_readfirstlane(src.item_job[item]);
    const Merge4Job &jr = src.jobs[jid];
    Merge4Job jb;
    jb.start = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(jr.start >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)jr.start);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        jb.n[r] = __builtin_amdgcn_readfirstlane(jr.n[r]);
    jb.cut_off = __builtin_amdgcn_readfirstlane(jr.cut_off);
    jb.item_off = __builtin_amdgcn_readfirstlane(jr.item_off);
    const uint32_t sel = __builtin_amdgcn_readfirstlane(((uint32_t)jr.dst << 16) | jr.src);
    const Group4 G = group_of_job(jb);
    const uint4 *P = src.cuts + jb.cut_off;
    const uint4 *Q = P + G.J + 1;
    uint4 c0, c1;
    if (!item_cuts(P, Q, G, item - jb.item_off, G.J, c0, c1))
        return;
    const uint32_t n01 = G.n[0] + G.n[1];
    const SampleSet none{nullptr, nullptr, nullptr, nullptr};
    merge4_item_pairs<NT, false>(G, c0, c1, buf_in(src.kb, sel & 0xffff) + G.start,
                                 buf_in(src.vb, sel & 0xffff) + G.start, G.n[0], n01, n01 + G.n[2],
                                 buf_out(src.kb, sel >> 16), buf_out(src.vb, sel >> 16), none, KeyMap{}, lds, lane);
}

// Merges of a table pass: one wave per item slot, the grid striding over the
// slots when it is smaller (plans made on the device size it by the chip).
template <bool NT>
__global__ __launch_bounds__(kWave *kMerge4Waves) __attribute__((amdgpu_waves_per_eu(4))) void k_merge4_table(
    Merge4Table src)
{
    __shared__ __align__(16) uint32_t lds[kHalfLdsWords];
    src.resolve();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t item = blockIdx.x; item < src.items; item += gridDim.x) {
        // the lane index re-derived per item keeps the compiler from hoisting
        // the per-register addresses out of the loop (registers held across it)
        merge4_table_item<NT>(src, item, lds, opaque(lane));
        wave_lds_fence();  // the next item writes the LDS this one read
    }
}

// The same for key/value table passes (two waves per SIMD, as k_merge4_pairs).
template <bool NT>
__global__ __launch_bounds__(kWave *kMerge4Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_merge4_table_pairs(
    Merge4Table src)
{
    __shared__ __align__(16) uint32_t lds[kHalfLdsWords];
    src.resolve();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t item = blockIdx.x; item < src.items; item += gridDim.x) {
        merge4_table_item_pairs<NT>(src, item, lds, opaque(lane));
        wave_lds_fence();  // the next item writes the LDS this one read
    }
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

// Work-groups of a persistent launch: enough to fill every CU at the
// kernel's occupancy, never more than the tiles need.
template <class K>
static uint32_t persistent_groups(K kernel, uint64_t tiles)
{
    static int resident = 0;  // per kernel instantiation
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave * kWavesPerGroup, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 1, cus = 256;
        resident = cus * per_cu;
    }
    const uint64_t need = (tiles + kWavesPerGroup - 1) / kWavesPerGroup;
    return (uint32_t)(need < (uint64_t)resident ? need : (uint64_t)resident);
}

template <bool P, class Src>
static hipError_t launch_sort(const Src &src, hipStream_t s, bool shear = false)
{
    if (src.ntiles == 0)
        return hipSuccess;
    if (shear) {
        const dim3 grid(persistent_groups(k_block_sort<P, Src, true>, src.ntiles)), block(kWave * kWavesPerGroup);
        hipLaunchKernelGGL((k_block_sort<P, Src, true>), grid, block, 0, s, src);
    } else {
        const dim3 grid(persistent_groups(k_block_sort<P, Src>, src.ntiles)), block(kWave * kWavesPerGroup);
        hipLaunchKernelGGL((k_block_sort<P, Src>), grid, block, 0, s, src);
    }
    return hipGetLastError();
}

template <class Src>
static hipError_t launch_partition(const Src &src, uint32_t *splits, hipStream_t s)
{
    if (src.ntiles == 0)
        return hipSuccess;
    const uint32_t pgroups = (src.ntiles + 2 * (256 / kWave) - 1) / (2 * (256 / kWave));
    hipLaunchKernelGGL((k_partition<Src>), dim3(pgroups), dim3(256), 0, s, src, splits);
    return hipGetLastError();
}

template <bool P, class Src, int MODE, bool NT = false, bool FUSED = false>
static hipError_t launch_merge_mode(const Src &src, const uint32_t *splits, hipStream_t s)
{
    constexpr int W = merge_group_waves<MODE>();
    const uint32_t groups = MODE == 2 ? (src.ntiles + W - 1) / W
                                      : persistent_groups(k_merge<P, Src, MODE, NT, FUSED>, src.ntiles);
    hipLaunchKernelGGL((k_merge<P, Src, MODE, NT, FUSED>), dim3(groups), dim3(kWave * W), 0, s, src, splits);
    return hipGetLastError();
}

template <bool P, class Src>
static hipError_t launch_merge(const Src &src, const uint32_t *splits, hipStream_t s)
{
    if (src.ntiles == 0)
        return hipSuccess;
    const Tuning tu = tuning();
    // variant 3: one tile per wave for keys (the lighter kernel fits three
    // waves' registers per SIMD), persistent waves for pairs
    const int variant = tu.merge_variant == 3 ? (P ? 1 : 2) : tu.merge_variant;
    switch (variant) {
    case 0: return P ? launch_merge_mode<P, Src, 1>(src, splits, s) : launch_merge_mode<P, Src, 0>(src, splits, s);
    case 2: return launch_merge_mode<P, Src, 2>(src, splits, s);
    default:
        return tu.nontemporal ? launch_merge_mode<P, Src, 1, true>(src, splits, s)
                              : launch_merge_mode<P, Src, 1>(src, splits, s);
    }
}

// MI355X's last-level cache (Infinity Cache): 256 MiB.
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

bool merge_fuses_partition(bool pairs, const SampleSet &in_smp, const Tuning &tu)
{
    return in_smp.f != nullptr && tu.fused_partition && (tu.merge_variant == 2 || (tu.merge_variant == 3 && !pairs));
}

hipError_t launch_block_sort_regular(bool pairs, bool shear, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                     uint32_t *vout, uint64_t n, SampleSet out_smp, hipStream_t s, KeyMap in_map,
                                     KeyMap out_map)
{
    RegularSortSrc src{kin, pairs ? vin : nullptr, kout, pairs ? vout : nullptr, n,
                       (uint32_t)((n + kTile - 1) / kTile), out_smp};
    if (in_map.sign || out_map.sign) {  // other key types: merge rounds only
        const Mapped<RegularSortSrc> ms{src, in_map, out_map};
        return pairs ? launch_sort<true>(ms, s) : launch_sort<false>(ms, s);
    }
    return pairs ? launch_sort<true>(src, s, shear) : launch_sort<false>(src, s, shear);
}

static uint32_t cu_count()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus = c;
    }
    return (uint32_t)cus;
}

template <int NW, bool P, class Src>
static hipError_t launch_group_src(const Src &src, hipStream_t s)
{
    if (src.ngroups == 0)
        return hipSuccess;
    // one group per CU fits the LDS (NW * 16.6 KiB); persistent over the groups
    const uint32_t groups = src.ngroups < cu_count() ? src.ngroups : cu_count();
    hipLaunchKernelGGL((k_block_sort_group<NW, P, Src>), dim3(groups), dim3(kWave * NW), 0, s, src);
    return hipGetLastError();
}

template <int NW, bool P>
static hipError_t launch_group(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                               uint64_t n, SampleSet smp, hipStream_t s, KeyMap in_map, KeyMap out_map)
{
    constexpr uint32_t keys = NW * kTile;
    RegularGroupSrc src{kin, P ? vin : nullptr, kout, P ? vout : nullptr, n, (uint32_t)((n + keys - 1) / keys), keys,
                        smp};
    if (in_map.sign || out_map.sign)
        return launch_group_src<NW, P>(Mapped<RegularGroupSrc>{src, in_map, out_map}, s);
    return launch_group_src<NW, P>(src, s);
}

hipError_t launch_block_sort_group_table(bool pairs, Bufs kb, Bufs vb, const BlockTile *tiles, uint32_t ngroups,
                                         hipStream_t s, const uint32_t *count_dev)
{
    if (!pairs)
        vb = Bufs{nullptr, nullptr, nullptr};
    TableGroupSrc src{kb, vb, tiles, ngroups, SampleSet{nullptr, nullptr, nullptr, nullptr}, count_dev};
    return pairs ? launch_group_src<kGroupWavesPairs, true>(src, s) : launch_group_src<kGroupWavesKeys, false>(src, s);
}

uint32_t group_run_keys(bool pairs) { return pairs ? kGroupWavesPairs * kTile : kGroupWavesKeys * kTile; }

hipError_t launch_block_sort_shear_group(const uint32_t *kin, uint32_t *kout, uint64_t n, SampleSet out_smp,
                                         hipStream_t s)
{
    constexpr uint32_t keys = kGroupWavesKeys * kTile;
    RegularGroupSrc src{kin, nullptr, kout, nullptr, n, (uint32_t)((n + keys - 1) / keys), keys, out_smp};
    if (src.ngroups == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_block_sort_shear_group<kGroupWavesKeys, RegularGroupSrc>), dim3(src.ngroups),
                       dim3(kWave * kGroupWavesKeys), 0, s, src);
    return hipGetLastError();
}

hipError_t launch_block_sort_group(bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                   uint32_t *vout, uint64_t n, SampleSet out_smp, hipStream_t s, KeyMap in_map,
                                   KeyMap out_map)
{
    return pairs ? launch_group<kGroupWavesPairs, true>(kin, vin, kout, vout, n, out_smp, s, in_map, out_map)
                 : launch_group<kGroupWavesKeys, false>(kin, vin, kout, vout, n, out_smp, s, in_map, out_map);
}

hipError_t launch_merge_regular(bool pairs, const uint32_t *ksrc, const uint32_t *vsrc, uint32_t *kdst,
                                uint32_t *vdst, uint64_t n, uint64_t run, uint32_t *splits, SampleSet in_smp,
                                SampleSet out_smp, bool partition, bool fused, hipStream_t s, KeyMap out_map)
{
    RegularMergeSrc src{ksrc, pairs ? vsrc : nullptr, kdst, pairs ? vdst : nullptr, n, run,
                        (uint32_t)((n + kTile - 1) / kTile), in_smp, out_smp};
    if (out_map.sign && !(partition && !fused)) {
        // the pass that writes the output of another key type: one tile per
        // wave, its split searched by the merge itself (fused) or read from
        // the partition launch before it
        if (fused && (run % kTile != 0 || in_smp.f == nullptr))
            return hipErrorInvalidValue;
        if (partition)
            return hipSuccess;
        const Mapped<RegularMergeSrc> ms{src, KeyMap{}, out_map};
        const bool nt = tuning().nontemporal && n * (pairs ? 8.0 : 4.0) * 2 > kLastLevelCacheBytes;
        using M = Mapped<RegularMergeSrc>;
        if (fused)
            return pairs ? (nt ? launch_merge_mode<true, M, 2, true, true>(ms, splits, s)
                               : launch_merge_mode<true, M, 2, false, true>(ms, splits, s))
                         : (nt ? launch_merge_mode<false, M, 2, true, true>(ms, splits, s)
                               : launch_merge_mode<false, M, 2, false, true>(ms, splits, s));
        return pairs ? (nt ? launch_merge_mode<true, M, 2, true>(ms, splits, s)
                           : launch_merge_mode<true, M, 2, false>(ms, splits, s))
                     : (nt ? launch_merge_mode<false, M, 2, true>(ms, splits, s)
                           : launch_merge_mode<false, M, 2, false>(ms, splits, s));
    }
    if (fused) {
        // one launch per pass: the merge kernel searches its own splits
        if (partition)
            return hipSuccess;
        if (run % kTile != 0 || in_smp.f == nullptr)
            return hipErrorInvalidValue;
        // nontemporal tile traffic only when a pass streams more than the
        // last-level cache holds (below that the hint makes the next pass miss)
        if (tuning().nontemporal && n * (pairs ? 8.0 : 4.0) * 2 > kLastLevelCacheBytes)
            return pairs ? launch_merge_mode<true, RegularMergeSrc, 2, true, true>(src, splits, s)
                         : launch_merge_mode<false, RegularMergeSrc, 2, true, true>(src, splits, s);
        return pairs ? launch_merge_mode<true, RegularMergeSrc, 2, false, true>(src, splits, s)
                     : launch_merge_mode<false, RegularMergeSrc, 2, false, true>(src, splits, s);
    }
    if (partition) {
        if (in_smp.f == nullptr)
            return launch_partition(src, splits, s);
        // runs must start at multiples of 4096 for the sample predicates
        if (run % kTile != 0)
            return hipErrorInvalidValue;
        if (tuning().partition_half) {
            const uint32_t groups = (src.ntiles + 2 * (256 / kWave) - 1) / (2 * (256 / kWave));
            hipLaunchKernelGGL(k_partition_sampled<true>, dim3(groups), dim3(256), 0, s, src, splits);
        } else {
            const uint32_t groups = (src.ntiles + (256 / kWave) - 1) / (256 / kWave);
            hipLaunchKernelGGL(k_partition_sampled<false>, dim3(groups), dim3(256), 0, s, src, splits);
        }
        return hipGetLastError();
    }
    return pairs ? launch_merge<true>(src, splits, s) : launch_merge<false>(src, splits, s);
}

uint64_t merge4_cut_bytes(uint64_t n, uint64_t run)
{
    if (run == 0 || run % kTile != 0)
        return 0;
    const uint64_t groups = (n + 4 * run - 1) / (4 * run);
    return groups * ((uint64_t)ab_segments(2 * run) + cd_cuts(2 * run) + 2) * sizeof(uint4);
}

uint64_t merge4_cut_bytes_max(uint64_t n)
{
    // four-way passes run while more than two runs remain (n > 2 run), on
    // runs of 4096 * 4^i keys, or of a keys or pairs group tile times 4^i
    uint64_t most = 0;
    for (uint64_t run0 : {(uint64_t)kTile, (uint64_t)kGroupWavesKeys * kTile, (uint64_t)kGroupWavesPairs * kTile})
        for (uint64_t run = run0; n > 2 * run; run *= 4)
            most = std::max(most, merge4_cut_bytes(n, run));
    return most;
}

hipError_t launch_merge4_regular(const uint32_t *ksrc, uint32_t *kdst, uint64_t n, uint64_t run, void *cuts,
                                 SampleSet in_smp, SampleSet out_smp, bool cut_phase, hipStream_t s, KeyMap out_map,
                                 const uint32_t *vsrc, uint32_t *vdst)
{
    // the cut searches read the samples of the input; runs start at multiples of 4096
    if (n == 0 || run % kTile != 0 || in_smp.f == nullptr || in_smp.l == nullptr || cuts == nullptr)
        return hipErrorInvalidValue;
    const uint64_t groups = (n + 4 * run - 1) / (4 * run);
    const bool pairs = vsrc != nullptr;
    if (pairs != (vdst != nullptr))
        return hipErrorInvalidValue;
    Merge4Src src{ksrc, kdst, n, run, (uint32_t)groups, ab_segments(2 * run), cd_cuts(2 * run),
                  static_cast<uint4 *>(cuts), in_smp, out_smp, out_map, vsrc, vdst};
    if (cut_phase) {
        const uint64_t tasks = groups * (src.jfull - 1 + src.mfull);  // kCutsPerWave per wave, four waves per block
        const uint64_t per_block = kCutsPerWave * (256 / kWave);
        hipLaunchKernelGGL(k_cuts4, dim3((uint32_t)((tasks + per_block - 1) / per_block)), dim3(256), 0, s, src);
        return hipGetLastError();
    }
    const uint64_t items = groups * (src.jfull + src.mfull);
    const dim3 grid((uint32_t)((items + kMerge4Waves - 1) / kMerge4Waves)), block(kWave * kMerge4Waves);
    // nontemporal tile traffic only when a pass streams more than the last-level cache
    const bool nt = tuning().nontemporal && n * (pairs ? 8.0 : 4.0) * 2 > kLastLevelCacheBytes;
    if (pairs) {
        if (out_map.sign && nt)
            hipLaunchKernelGGL((k_merge4_pairs<true, true>), grid, block, 0, s, src);
        else if (out_map.sign)
            hipLaunchKernelGGL((k_merge4_pairs<false, true>), grid, block, 0, s, src);
        else if (nt)
            hipLaunchKernelGGL((k_merge4_pairs<true, false>), grid, block, 0, s, src);
        else
            hipLaunchKernelGGL((k_merge4_pairs<false, false>), grid, block, 0, s, src);
        return hipGetLastError();
    }
    if (out_map.sign && nt)
        hipLaunchKernelGGL((k_merge4<true, true>), grid, block, 0, s, src);
    else if (out_map.sign)
        hipLaunchKernelGGL((k_merge4<false, true>), grid, block, 0, s, src);
    else if (nt)
        hipLaunchKernelGGL((k_merge4<true, false>), grid, block, 0, s, src);
    else
        hipLaunchKernelGGL((k_merge4<false, false>), grid, block, 0, s, src);
    return hipGetLastError();
}

// Work-groups of a launch whose count is known only on the device: enough to
// fill every CU at the kernel's occupancy, never more than the bound needs.
template <class K>
static uint32_t resident_blocks(K kernel, int threads, uint64_t need)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1, cus = 256;
    const uint64_t most = (uint64_t)cus * per_cu;
    return (uint32_t)(need < most ? need : most);
}

hipError_t launch_merge4_table(Bufs kb, const Merge4Job *jobs, uint32_t njobs, uint32_t *task_job, uint32_t tasks,
                               uint32_t *item_job, uint32_t items, void *cuts, uint64_t keys, int phase, hipStream_t s,
                               const uint32_t *counts_dev, Bufs vb)
{
    Merge4Table src{kb, jobs, task_job, item_job, njobs, tasks, items, static_cast<uint4 *>(cuts), counts_dev, vb};
    const bool pairs = vb.in != nullptr;
    if (njobs == 0)
        return hipSuccess;
    const bool dev_counts = counts_dev != nullptr;
    if (phase == 0) {
        const uint32_t most = tasks > items ? tasks : items;
        const uint64_t need = (most + 255) / 256;
        const uint32_t grid = dev_counts ? resident_blocks(k_map4_table, 256, need) : (uint32_t)need;
        if (grid == 0)
            return hipSuccess;
        hipLaunchKernelGGL(k_map4_table, dim3(grid), dim3(256), 0, s, src);
        return hipGetLastError();
    }
    if (phase == 1) {
        if (tasks == 0)
            return hipSuccess;
        const uint32_t per_block = kTableCutsPerWave * (256 / kWave);
        const uint64_t need = (tasks + per_block - 1) / per_block;
        const uint32_t grid = dev_counts ? resident_blocks(k_cuts4_table, 256, need) : (uint32_t)need;
        hipLaunchKernelGGL(k_cuts4_table, dim3(grid), dim3(256), 0, s, src);
        return hipGetLastError();
    }
    if (items == 0)
        return hipSuccess;
    const bool nt = tuning().nontemporal && keys * (pairs ? 8.0 : 4.0) * 2 > kLastLevelCacheBytes;
    const dim3 block(kWave * kMerge4Waves);
    if (pairs) {
        if (nt) {
            const uint32_t grid =
                dev_counts ? resident_blocks(k_merge4_table_pairs<true>, kWave * kMerge4Waves, items) : items;
            hipLaunchKernelGGL(k_merge4_table_pairs<true>, dim3(grid), block, 0, s, src);
        } else {
            const uint32_t grid =
                dev_counts ? resident_blocks(k_merge4_table_pairs<false>, kWave * kMerge4Waves, items) : items;
            hipLaunchKernelGGL(k_merge4_table_pairs<false>, dim3(grid), block, 0, s, src);
        }
        return hipGetLastError();
    }
    if (nt) {
        const uint32_t grid = dev_counts ? resident_blocks(k_merge4_table<true>, kWave * kMerge4Waves, items) : items;
        hipLaunchKernelGGL(k_merge4_table<true>, dim3(grid), block, 0, s, src);
    } else {
        const uint32_t grid = dev_counts ? resident_blocks(k_merge4_table<false>, kWave * kMerge4Waves, items) : items;
        hipLaunchKernelGGL(k_merge4_table<false>, dim3(grid), block, 0, s, src);
    }
    return hipGetLastError();
}

hipError_t launch_block_sort_table(bool pairs, Bufs kb, Bufs vb, const BlockTile *tiles, uint32_t ntiles,
                                   hipStream_t s, const uint32_t *count_dev)
{
    if (!pairs)
        vb = Bufs{nullptr, nullptr, nullptr};
    TableSortSrc src{kb, vb, tiles, ntiles, SampleSet{nullptr, nullptr, nullptr, nullptr}, count_dev};
    return pairs ? launch_sort<true>(src, s) : launch_sort<false>(src, s);
}

hipError_t launch_merge_table(bool pairs, Bufs kb, Bufs vb, const MergeJob *jobs, const uint32_t *tile_job,
                              uint32_t ntiles, uint32_t *splits, bool partition, hipStream_t s,
                              const uint32_t *count_dev)
{
    if (!pairs)
        vb = Bufs{nullptr, nullptr, nullptr};
    TableMergeSrc src{kb, vb, jobs, tile_job, ntiles, SampleSet{nullptr, nullptr, nullptr, nullptr}, count_dev};
    if (count_dev != nullptr) {
        // the count is known only on the device: persistent waves (a grid the
        // size of the chip, not of the bound)
        if (ntiles == 0)
            return hipSuccess;
        if (partition) {
            const uint32_t pg = persistent_groups(k_partition_persist<TableMergeSrc>, ntiles);
            hipLaunchKernelGGL((k_partition_persist<TableMergeSrc>), dim3(pg), dim3(256), 0, s, src, splits);
            return hipGetLastError();
        }
        const bool nt = tuning().nontemporal;
        if (pairs)
            return nt ? launch_merge_mode<true, TableMergeSrc, 1, true>(src, splits, s)
                      : launch_merge_mode<true, TableMergeSrc, 1>(src, splits, s);
        return nt ? launch_merge_mode<false, TableMergeSrc, 1, true>(src, splits, s)
                  : launch_merge_mode<false, TableMergeSrc, 1>(src, splits, s);
    }
    if (partition)
        return launch_partition(src, splits, s);
    return pairs ? launch_merge<true>(src, splits, s) : launch_merge<false>(src, splits, s);
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

const char *kname_partition(bool pairs, bool table)
{
    return pairs ? (table ? "partition_pairs_table" : "partition_pairs")
                 : (table ? "partition_keys_table" : "partition_keys");
}

const char *kname_merge(bool pairs, bool table)
{
    return pairs ? (table ? "merge_pairs_table" : "merge_pairs") : (table ? "merge_keys_table" : "merge_keys");
}

}  // namespace bcf
