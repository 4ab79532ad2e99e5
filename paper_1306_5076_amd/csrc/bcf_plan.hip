// Device planning of table-driven sorts and merges whose run or segment
// offsets live in device memory: the block-sort tile list, and for every
// merge pass its job list and tile-to-job map, are computed by small kernels
// from the offsets, so that nothing is read back to the host and a captured
// graph stays valid when the offsets change between replays (as long as the
// total stays within the capacity the temp buffer was sized for).
//
// The merges are the paper's binary merging (Sec. 3.2) of groups of runs:
// group g's runs are merged pairwise, pass after pass, until one run remains;
// every group has its own pass count and buffer parity, so its last pass
// writes the output.  Three kinds of groups:
//   * merge_runs: one group of k explicit runs [off[r], off[r+1]);
//   * buckets (the final merge after a distribution, Sec. 3.2 and 3.3): group
//     b holds the s pieces [off[b s + r], off[b s + r + 1]) of bucket b; a
//     pivot bucket holds one key value, so its pieces are already merged and
//     the group is one copy;
//   * segments: segment g = [off[g], off[g+1]) is block-sorted into runs of
//     4096 keys (wave tiles) or of a group tile (long segments), then those
//     runs are merged.
// The tables are the same BlockTile / MergeJob / tile-to-job tables the host
// planner of bcf_api.hip builds, read by the same kernels, which take their
// tile counts from device words written here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "bcf.h"
#include "bcf_device.hpp"
#include "bcf_internal.hpp"

namespace bcf {

// Host services of bcf_api.hip: a profiling scope around one launch.
void *prof_begin(const char *name, hipStream_t s, double bytes);
void prof_end(void *scope);

namespace {

#define BCF_PLAN_TRY(x)                     \
    do {                                    \
        bcf_status st_ = (x);               \
        if (st_ != BCF_OK)                  \
            return st_;                     \
    } while (0)

constexpr int kMaxPlanPasses = 24;  // 4096 << 24 keys > 2^32
constexpr int kMaxPlan4Passes = 12; // fan-in 4 steps: 4096 << 24 keys > 2^32
constexpr uint32_t kPlanBlock = 256;
constexpr uint64_t kMaxKeys = 0xFFFFFFFFull;

uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint32_t clog2(uint64_t x)
{
    uint32_t p = 0;
    while ((uint64_t(1) << p) < x)
        ++p;
    return p;
}

__host__ __device__ inline uint32_t ceil_log2_u(uint64_t x)
{
    uint32_t p = 0;
    while ((uint64_t(1) << p) < x)
        ++p;
    return p;
}

enum GroupKind : uint32_t { kKindRuns = 0, kKindBuckets = 1, kKindSegments = 2 };

// One group as the planner sees it.  A segment (keys, fan-in 4 on) first
// takes `steps4` fan-in 4 steps while more than two runs remain, then its
// binary steps.
struct GroupInfo {
    uint32_t first;   // explicit runs: index of the group's first offset
    uint32_t nruns;   // runs before the merge passes
    uint32_t steps4;  // fan-in 4 steps (segments only)
    uint32_t merges;  // binary merge passes after them
    uint32_t passes;  // steps4 + merges, or merges + 1 with a final copy, or 1 copy
    uint32_t run0;    // segments: run length after the block sort (0: explicit runs)
    uint64_t start, end;
};

// Everything the planner kernels read: the offsets, the kind of groups, and
// where the tables go.
struct PlanArgs {
    const uint64_t *off;
    uint32_t kind;
    uint32_t G;          // groups
    uint32_t k;          // explicit runs: offsets k + 1
    uint32_t s;          // buckets: runs (pieces) per bucket
    uint32_t pivot;      // buckets: odd buckets are pivot buckets
    uint32_t extra_copy; // runs: one more pass copying temp into the output
    uint64_t gmin;       // segments: group tiles from this many keys (and more than 4096)
    uint32_t grun;       // segments: keys per group tile
    uint32_t PM;         // merge passes planned
    uint32_t four;       // segments: fan-in 4 steps 0 off, 1 on, 2 from kAutoFourWayMinN keys in all
    uint32_t PM4;        // passes with fan-in 4 tables (at most kMaxPlan4Passes)
    uint64_t cap;        // the most keys the temp buffer holds
    uint32_t *status;    // 0: plan valid; 1: offsets invalid or past the capacity
    // block-sort tiles (segments): counts per group, prefix, lists, totals
    uint32_t *bw, *bg;
    BlockTile *wtiles, *gtiles;
    uint32_t wb, gb;     // list bounds
    uint32_t *wcount, *gcount;
    // merge pass j (0-based): job counts per group (prefix), jobs, tiles per job (prefix), tile map, total
    uint32_t *gjob[kMaxPlanPasses];
    MergeJob *jobs[kMaxPlanPasses];
    uint32_t *jtile[kMaxPlanPasses];
    uint32_t *tjob[kMaxPlanPasses];
    uint32_t jb[kMaxPlanPasses], tb[kMaxPlanPasses];  // bounds
    uint32_t *tcount;    // [PM] tiles of each pass
    // fan-in 4 pass j: job counts per group (prefix), jobs, per-job searches /
    // item slots / cut records (prefix: the jobs' first indices), and the
    // pass's counts (jobs, searches, item slots); bounds
    uint32_t *gjob4[kMaxPlan4Passes];
    Merge4Job *jobs4[kMaxPlan4Passes];
    uint32_t *jt4[kMaxPlan4Passes], *ji4[kMaxPlan4Passes], *jr4[kMaxPlan4Passes];
    uint32_t *c4[kMaxPlan4Passes];
    uint32_t j4b[kMaxPlan4Passes];
    uint32_t t4b, i4b, r4b;
};
static_assert(sizeof(PlanArgs) <= 4096, "kernel arguments are limited to 4 KiB");

__device__ GroupInfo group_info(const PlanArgs &a, uint32_t g)
{
    GroupInfo gi;
    if (a.kind == kKindSegments) {
        gi.start = a.off[g];
        gi.end = a.off[g + 1];
        const uint64_t len = gi.end - gi.start;
        gi.run0 = (len > (uint64_t)kTile && len >= a.gmin) ? a.grun : (uint32_t)kTile;
        gi.nruns = (uint32_t)((len + gi.run0 - 1) / gi.run0);
        uint32_t r = gi.nruns;
        gi.steps4 = 0;
        const bool four = a.four == 1 || (a.four == 2 && a.off[a.G] >= kAutoFourWayMinN);
        while (four && r > 2 && gi.steps4 < a.PM4) {
            r = (r + 3) / 4;
            ++gi.steps4;
        }
        gi.merges = ceil_log2_u(r);
        gi.passes = gi.steps4 + gi.merges;
        gi.first = 0;
    } else {
        gi.run0 = 0;
        gi.steps4 = 0;
        if (a.kind == kKindRuns) {
            gi.first = 0;
            gi.nruns = a.k;
        } else {
            gi.first = g * a.s;
            gi.nruns = a.s;
        }
        const bool pivot = a.kind == kKindBuckets && a.pivot && (g & 1u);
        // explicit runs: fan-in 4 steps only when the host asked for them (it
        // plans the pass count, and the extra copy of an in-place merge, the same way)
        uint32_t r = gi.nruns;
        while (a.four == 1 && !pivot && r > 2 && gi.steps4 < a.PM4) {
            r = (r + 3) / 4;
            ++gi.steps4;
        }
        gi.merges = pivot ? 0 : ceil_log2_u(r);
        const uint32_t levels = gi.steps4 + gi.merges;
        if (a.kind == kKindRuns)
            gi.passes = levels + (a.extra_copy ? 1 : 0);
        else
            gi.passes = levels ? levels : 1;  // a group of one run (or a pivot bucket) is copied
        gi.start = a.off[gi.first];
        gi.end = a.off[gi.first + gi.nruns];
    }
    return gi;
}

// Offset of run boundary r (0 <= r <= nruns) of a group.
__device__ uint64_t run_bound(const PlanArgs &a, const GroupInfo &gi, uint32_t r)
{
    if (gi.run0) {
        const uint64_t p = gi.start + (uint64_t)r * gi.run0;
        return p < gi.end ? p : gi.end;
    }
    return a.off[gi.first + r];
}

// Runs (of run0 keys, segments) a binary step after the fan-in 4 steps
// merges per pair: 4^steps4 2^(b - 1) for binary step b (1-based).
__device__ uint64_t binary_unit(const GroupInfo &gi, uint32_t b) { return (1ull << (2 * gi.steps4)) << (b - 1); }

// Binary jobs of pass j (1-based).
__device__ uint32_t jobs_in(const GroupInfo &gi, uint32_t j)
{
    if (gi.end == gi.start || j > gi.passes || j <= gi.steps4)
        return 0;
    const uint32_t b = j - gi.steps4;
    if (b <= gi.merges) {
        const uint64_t span = 2 * binary_unit(gi, b);
        return (uint32_t)((gi.nruns + span - 1) / span);
    }
    return 1;  // the copy pass
}

// Fan-in 4 jobs of pass j (1-based): groups of four runs of 4^(j-1) run0 keys.
__device__ uint32_t jobs4_in(const GroupInfo &gi, uint32_t j)
{
    if (gi.end == gi.start || j > gi.steps4)
        return 0;
    const uint64_t span = 1ull << (2 * j);
    return (uint32_t)((gi.nruns + span - 1) / span);
}

// Buffer of group gi after its pass j (0: after the block sort, segments);
// its last pass writes the output.
__device__ uint16_t buf_after(const GroupInfo &gi, uint32_t j)
{
    return ((gi.passes - j) % 2 == 0) ? (uint16_t)kBufOut : (uint16_t)kBufTemp;
}

// The words the other planner kernels accumulate into or test start at zero:
// status, block-tile totals, pass totals.
__global__ void k_plan_zero(PlanArgs a)
{
    if (threadIdx.x == 0) {
        *a.status = 0;
        *a.wcount = 0;
        *a.gcount = 0;
    }
    for (uint32_t j = threadIdx.x; j < kMaxPlanPasses; j += blockDim.x)
        a.tcount[j] = 0;
}

// Validity of the offsets: off[0] == 0, nondecreasing, total within the
// capacity.  One thread per offset pair; any failure sets the status word.
__global__ __launch_bounds__(kPlanBlock) void k_plan_check(PlanArgs a, uint32_t noff)
{
    const uint32_t i = blockIdx.x * kPlanBlock + threadIdx.x;
    if (i == 0 && (a.off[0] != 0 || a.off[noff - 1] > a.cap))
        *a.status = 1;
    if (i + 1 < noff && a.off[i + 1] < a.off[i])
        *a.status = 1;
}

// Per-group counts: x = 0 wave tiles, 1 group tiles, 2 + j binary job counts
// of pass j, 2 + PM + j fan-in 4 job counts of pass j.
__global__ __launch_bounds__(kPlanBlock) void k_plan_count(PlanArgs a, uint32_t arrays)
{
    const uint64_t t = (uint64_t)blockIdx.x * kPlanBlock + threadIdx.x;
    const uint32_t x = (uint32_t)(t / a.G), g = (uint32_t)(t % a.G);
    if (x >= arrays)
        return;
    const bool ok = *a.status == 0;
    const GroupInfo gi = group_info(a, ok ? g : 0);
    if (x == 0) {
        a.bw[g] = (ok && gi.run0 == (uint32_t)kTile) ? gi.nruns : 0;
    } else if (x == 1) {
        a.bg[g] = (ok && gi.run0 > (uint32_t)kTile) ? gi.nruns : 0;
    } else if (x < 2 + a.PM) {
        const uint32_t j = x - 1;  // 1-based pass
        a.gjob[j - 1][g] = ok ? jobs_in(gi, j) : 0;
    } else {
        const uint32_t j = x - 1 - a.PM;  // 1-based pass
        a.gjob4[j - 1][g] = ok ? jobs4_in(gi, j) : 0;
    }
}

// Exclusive prefix sum of v[0, len) in place, v[len] = total (also to *total
// when set).  One work-group per array, in chunks of kPlanBlock * kScanPer
// elements: each thread sums kScanPer consecutive elements, the work-group
// scans those sums, and each thread writes its elements' prefixes.
constexpr uint32_t kScanPer = 4;

__device__ void block_scan(uint32_t *v, uint32_t len, uint32_t *total)
{
    __shared__ uint32_t sh[kPlanBlock];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < len; base += kPlanBlock * kScanPer) {
        const uint32_t i0 = base + threadIdx.x * kScanPer;
        uint32_t x[kScanPer], sum = 0;
#pragma unroll
        for (uint32_t e = 0; e < kScanPer; ++e) {
            x[e] = i0 + e < len ? v[i0 + e] : 0;
            sum += x[e];
        }
        sh[threadIdx.x] = sum;
        __syncthreads();
        for (uint32_t d = 1; d < kPlanBlock; d <<= 1) {
            const uint32_t y = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        const uint32_t incl = sh[threadIdx.x];
        const uint32_t c = carry;
        uint32_t run = c + incl - sum;  // prefix of this thread's first element
#pragma unroll
        for (uint32_t e = 0; e < kScanPer; ++e) {
            if (i0 + e < len)
                v[i0 + e] = run;
            run += x[e];
        }
        __syncthreads();
        if (threadIdx.x == kPlanBlock - 1)
            carry = c + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        v[len] = carry;
        if (total)
            *total = carry;
    }
}

// Scans of the per-group counts: block y = 0 wave tiles, 1 group tiles,
// 2 + j the binary job counts of pass j, 2 + PM + j the fan-in 4 ones.
__global__ __launch_bounds__(kPlanBlock) void k_plan_scan_groups(PlanArgs a, uint32_t first_array)
{
    const uint32_t x = blockIdx.x + first_array;
    if (x == 0)
        block_scan(a.bw, a.G, a.wcount);
    else if (x == 1)
        block_scan(a.bg, a.G, a.gcount);
    else if (x < 2 + a.PM)
        block_scan(a.gjob[x - 2], a.G, nullptr);
    else
        block_scan(a.gjob4[x - 2 - a.PM], a.G, nullptr);
}

// Largest i in [0, n) with v[i] <= x (v nondecreasing, v[0] <= x).
__device__ uint32_t upper_index(const uint32_t *v, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;  // v[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (v[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Block-sort tiles (segments): slot t of the wave (y = 0) or group (y = 1)
// list.
__global__ __launch_bounds__(kPlanBlock) void k_plan_block_tiles(PlanArgs a)
{
    const uint32_t t = blockIdx.x * kPlanBlock + threadIdx.x;
    const bool group = blockIdx.y == 1;
    const uint32_t *pre = group ? a.bg : a.bw;
    if (t >= (group ? a.gb : a.wb) || t >= pre[a.G])
        return;
    const uint32_t g = upper_index(pre, a.G, t);
    const GroupInfo gi = group_info(a, g);
    const uint64_t o = (uint64_t)(t - pre[g]) * gi.run0;
    BlockTile b;
    b.start = gi.start + o;
    b.count = (uint32_t)min<uint64_t>(gi.run0, gi.end - gi.start - o);
    b.dst = buf_after(gi, 0);
    (group ? a.gtiles : a.wtiles)[t] = b;
}

// Jobs of every pass: thread (j, slot) builds job `slot` of pass j from its
// group's run boundaries and writes its tile count.
__global__ __launch_bounds__(kPlanBlock) void k_plan_jobs(PlanArgs a)
{
    const uint32_t j = blockIdx.y;  // 0-based pass
    const uint32_t slot = blockIdx.x * kPlanBlock + threadIdx.x;
    const uint32_t *pre = a.gjob[j];
    const uint32_t total = min(pre[a.G], a.jb[j]);
    if (slot >= total)
        return;
    const uint32_t g = upper_index(pre, a.G, slot);
    const uint32_t q = slot - pre[g];
    const GroupInfo gi = group_info(a, g);
    const uint32_t pass = j + 1;
    MergeJob m;
    if (pass - gi.steps4 <= gi.merges) {  // pass > steps4: binary jobs exist only then
        const uint64_t half = binary_unit(gi, pass - gi.steps4), span = 2 * half;
        const uint64_t r0 = q * span;
        const uint32_t rm = (uint32_t)min<uint64_t>(r0 + half, gi.nruns);
        const uint32_t r1 = (uint32_t)min<uint64_t>(r0 + span, gi.nruns);
        const uint64_t b0 = run_bound(a, gi, (uint32_t)r0), bm = run_bound(a, gi, rm), b1 = run_bound(a, gi, r1);
        m.a_start = b0;
        m.na = (uint32_t)(bm - b0);
        m.nb = (uint32_t)(b1 - bm);
    } else {  // copy pass: the whole group as one run
        m.a_start = gi.start;
        m.na = (uint32_t)(gi.end - gi.start);
        m.nb = 0;
    }
    m.first_tile = 0;
    m.src = pass == 1 ? (gi.run0 ? buf_after(gi, 0) : (uint16_t)kBufIn) : buf_after(gi, pass - 1);
    m.dst = buf_after(gi, pass);
    a.jobs[j][slot] = m;
    a.jtile[j][slot] = (uint32_t)(((uint64_t)m.na + m.nb + kTile - 1) / kTile);
}

// Tile counts of every pass's jobs -> first tiles (one work-group per pass).
__global__ __launch_bounds__(kPlanBlock) void k_plan_scan_jobs(PlanArgs a)
{
    const uint32_t j = blockIdx.x;
    const uint32_t njobs = min(a.gjob[j][a.G], a.jb[j]);
    block_scan(a.jtile[j], njobs, a.tcount + j);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < njobs; i += kPlanBlock)
        a.jobs[j][i].first_tile = a.jtile[j][i];
    if (threadIdx.x == 0 && a.tcount[j] > a.tb[j])
        a.tcount[j] = a.tb[j];  // never more tiles than the launches cover
}

// Tile-to-job maps of every pass.
__global__ __launch_bounds__(kPlanBlock) void k_plan_tile_map(PlanArgs a)
{
    const uint32_t j = blockIdx.y;
    const uint32_t t = blockIdx.x * kPlanBlock + threadIdx.x;
    if (t >= a.tb[j] || t >= a.tcount[j])
        return;
    const uint32_t njobs = min(a.gjob[j][a.G], a.jb[j]);
    a.tjob[j][t] = upper_index(a.jtile[j], njobs, t);
}

// Fan-in 4 jobs of every pass: thread (j, slot) builds job `slot` of pass j
// (four runs of 4^j run0 / 4 keys of its segment) and its counts of cut
// searches, item slots and cut records.
__global__ __launch_bounds__(kPlanBlock) void k_plan_jobs4(PlanArgs a)
{
    const uint32_t j = blockIdx.y;  // 0-based pass
    const uint32_t slot = blockIdx.x * kPlanBlock + threadIdx.x;
    const uint32_t *pre = a.gjob4[j];
    const uint32_t total = min(pre[a.G], a.j4b[j]);
    if (slot >= total)
        return;
    const uint32_t g = upper_index(pre, a.G, slot);
    const uint32_t q = slot - pre[g];
    const GroupInfo gi = group_info(a, g);
    const uint32_t pass = j + 1;
    const uint64_t unit = 1ull << (2 * j), span = 4 * unit;  // runs of run0 keys
    uint64_t b[5];
    for (int t = 0; t <= 4; ++t)
        b[t] = run_bound(a, gi, (uint32_t)min<uint64_t>(q * span + t * unit, gi.nruns));
    Merge4Job m;
    m.start = b[0];
    for (int t = 0; t < 4; ++t)
        m.n[t] = (uint32_t)(b[t + 1] - b[t]);
    m.cut_off = m.item_off = m.task_off = 0;
    // the first pass of explicit runs reads the caller's input
    m.src = pass == 1 ? (gi.run0 ? buf_after(gi, 0) : (uint16_t)kBufIn) : buf_after(gi, pass - 1);
    m.dst = buf_after(gi, pass);
    a.jobs4[j][slot] = m;
    const uint32_t J = merge4_ab_segments((uint64_t)m.n[0] + m.n[1]), M = merge4_cd_cuts((uint64_t)m.n[2] + m.n[3]);
    a.jt4[j][slot] = merge4_tasks(J, M);
    a.ji4[j][slot] = merge4_items(J, M);
    a.jr4[j][slot] = merge4_records(J, M);
}

// The fan-in 4 jobs' first search, item slot and cut record of every pass
// (one work-group per pass), and the pass's counts.  Counts past the bounds
// the launches and areas were sized for (never, by the bounds' construction)
// leave the pass with no job: nothing is read or written out of range.
__global__ __launch_bounds__(kPlanBlock) void k_plan_scan_jobs4(PlanArgs a)
{
    const uint32_t j = blockIdx.x;
    const uint32_t njobs = min(a.gjob4[j][a.G], a.j4b[j]);
    __shared__ uint32_t tot[3];
    block_scan(a.jt4[j], njobs, &tot[0]);
    __syncthreads();
    block_scan(a.ji4[j], njobs, &tot[1]);
    __syncthreads();
    block_scan(a.jr4[j], njobs, &tot[2]);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < njobs; i += kPlanBlock) {
        a.jobs4[j][i].task_off = a.jt4[j][i];
        a.jobs4[j][i].item_off = a.ji4[j][i];
        a.jobs4[j][i].cut_off = a.jr4[j][i];
    }
    if (threadIdx.x == 0) {
        const bool fits = tot[0] <= a.t4b && tot[1] <= a.i4b && tot[2] <= a.r4b;
        a.c4[j][0] = fits ? njobs : 0;
        a.c4[j][1] = fits ? tot[0] : 0;
        a.c4[j][2] = fits ? tot[1] : 0;
    }
}

// ------------------------------------------------------------- host side

struct PlanSpec {
    uint32_t kind;
    uint32_t G, k, s, pivot, extra_copy;
    uint64_t gmin;
    uint32_t grun;
    bool pairs;
    uint32_t noff;  // offsets read (validity check)
    uint32_t four;  // fan-in 4 steps (PlanArgs::four); the areas are reserved for every segmented plan
    bool reserve_four;  // explicit runs / buckets: size the areas of both fan-ins (temp queries)
};

// Bounds of a plan for at most cap keys.
struct PlanBounds {
    uint32_t PM;
    uint64_t wb, gb;
    uint64_t jb[kMaxPlanPasses], tb[kMaxPlanPasses];
    // fan-in 4 steps (segments): passes, jobs per pass, and cut
    // searches / item slots / cut records of any one pass
    uint32_t PM4;
    uint64_t j4b[kMaxPlan4Passes];
    uint64_t t4b, i4b, r4b;
};

// Fan-in 4 steps of a segment of `runs` runs: while more than two remain.
uint32_t four_steps(uint64_t runs)
{
    uint32_t st = 0;
    for (; runs > 2; runs = (runs + 3) / 4)
        ++st;
    return st;
}

// Merge levels of a group of `runs` runs: fan-in 4 steps (when `four`) while
// more than two remain, then binary ones.
uint32_t merge_levels(uint64_t runs, bool four)
{
    const uint32_t st = four ? four_steps(runs) : 0;
    for (uint32_t i = 0; i < st; ++i)
        runs = (runs + 3) / 4;
    return st + clog2(std::max<uint64_t>(runs, 1));
}

PlanBounds plan_bounds(const PlanSpec &sp, uint64_t cap)
{
    PlanBounds b{};
    const uint64_t tiles = (cap + kTile - 1) / kTile;
    if (sp.kind == kKindSegments) {
        b.PM = clog2(std::max<uint64_t>(tiles, 1));
        b.wb = tiles + sp.G;
        b.gb = (cap + sp.grun - 1) / sp.grun + sp.G;
        for (uint32_t j = 1; j <= b.PM; ++j)
            b.jb[j - 1] = ((tiles + sp.G) >> j) + 1 + sp.G;
        {
            // segment g has at most ceil(len_g / 4096) runs, so step j (of four
            // runs of 4^(j-1) each) at most (tiles + G) / 4^j + G jobs; a job of
            // t keys takes at most t / kAbStep + 1 searches and item slots, and
            // two more cut records
            b.PM4 = four_steps(tiles);
            for (uint32_t j = 1; j <= b.PM4; ++j)
                b.j4b[j - 1] = ((tiles + sp.G) >> (2 * j)) + sp.G + 1;
            const uint64_t most = b.PM4 ? b.j4b[0] : 0;
            b.t4b = b.i4b = (cap + kAbStep - 1) / kAbStep + most;
            b.r4b = b.i4b + 2 * most;
        }
    } else {
        const uint32_t nr = sp.kind == kKindRuns ? sp.k : sp.s;
        // a query reserves the binary pass count (the larger) and the fan-in 4 areas
        const uint32_t levels = merge_levels(nr, sp.four == 1 && !sp.reserve_four);
        if (sp.kind == kKindRuns)
            b.PM = levels + (sp.extra_copy ? 1 : 0);
        else
            b.PM = std::max<uint32_t>(levels, 1);
        for (uint32_t j = 1; j <= b.PM; ++j) {
            // every group: at most ceil(nr / 2^j) binary jobs while merging
            // (after fan-in 4 steps fewer), else one copy
            const uint64_t per = j <= levels ? ((uint64_t)nr + (1ull << j) - 1) >> j : 1;
            b.jb[j - 1] = per * sp.G;
        }
        if ((sp.four == 1 || sp.reserve_four) && four_steps(nr) <= (uint32_t)kMaxPlan4Passes) {
            // step j: ceil(nr / 4^j) jobs per group, every job of t keys at most
            // t / kAbStep + 1 searches and item slots and two more cut records
            b.PM4 = four_steps(nr);
            for (uint32_t j = 1; j <= b.PM4; ++j)
                b.j4b[j - 1] = (((uint64_t)nr + (1ull << (2 * j)) - 1) >> (2 * j)) * sp.G + 1;
            const uint64_t most = b.PM4 ? b.j4b[0] : 0;
            b.t4b = b.i4b = (cap + kAbStep - 1) / kAbStep + most;
            b.r4b = b.i4b + 2 * most;
        }
    }
    for (uint32_t j = 1; j <= b.PM; ++j)
        b.tb[j - 1] = tiles + b.jb[j - 1];
    return b;
}

// Temp layout: data ping-pong (keys [, values]), split list, status word,
// block-tile counts and lists, then per pass the job counts, jobs, tile
// counts and tile map, then the per-pass tile totals.
struct PlanLayout {
    uint64_t data, splits, status, bw, bg, wtiles, gtiles, wcount, gcount, tcount;
    uint64_t gjob[kMaxPlanPasses], jobs[kMaxPlanPasses], jtile[kMaxPlanPasses], tjob[kMaxPlanPasses];
    // fan-in 4 steps: per pass the job counts, jobs, per-job counts and pass
    // counts; one search map, item map and cut record area all passes share
    uint64_t gjob4[kMaxPlan4Passes], jobs4[kMaxPlan4Passes];
    uint64_t jt4[kMaxPlan4Passes], ji4[kMaxPlan4Passes], jr4[kMaxPlan4Passes], c4;
    uint64_t tmap4, imap4, cuts4;
    uint64_t total;
};

PlanLayout plan_layout(const PlanSpec &sp, const PlanBounds &b, uint64_t cap)
{
    PlanLayout L{};
    uint64_t o = 0;
    L.data = o;
    o += a256(cap * 4) * (sp.pairs ? 2 : 1);
    uint64_t maxtb = 1;
    for (uint32_t j = 0; j < b.PM; ++j)
        maxtb = std::max(maxtb, b.tb[j]);
    L.splits = o;
    o = a256(o + (maxtb + 1) * 4);
    L.status = o;
    L.wcount = o + 4;
    L.gcount = o + 8;
    o = a256(o + 16);
    L.tcount = o;
    o = a256(o + kMaxPlanPasses * 4);
    L.bw = o;
    o = a256(o + ((uint64_t)sp.G + 1) * 4);
    L.bg = o;
    o = a256(o + ((uint64_t)sp.G + 1) * 4);
    L.wtiles = o;
    o = a256(o + (sp.kind == kKindSegments ? b.wb : 0) * sizeof(BlockTile));
    L.gtiles = o;
    o = a256(o + (sp.kind == kKindSegments ? b.gb : 0) * sizeof(BlockTile));
    for (uint32_t j = 0; j < b.PM; ++j) {
        L.gjob[j] = o;
        o = a256(o + ((uint64_t)sp.G + 1) * 4);
        L.jobs[j] = o;
        o = a256(o + b.jb[j] * sizeof(MergeJob));
        L.jtile[j] = o;
        o = a256(o + (b.jb[j] + 1) * 4);
        L.tjob[j] = o;
        o = a256(o + b.tb[j] * 4);
    }
    if (b.PM4) {
        for (uint32_t j = 0; j < b.PM4; ++j) {
            L.gjob4[j] = o;
            o = a256(o + ((uint64_t)sp.G + 1) * 4);
            L.jobs4[j] = o;
            o = a256(o + b.j4b[j] * sizeof(Merge4Job));
            L.jt4[j] = o;
            o = a256(o + (b.j4b[j] + 1) * 4);
            L.ji4[j] = o;
            o = a256(o + (b.j4b[j] + 1) * 4);
            L.jr4[j] = o;
            o = a256(o + (b.j4b[j] + 1) * 4);
        }
        L.c4 = o;
        o = a256(o + kMaxPlan4Passes * 4 * 4);
        L.tmap4 = o;
        o = a256(o + b.t4b * 4);
        L.imap4 = o;
        o = a256(o + b.i4b * 4);
        L.cuts4 = o;
        o = a256(o + b.r4b * 16);
    }
    L.total = o;
    return L;
}

uint64_t plan_need(const PlanSpec &sp, uint64_t cap) { return plan_layout(sp, plan_bounds(sp, cap), cap).total; }

// The most keys a temp buffer of `bytes` holds for this plan (0 if none).
uint64_t plan_capacity(const PlanSpec &sp, uint64_t bytes)
{
    if (plan_need(sp, 0) > bytes)
        return 0;
    uint64_t lo = 0, hi = kMaxKeys;  // need(lo) <= bytes
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (plan_need(sp, mid) <= bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

bcf_status dev(hipError_t e) { return e == hipSuccess ? BCF_OK : BCF_ERR_DEVICE; }

// Enqueue the planner kernels and the sort / merge kernels of a plan.  keys
// (and values) in kb / vb; temp holds the layout for capacity cap.
bcf_status plan_and_run(const PlanSpec &sp, const uint64_t *off_dev, Bufs kb, Bufs vb, char *temp, uint64_t cap,
                        hipStream_t s)
{
    const PlanBounds b = plan_bounds(sp, cap);
    const PlanLayout L = plan_layout(sp, b, cap);
    if (b.PM > kMaxPlanPasses || sp.G == 0)
        return BCF_ERR_INVALID;
    for (uint32_t j = 0; j < b.PM; ++j)
        if (b.jb[j] > 0xFFFFFFFFull || b.tb[j] > 0xFFFFFFFFull)
            return BCF_ERR_INVALID;
    if (b.PM4 > kMaxPlan4Passes || b.t4b > 0xFFFFFFFFull || b.r4b > 0xFFFFFFFFull)
        return BCF_ERR_INVALID;
    // fan-in 4 launches only when some segment may take them: on, or auto with
    // a capacity that reaches the threshold
    const uint32_t P4 = (sp.four == 1 || (sp.four == 2 && cap >= kAutoFourWayMinN)) ? b.PM4 : 0;
    PlanArgs a{};
    a.off = off_dev;
    a.kind = sp.kind;
    a.G = sp.G;
    a.k = sp.k;
    a.s = sp.s;
    a.pivot = sp.pivot;
    a.extra_copy = sp.extra_copy;
    a.gmin = sp.gmin;
    a.grun = sp.grun;
    a.PM = b.PM;
    a.four = P4 ? sp.four : 0;
    a.PM4 = P4;
    a.cap = cap;
    a.status = reinterpret_cast<uint32_t *>(temp + L.status);
    a.bw = reinterpret_cast<uint32_t *>(temp + L.bw);
    a.bg = reinterpret_cast<uint32_t *>(temp + L.bg);
    a.wtiles = reinterpret_cast<BlockTile *>(temp + L.wtiles);
    a.gtiles = reinterpret_cast<BlockTile *>(temp + L.gtiles);
    a.wb = (uint32_t)std::min<uint64_t>(b.wb, 0xFFFFFFFFull);
    a.gb = (uint32_t)std::min<uint64_t>(b.gb, 0xFFFFFFFFull);
    a.wcount = reinterpret_cast<uint32_t *>(temp + L.wcount);
    a.gcount = reinterpret_cast<uint32_t *>(temp + L.gcount);
    a.tcount = reinterpret_cast<uint32_t *>(temp + L.tcount);
    for (uint32_t j = 0; j < b.PM; ++j) {
        a.gjob[j] = reinterpret_cast<uint32_t *>(temp + L.gjob[j]);
        a.jobs[j] = reinterpret_cast<MergeJob *>(temp + L.jobs[j]);
        a.jtile[j] = reinterpret_cast<uint32_t *>(temp + L.jtile[j]);
        a.tjob[j] = reinterpret_cast<uint32_t *>(temp + L.tjob[j]);
        a.jb[j] = (uint32_t)b.jb[j];
        a.tb[j] = (uint32_t)b.tb[j];
    }
    for (uint32_t j = 0; j < P4; ++j) {
        a.gjob4[j] = reinterpret_cast<uint32_t *>(temp + L.gjob4[j]);
        a.jobs4[j] = reinterpret_cast<Merge4Job *>(temp + L.jobs4[j]);
        a.jt4[j] = reinterpret_cast<uint32_t *>(temp + L.jt4[j]);
        a.ji4[j] = reinterpret_cast<uint32_t *>(temp + L.ji4[j]);
        a.jr4[j] = reinterpret_cast<uint32_t *>(temp + L.jr4[j]);
        a.c4[j] = reinterpret_cast<uint32_t *>(temp + L.c4) + 4 * j;
        a.j4b[j] = (uint32_t)b.j4b[j];
    }
    a.t4b = (uint32_t)b.t4b;
    a.i4b = (uint32_t)b.i4b;
    a.r4b = (uint32_t)b.r4b;
    // status, the block-tile totals and the pass totals start at zero (a small
    // fill kernel rather than a memset: the sequence may be captured in a graph)
    hipLaunchKernelGGL(k_plan_zero, dim3(1), dim3(64), 0, s, a);
    BCF_PLAN_TRY(dev(hipGetLastError()));
    {
        const uint32_t blocks = (sp.noff + kPlanBlock - 1) / kPlanBlock;
        hipLaunchKernelGGL(k_plan_check, dim3(blocks), dim3(kPlanBlock), 0, s, a, sp.noff);
        BCF_PLAN_TRY(dev(hipGetLastError()));
    }
    const bool segs = sp.kind == kKindSegments;
    const uint32_t arrays = 2 + b.PM + P4;
    {
        const uint64_t threads = (uint64_t)arrays * sp.G;
        hipLaunchKernelGGL(k_plan_count, dim3((uint32_t)((threads + kPlanBlock - 1) / kPlanBlock)), dim3(kPlanBlock),
                           0, s, a, arrays);
        BCF_PLAN_TRY(dev(hipGetLastError()));
        const uint32_t first = segs ? 0 : 2;
        if (arrays > first) {  // nothing to scan when no pass is planned (a lone run merged in place)
            hipLaunchKernelGGL(k_plan_scan_groups, dim3(arrays - first), dim3(kPlanBlock), 0, s, a, first);
            BCF_PLAN_TRY(dev(hipGetLastError()));
        }
    }
    if (segs) {
        const uint64_t most = std::max(b.wb, b.gb);
        hipLaunchKernelGGL(k_plan_block_tiles, dim3((uint32_t)((most + kPlanBlock - 1) / kPlanBlock), 2),
                           dim3(kPlanBlock), 0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
    }
    if (b.PM) {
        uint64_t mj = 1, mt = 1;
        for (uint32_t j = 0; j < b.PM; ++j) {
            mj = std::max(mj, b.jb[j]);
            mt = std::max(mt, b.tb[j]);
        }
        hipLaunchKernelGGL(k_plan_jobs, dim3((uint32_t)((mj + kPlanBlock - 1) / kPlanBlock), b.PM), dim3(kPlanBlock),
                           0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
        hipLaunchKernelGGL(k_plan_scan_jobs, dim3(b.PM), dim3(kPlanBlock), 0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
        hipLaunchKernelGGL(k_plan_tile_map, dim3((uint32_t)((mt + kPlanBlock - 1) / kPlanBlock), b.PM),
                           dim3(kPlanBlock), 0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
    }
    if (P4) {
        hipLaunchKernelGGL(k_plan_jobs4, dim3((uint32_t)((b.j4b[0] + kPlanBlock - 1) / kPlanBlock), P4),
                           dim3(kPlanBlock), 0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
        hipLaunchKernelGGL(k_plan_scan_jobs4, dim3(P4), dim3(kPlanBlock), 0, s, a);
        BCF_PLAN_TRY(dev(hipGetLastError()));
    }
    const bool pairs = sp.pairs;
    if (segs) {
        {
            void *p = prof_begin(kname_block_sort(pairs, true), s, 0.0);
            const hipError_t e = launch_block_sort_table(pairs, kb, vb, a.wtiles, a.wb, s, a.wcount);
            prof_end(p);
            BCF_PLAN_TRY(dev(e));
        }
        {
            void *p = prof_begin(kname_block_sort(pairs, true), s, 0.0);
            const hipError_t e = launch_block_sort_group_table(pairs, kb, vb, a.gtiles, a.gb, s, a.gcount);
            prof_end(p);
            BCF_PLAN_TRY(dev(e));
        }
    }
    uint32_t *splits = reinterpret_cast<uint32_t *>(temp + L.splits);
    uint32_t *tmap4 = reinterpret_cast<uint32_t *>(temp + L.tmap4);
    uint32_t *imap4 = reinterpret_cast<uint32_t *>(temp + L.imap4);
    for (uint32_t j = 0; j < b.PM; ++j) {
        // the fan-in 4 jobs of the pass (segments still taking fan-in 4 steps),
        // then its binary jobs (the other segments); they touch disjoint ranges
        for (int phase = 0; j < P4 && phase < 3; ++phase) {
            static const char *const names[2][3] = {{"map4_keys_table", "cuts4_keys_table", "merge4_keys_table"},
                                                    {"map4_pairs_table", "cuts4_pairs_table", "merge4_pairs_table"}};
            void *p = prof_begin(names[sp.pairs][phase], s, 0.0);
            const hipError_t e = launch_merge4_table(kb, a.jobs4[j], a.j4b[j], tmap4, a.t4b, imap4, a.i4b,
                                                     temp + L.cuts4, cap, phase, s, a.c4[j], vb);
            prof_end(p);
            BCF_PLAN_TRY(dev(e));
        }
        for (int phase = 0; phase < 2; ++phase) {
            const bool part = phase == 0;
            void *p = prof_begin(part ? kname_partition(pairs, true) : kname_merge(pairs, true), s, 0.0);
            const hipError_t e = launch_merge_table(pairs, kb, vb, a.jobs[j], a.tjob[j], a.tb[j], splits, part, s,
                                                    a.tcount + j);
            prof_end(p);
            BCF_PLAN_TRY(dev(e));
        }
    }
    return BCF_OK;
}

// The total of a device offset array (its last entry), read on the host:
// for temp queries only (synchronises the stream).
bcf_status read_total(const uint64_t *off_dev, uint64_t last, hipStream_t s, uint64_t &n)
{
    n = 0;
    if (hipMemcpyAsync(&n, off_dev + last, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return BCF_ERR_DEVICE;
    return n > kMaxKeys ? BCF_ERR_INVALID : BCF_OK;
}

// Layout of the keys [and values] ping-pong at the start of a plan's temp.
Bufs key_bufs(const uint32_t *in, uint32_t *out, char *temp) { return Bufs{in, out, reinterpret_cast<uint32_t *>(temp)}; }
Bufs val_bufs(const uint32_t *in, uint32_t *out, char *temp, uint64_t cap)
{
    return Bufs{in, out, reinterpret_cast<uint32_t *>(temp + a256(cap * 4))};
}

// A planned call: query (temp == NULL: the total is read from the device) or
// run with the capacity the temp buffer holds.
bcf_status planned_call(const PlanSpec &worst, const PlanSpec &actual, const uint64_t *off_dev, const uint32_t *kin,
                        const uint32_t *vin, uint32_t *kout, uint32_t *vout, void *temp, uint64_t *temp_bytes,
                        hipStream_t s)
{
    if (!temp) {
        uint64_t n = 0;
        BCF_PLAN_TRY(read_total(off_dev, worst.noff - 1, s, n));
        *temp_bytes = plan_need(worst, n);
        return BCF_OK;
    }
    if (!kin || !kout || (actual.pairs && (!vin || !vout)))
        return BCF_ERR_INVALID;
    const uint64_t cap = plan_capacity(actual, *temp_bytes);
    if (plan_need(actual, cap) > *temp_bytes)
        return BCF_ERR_TEMP_TOO_SMALL;
    char *tb = static_cast<char *>(temp);
    const Bufs kb = key_bufs(kin, kout, tb);
    const Bufs vb = actual.pairs ? val_bufs(vin, vout, tb, cap) : Bufs{nullptr, nullptr, nullptr};
    return plan_and_run(actual, off_dev, kb, vb, tb, cap, s);
}

uint64_t seg_group_min(bool pairs, uint64_t knob) { return knob ? knob : group_run_keys(pairs) / 2; }

// Fan-in 4 steps for the merges of explicit runs (bcf_merge_runs) or of the
// buckets of the sort by distribution, groups of nr runs: tuning knob
// merge_fan_in 4 on, 2 off, 0 (auto) from 16 runs per group (decided on the
// host, which does not know the key count: 2^20 keys in 8 runs merge in
// 0.146 ms binary against 0.166 ms four-way, 2^24 keys in 16 runs alike, 2^26
// keys in 16 / 256 / 4096 runs 0.72 / 1.30 / 1.77 ms binary against 0.58 /
// 1.02 / 1.41 ms); never for more runs than kMaxPlan4Passes steps reduce.
bool runs_four_way(uint32_t nr)
{
    const int f = tuning().merge_fan_in;
    return (f == 4 || (f == 0 && nr >= 16)) && four_steps(nr) <= (uint32_t)kMaxPlan4Passes;
}

bcf_status segmented_device(bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                            const uint64_t *off, uint32_t nseg, void *temp, uint64_t *temp_bytes, hipStream_t s)
{
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    if (nseg == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    if (!off)
        return BCF_ERR_INVALID;
    PlanSpec sp{};
    sp.kind = kKindSegments;
    sp.G = nseg;
    sp.gmin = seg_group_min(pairs, tuning().group_min_keys);
    sp.grun = group_run_keys(pairs);
    sp.pairs = pairs;
    sp.noff = nseg + 1;
    const int fan_in = tuning().merge_fan_in;
    sp.four = fan_in == 4 ? 1u : (fan_in == 0 ? 2u : 0u);
    return planned_call(sp, sp, off, kin, vin, kout, vout, temp, temp_bytes, s);
}

}  // namespace

}  // namespace bcf

using namespace bcf;

extern "C" {

bcf_status bcf_merge_runs(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets, uint32_t k,
                          uint32_t *keys_out, uint32_t *vals_out, void *temp, uint64_t *temp_bytes, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    if (k == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    if (!run_offsets || k == 0xFFFFFFFFu)
        return BCF_ERR_INVALID;
    const bool pairs = vals_in != nullptr;
    const bool four = runs_four_way(k);
    const uint32_t merges = merge_levels(k, four);
    PlanSpec sp{};
    sp.kind = kKindRuns;
    sp.G = 1;
    sp.k = k;
    sp.pairs = pairs;
    sp.noff = k + 1;
    sp.four = four ? 1u : 0u;
    PlanSpec worst = sp;
    // the temp size depends neither on whether the call is in place nor on the fan-in
    worst.extra_copy = 1;
    worst.four = 0;
    worst.reserve_four = true;
    const bool inplace = keys_in == keys_out || (pairs && vals_in == vals_out);
    // in place, a run count whose merge levels are odd would make the first pass
    // read and write the output: one more pass copies the result from temp; a
    // lone run not in place is one copy
    sp.extra_copy = merges == 0 ? (inplace ? 0u : 1u) : ((inplace && merges % 2 == 1) ? 1u : 0u);
    if (temp && tuning().check_runs && keys_in) {
        // sortedness of every run, flagged in a spare word of the plan's
        // status area (synchronises the stream)
        uint64_t n = 0;
        BCF_PLAN_TRY(read_total(run_offsets, k, s, n));
        const uint64_t cap = plan_capacity(sp, *temp_bytes);
        if (plan_need(sp, cap) > *temp_bytes || n > cap)
            return BCF_ERR_TEMP_TOO_SMALL;
        const PlanLayout L = plan_layout(sp, plan_bounds(sp, cap), cap);
        uint32_t *flag_d = reinterpret_cast<uint32_t *>(static_cast<char *>(temp) + L.status + 12);
        uint32_t flag = 0;
        const bool ok = hipMemsetAsync(flag_d, 0, sizeof(uint32_t), s) == hipSuccess &&
                        launch_check_runs(keys_in, run_offsets, k, n, flag_d, s) == hipSuccess &&
                        hipMemcpyAsync(&flag, flag_d, sizeof(uint32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
                        hipStreamSynchronize(s) == hipSuccess;
        if (!ok)
            return BCF_ERR_DEVICE;
        if (flag)
            return BCF_ERR_UNSORTED_RUN;
    }
    return planned_call(worst, sp, run_offsets, keys_in, vals_in, keys_out, vals_out, temp, temp_bytes, s);
}

bcf_status bcf_segmented_sort(const uint32_t *keys_in, uint32_t *keys_out, const uint64_t *seg_offsets, uint32_t nseg,
                              void *temp, uint64_t *temp_bytes, void *stream)
{
    return segmented_device(false, keys_in, nullptr, keys_out, nullptr, seg_offsets, nseg, temp, temp_bytes,
                            static_cast<hipStream_t>(stream));
}

bcf_status bcf_segmented_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                    uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg, void *temp,
                                    uint64_t *temp_bytes, void *stream)
{
    return segmented_device(true, keys_in, vals_in, keys_out, vals_out, seg_offsets, nseg, temp, temp_bytes,
                            static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_u32_pb(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, uint32_t P, uint32_t run_keys,
                           int pivot_buckets, void *temp, uint64_t *temp_bytes, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!temp_bytes || n > kMaxKeys || P < 1 || P > 65536 || run_keys < 1)
        return BCF_ERR_INVALID;
    if (n == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    const uint64_t s64 = (n + run_keys - 1) / run_keys;
    const uint32_t nb = pivot_buckets ? 2 * P - 1 : P;
    // the distribution step's limits (bcf_distribute_runs)
    if (s64 > (1u << 22) || s64 * P > (1ull << 26) || (uint64_t)nb * s64 > (1ull << 24))
        return BCF_ERR_INVALID;
    const uint32_t s = (uint32_t)s64;
    std::vector<uint64_t> seg(s + 1);
    for (uint32_t r = 0; r <= s; ++r)
        seg[r] = std::min<uint64_t>((uint64_t)r * run_keys, n);
    // temp: the distributed keys, the piece offsets, then one scratch area the
    // three steps use in turn (run sort, distribution, bucket merge)
    uint64_t need_runs = 0, need_dist = 0;
    BCF_PLAN_TRY(bcf_segmented_sort_host(nullptr, nullptr, seg.data(), s, nullptr, &need_runs, st));
    BCF_PLAN_TRY(bcf_distribute_runs(nullptr, seg.data(), s, P, P, pivot_buckets, nullptr, nullptr, nullptr, nullptr,
                                     &need_dist, st));
    PlanSpec sp{};
    sp.kind = kKindBuckets;
    sp.G = nb;
    sp.s = s;
    sp.pivot = pivot_buckets ? 1 : 0;
    sp.noff = nb * s + 1;
    sp.four = runs_four_way(s) ? 1u : 0u;
    PlanSpec worst = sp;  // the temp size does not depend on the fan-in
    worst.four = 0;
    worst.reserve_four = true;
    const uint64_t need_merge = plan_need(worst, n);
    const uint64_t d_bytes = a256(n * 4), p_bytes = a256(((uint64_t)nb * s + 1) * 8);
    const uint64_t scratch = std::max(need_runs, std::max(need_dist, need_merge));
    const uint64_t need = d_bytes + p_bytes + scratch;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (!keys_in || !keys_out || keys_in == keys_out)
        return BCF_ERR_INVALID;
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    char *tb = static_cast<char *>(temp);
    uint32_t *dist = reinterpret_cast<uint32_t *>(tb);
    uint64_t *pieces = reinterpret_cast<uint64_t *>(tb + d_bytes);
    void *scr = tb + d_bytes + p_bytes;
    uint64_t sb = scratch;
    // sorted runs of run_keys keys into the output, then the distribution of
    // the runs into bucket-major pieces, then every bucket merged into the
    // output (piece offsets stay on the device)
    BCF_PLAN_TRY(bcf_segmented_sort_host(keys_in, keys_out, seg.data(), s, scr, &sb, st));
    sb = scratch;
    BCF_PLAN_TRY(bcf_distribute_runs(keys_out, seg.data(), s, P, P, pivot_buckets, dist, pieces, nullptr, scr, &sb,
                                     st));
    return plan_and_run(sp, pieces, key_bufs(dist, keys_out, static_cast<char *>(scr)), Bufs{nullptr, nullptr, nullptr},
                        static_cast<char *>(scr), n, st);
}

}  // extern "C"
