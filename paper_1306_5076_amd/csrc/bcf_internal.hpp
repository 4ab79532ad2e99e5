// Internal interface between the host planner (bcf_api.hip) and the kernels
// (bcf_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcf {

// Buffer selector used by table-driven launches: kernels receive the three
// candidate buffers {caller input, caller output, temp} and each work item
// names which one it reads from and which one it writes to.
enum BufSel : uint32_t { kBufIn = 0, kBufOut = 1, kBufTemp = 2 };

struct Bufs {
    const uint32_t *in;  // caller input (read only)
    uint32_t *out;       // caller output
    uint32_t *temp;      // library scratch
};

// Key samples of a sorted array, written by the pass that produces it and
// read by the partition of the next merge pass: the key at every position
// 64j (f) and 64j + 63 (l), and at every position 4096t (cf) and
// 4096t + 4095 (cl).  f == nullptr means "no samples".
struct SampleSet {
    uint32_t *f, *l, *cf, *cl;
};

// Order-preserving map between another 32-bit key type and u32, applied to a
// key as it is loaded (forward) or stored (inverse): x ^ (sign | (s & rest))
// with s the arithmetic sign extension of x (forward) or of ~x (inverse).
// int32: (sign, rest) = (0x80000000, 0); IEEE binary32 ordered by totalOrder:
// (0x80000000, 0x7fffffff).  sign == 0 is the identity (u32 keys).
struct KeyMap {
    uint32_t sign = 0, rest = 0, inverse = 0;
};
KeyMap key_map(int kind, bool inverse);  // kind 0 (identity), 1 int32, 2 float

// One tile of the block sort: `count` (<= kTile) keys starting at element
// `start` of the input, sorted into buffer `dst` at the same offset.
struct BlockTile {
    uint64_t start;
    uint32_t count;
    uint32_t dst;
};

// One binary merge of two adjacent sorted runs A = [a_start, a_start + na)
// and B = [a_start + na, a_start + na + nb) of buffer `src`, written to the
// same range of buffer `dst`.  Its output is cut into ceil((na+nb)/kTile)
// tiles numbered first_tile, first_tile + 1, ... in the launch.
struct MergeJob {
    uint64_t a_start;
    uint32_t na;
    uint32_t nb;
    uint32_t first_tile;
    uint16_t src;
    uint16_t dst;
};

// One fan-in 4 merge of a table-driven pass (keys only): runs A, B, C, D of
// n[0..3] keys lying back to back from `start` in buffer `src`, merged into
// the same range of buffer `dst`.  Its cut records (AB cuts P[0..J], then CD
// cuts Q[0..M]) start at record cut_off of the pass's cut array, its merge
// items at slot item_off and its cut searches at task task_off of the pass
// (J = AB segments, M = interior CD cuts of the job, see the four-way merge).
struct Merge4Job {
    uint64_t start;
    uint32_t n[4];
    uint32_t cut_off, item_off, task_off;
    uint16_t src, dst;
};

// Waves per work-group of the group block sort (keys / pairs); the sorted
// runs it produces hold that many 4096-key tiles.
constexpr int kGroupWavesKeys = 8;
constexpr int kGroupWavesPairs = 4;
uint32_t group_run_keys(bool pairs);

// Launchers (enqueue only; return the launch status).
// in_map is applied to the keys as they are loaded, out_map as they are stored
// (the block sort writes the output itself when it is the only pass).
hipError_t launch_block_sort_group(bool pairs, const uint32_t *kin, const uint32_t *vin,
                                   uint32_t *kout, uint32_t *vout, uint64_t n, SampleSet out_smp,
                                   hipStream_t s, KeyMap in_map = {}, KeyMap out_map = {});
// Keys only: group tiles sorted by the paper's long ShearSort over the waves
// of a work-group (block-sort ablation); same runs and samples as the group
// sort of launch_block_sort_group.
hipError_t launch_block_sort_shear_group(const uint32_t *kin, uint32_t *kout, uint64_t n, SampleSet out_smp,
                                         hipStream_t s);
// Wave tiles of 4096 keys (runs of 4096), sorted by merge rounds or, with
// shear, by the paper's ShearSort; writes the samples of its output (out_smp).
hipError_t launch_block_sort_regular(bool pairs, bool shear, const uint32_t *kin, const uint32_t *vin,
                                     uint32_t *kout, uint32_t *vout, uint64_t n, SampleSet out_smp,
                                     hipStream_t s, KeyMap in_map = {}, KeyMap out_map = {});
// A merge pass is two launches: with partition = true the split of every
// tile is written to `splits` (one u32 per tile of the pass); with
// partition = false the tiles are merged using those splits.
// The regular partition reads the samples of its input (in_smp, written by
// the previous launch); the regular merge writes those of its output (out_smp).
struct Tuning;
// Whether, under tuning tu, a regular merge pass is one launch (its merge
// kernel searches the splits from the samples in in_smp) instead of a
// partition launch and a merge launch.  The caller decides once per pass and
// passes the answer to both launch_merge_regular calls (with fused = true the
// partition call enqueues nothing).
bool merge_fuses_partition(bool pairs, const SampleSet &in_smp, const Tuning &tu);
hipError_t launch_merge_regular(bool pairs, const uint32_t *ksrc, const uint32_t *vsrc,
                                uint32_t *kdst, uint32_t *vdst, uint64_t n, uint64_t run,
                                uint32_t *splits, SampleSet in_smp, SampleSet out_smp,
                                bool partition, bool fused, hipStream_t s, KeyMap out_map = {});
// Fan-in 4 merge pass of a regular sort: groups of four runs of `run` keys
// (a multiple of 4096) become runs of 4 run.  The cut phase (cut_phase =
// true) searches the pass's work split from the samples of the input (in_smp,
// required) into `cuts` (merge4_cut_bytes(n, run) bytes); the merge phase then
// merges and writes the samples of its output (out_smp).  With vsrc / vdst the
// pass is a stable key/value pass (values laid out like the keys).
uint64_t merge4_cut_bytes(uint64_t n, uint64_t run);
uint64_t merge4_cut_bytes_max(uint64_t n);  // the largest over every plan of an n-key sort (keys or pairs)
hipError_t launch_merge4_regular(const uint32_t *ksrc, uint32_t *kdst, uint64_t n, uint64_t run, void *cuts,
                                 SampleSet in_smp, SampleSet out_smp, bool cut_phase, hipStream_t s,
                                 KeyMap out_map = {}, const uint32_t *vsrc = nullptr, uint32_t *vdst = nullptr);
// Table launches: the grid covers ntiles (ngroups) tiles; with count_dev set
// the kernels take the actual count from that device word (at most the bound),
// so that a device planner can size the work after the launch was enqueued.
hipError_t launch_block_sort_table(bool pairs, Bufs kb, Bufs vb, const BlockTile *tiles,
                                   uint32_t ntiles, hipStream_t s, const uint32_t *count_dev = nullptr);
// Group tiles (count <= group_run_keys(pairs)) sorted by a multi-wave work-group.
hipError_t launch_block_sort_group_table(bool pairs, Bufs kb, Bufs vb, const BlockTile *tiles,
                                         uint32_t ngroups, hipStream_t s, const uint32_t *count_dev = nullptr);
hipError_t launch_merge_table(bool pairs, Bufs kb, Bufs vb, const MergeJob *jobs,
                              const uint32_t *tile_job, uint32_t ntiles, uint32_t *splits,
                              bool partition, hipStream_t s, const uint32_t *count_dev = nullptr);
// Fan-in 4 table pass (keys): AB / CD segment and cut counts of a job (the
// planner sizes its records and items by them), and the three launches of a
// pass over `njobs` jobs (phase 0: the maps from cut searches and item slots
// to jobs, task_job and item_job, from the jobs' first indices; 1: the
// `tasks` cut searches, which also write every job's first and last AB cut
// into `cuts`; 2: the merges of the `items` slots).  `keys` is the number of
// keys the pass merges (it decides the nontemporal hints).
// Cut steps of the four-way merge (multiples of the 64-key sample blocks, at
// most half a 4096-key tile): AB cuts every kAbStep keys, CD cuts every
// kCdStep keys.  AB segments of a group whose AB side holds nab keys (at
// least one, so that a group with an empty AB side still has an item), and
// its interior CD cuts (CD positions kCdStep m with 0 < kCdStep m < ncd).
constexpr uint32_t kAbStep = 1920;
constexpr uint32_t kCdStep = 2048;
__host__ __device__ constexpr uint32_t ab_segments(uint64_t nab)
{
    return nab > kAbStep ? (uint32_t)((nab + kAbStep - 1) / kAbStep) : 1u;
}
__host__ __device__ constexpr uint32_t cd_cuts(uint64_t ncd) { return ncd ? (uint32_t)((ncd - 1) / kCdStep) : 0u; }
__host__ __device__ constexpr uint32_t merge4_ab_segments(uint64_t nab) { return ab_segments(nab); }
__host__ __device__ constexpr uint32_t merge4_cd_cuts(uint64_t ncd) { return cd_cuts(ncd); }
// Cut searches, item slots and cut records of one fan-in 4 job (J AB
// segments, M interior CD cuts): at least one search (the first writes the
// job's end records).
__host__ __device__ constexpr uint32_t merge4_tasks(uint32_t J, uint32_t M) { return J - 1 + M > 0 ? J - 1 + M : 1u; }
__host__ __device__ constexpr uint32_t merge4_items(uint32_t J, uint32_t M) { return J + M; }
__host__ __device__ constexpr uint32_t merge4_records(uint32_t J, uint32_t M) { return J + M + 2; }
// With counts_dev set the three counts come from device words (jobs,
// searches, item slots) and njobs / tasks / items are their bounds: the
// launches then stride over the counts with grids sized by the chip.
// With vb.in set the merges carry values (stable key/value jobs, values laid
// out like the keys in vb's three buffers).
hipError_t launch_merge4_table(Bufs kb, const Merge4Job *jobs, uint32_t njobs, uint32_t *task_job, uint32_t tasks,
                               uint32_t *item_job, uint32_t items, void *cuts, uint64_t keys, int phase,
                               hipStream_t s, const uint32_t *counts_dev = nullptr,
                               Bufs vb = Bufs{nullptr, nullptr, nullptr});
hipError_t launch_check_runs(const uint32_t *keys, const uint64_t *run_ends_dev, uint32_t k,
                             uint64_t n, uint32_t *flag, hipStream_t s);

// Segmented sorts of at least this many keys in all take four-way merge
// steps under the default (auto) fan-in.
constexpr uint64_t kAutoFourWayMinN = 1ull << 25;
// Sorts of keys take four-way merge passes under the default fan-in from
// this many keys (uniform keys, binary / four-way: 2^18 0.072 / 0.076 ms,
// 2^20 0.102 / 0.104, 2^22 0.168 / 0.156, 2^23 0.196 / 0.198, 2^24 0.365 /
// 0.311, 2^25 0.709 / 0.558); below it a pass's data stays in the 256 MiB
// last-level cache and halving the passes barely pays for the second launch
// and the heavier merge.  Key/value sorts take them at every size (2^18
// pairs 0.169 / 0.135 ms, 2^20 0.197 / 0.163, 2^24 1.021 / 0.702).
constexpr uint64_t kAutoFourWayMinKeys = 1ull << 24;

// Current process-wide tuning (see bcf_tuning in bcf.h); a copy.
struct Tuning {
    int block_sort;  // 0 auto, 1 wave tiles (merge rounds), 2 wave tiles (ShearSort), 3 group tiles
    bool partition_half;  // sampled partition: one half-wave (else one wave) per tile (env BCF_PARTITION_HALF)
    bool fused_partition; // one-tile-per-wave merges of regular passes search their own splits
    int merge_variant;
    bool nontemporal;
    bool sampled_partition;
    bool tile_samples;
    uint64_t group_min_keys;
    bool check_runs;
    int merge_fan_in;  // 0 auto, 2 or 4: runs merged per group in the merge passes of a keys-only sort
};
Tuning tuning();

// While an object of this type lives, the calling thread's library calls
// create and record no per-launch timing events (bcf_profile_enable): for
// entry points that must not create runtime objects.
struct ProfilingOff {
    ProfilingOff();
    ~ProfilingOff();
    ProfilingOff(const ProfilingOff &) = delete;
    ProfilingOff &operator=(const ProfilingOff &) = delete;
};

// Names used for per-kernel timing records.
const char *kname_block_sort(bool pairs, bool table);
const char *kname_partition(bool pairs, bool table);
const char *kname_merge(bool pairs, bool table);

// Work-group shape of the sort kernels: waves per work-group.
constexpr int kWavesPerGroup = 2;

}  // namespace bcf
