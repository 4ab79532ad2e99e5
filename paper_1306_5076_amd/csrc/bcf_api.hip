// C ABI of the bank-conflict-free sort: argument checking, host-side pass
// planning, descriptor upload and kernel launches.  See include/bcf.h.
//
// Plan of a sort of n keys (BCFMergesort, paper Sec. 3 and Lemma 2):
//   one block-sort launch turns [0, n) into sorted runs of 4096 keys (wave
//   tiles) or 32768 keys (16384 pairs; multi-wave group tiles), then
//   ceil(log2(#runs)) binary merge passes double the run length until one run
//   remains.  Passes ping-pong between the output and the temp buffer; the
//   block sort writes to whichever buffer makes the last pass end in the
//   output.  Every launch is enqueued on the caller's stream; nothing
//   synchronises the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bcf.h"
#include "bcf_device.hpp"
#include "bcf_internal.hpp"

using namespace bcf;

namespace {

constexpr uint64_t kMaxN = 0xFFFFFFFFull;

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint32_t ceil_log2(uint64_t x)
{
    uint32_t p = 0;
    while ((uint64_t(1) << p) < x)
        ++p;
    return p;
}

uint64_t tiles_of(uint64_t n) { return (n + kTile - 1) / kTile; }

// ------------------------------------------------------------------ profiling

struct ProfRec {
    hipEvent_t a, b;
    double bytes;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, std::vector<ProfRec>> g_prof;
thread_local int t_prof_off = 0;  // > 0: this thread's calls record no timing events

struct ProfScope {
    const char *name;
    hipStream_t s;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    ProfScope(const char *nm, hipStream_t st, double by) : name(nm), s(st), bytes(by)
    {
        {
            std::lock_guard<std::mutex> g(g_prof_mu);
            on = g_prof_on && t_prof_off == 0;
        }
        if (on) {
            if (hipEventCreate(&a) != hipSuccess) {
                on = false;
                return;
            }
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                on = false;
                return;
            }
            (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope()
    {
        if (!on)
            return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof[name].push_back({a, b, bytes});
    }
};

// ------------------------------------------------------- descriptor staging

// Pinned host buffers holding descriptor tables while their host-to-device
// copy is in flight.  A buffer is reused once the event recorded after its
// copy has completed.
struct Staging {
    void *ptr = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

std::mutex g_stage_mu;
std::vector<Staging> g_stage;

// Copy `bytes` from host memory `src` to device `dst` on stream `s` through a
// pinned staging buffer.
bcf_status upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return BCF_OK;
    std::lock_guard<std::mutex> g(g_stage_mu);
    Staging *slot = nullptr;
    for (auto &st : g_stage) {
        if (st.cap >= bytes && hipEventQuery(st.done) == hipSuccess) {
            slot = &st;
            break;
        }
    }
    if (!slot) {
        Staging st;
        st.cap = std::max<size_t>(bytes, 1 << 20);
        if (hipHostMalloc(&st.ptr, st.cap, hipHostMallocDefault) != hipSuccess)
            return BCF_ERR_NOMEM;
        if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(st.ptr);
            return BCF_ERR_DEVICE;
        }
        g_stage.push_back(st);
        slot = &g_stage.back();
    }
    std::memcpy(slot->ptr, src, bytes);
    if (hipMemcpyAsync(dst, slot->ptr, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return BCF_ERR_DEVICE;
    if (hipEventRecord(slot->done, s) != hipSuccess)
        return BCF_ERR_DEVICE;
    return BCF_OK;
}

bcf_status dev_status(hipError_t e) { return e == hipSuccess ? BCF_OK : BCF_ERR_DEVICE; }

// ------------------------------------------------------------------- tuning

std::mutex g_tune_mu;
bool g_tune_init = false;
Tuning g_tune;

int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return (e && *e) ? std::atoi(e) : dflt;
}

Tuning &tuning_locked()
{
    if (!g_tune_init) {
        g_tune.merge_variant = env_int("BCF_MERGE_MODE", 3);
        if (g_tune.merge_variant < 0 || g_tune.merge_variant > 3)
            g_tune.merge_variant = 3;
        g_tune.nontemporal = env_int("BCF_NT", 1) != 0;
        g_tune.sampled_partition = std::getenv("BCF_NO_SAMPLES") == nullptr;
        g_tune.tile_samples = env_int("BCF_TILE_SAMPLES", 1) != 0;
        const char *e = std::getenv("BCF_SEG_GROUP_MIN");
        g_tune.group_min_keys = (e && *e) ? std::strtoull(e, nullptr, 10) : 0;
        g_tune.check_runs = env_int("BCF_CHECK", 0) == 1;
        g_tune.partition_half = env_int("BCF_PARTITION_HALF", 1) != 0;
        g_tune.fused_partition = env_int("BCF_FUSED", 1) != 0;
        g_tune.block_sort = env_int("BCF_BLOCK_SORT", 0);
        if (g_tune.block_sort < 0 || g_tune.block_sort > 4)
            g_tune.block_sort = 0;
        g_tune.merge_fan_in = env_int("BCF_FAN_IN", 0);
        if (g_tune.merge_fan_in != 2 && g_tune.merge_fan_in != 4)
            g_tune.merge_fan_in = 0;
        g_tune_init = true;
    }
    return g_tune;
}

#define BCF_TRY(x)                          \
    do {                                    \
        bcf_status st_ = (x);               \
        if (st_ != BCF_OK)                  \
            return st_;                     \
    } while (0)

bool offsets_valid(const uint64_t *off, uint32_t k)
{
    if (!off || off[0] != 0)
        return false;
    for (uint32_t r = 0; r < k; ++r)
        if (off[r + 1] < off[r])
            return false;
    return off[k] <= kMaxN;
}

// ---------------------------------------------------- full sort (regular)

// Sort keys (and values) with the regular plan.  temp holds the ping-pong
// key buffer followed by the value buffer.
// Sorts of at most this many keys take wave tiles under the default (auto)
// block sort: a group tile occupies one CU for the whole block sort, so a
// sort with fewer groups than CUs finishes sooner with 8x more, smaller
// tiles and a few more (short) merge passes.
constexpr uint64_t kAutoWaveTilesMaxN = 1ull << 19;

// Whether the block sort of an n-key regular sort uses multi-wave group tiles.
bool sort_uses_groups(uint64_t n, const Tuning &tu)
{
    return tu.block_sort >= 3 || (tu.block_sort == 0 && n > kAutoWaveTilesMaxN);
}

// Length of the sorted runs the block sort of an n-key regular sort produces.
uint64_t sort_run_keys(bool pairs, uint64_t n, const Tuning &tu)
{
    return sort_uses_groups(n, tu) ? group_run_keys(pairs) : (uint64_t)kTile;
}

// Fan-in of every merge pass of an n-key regular sort, first pass first:
// four-way passes while more than two runs remain (keys or key/value pairs;
// their work split is searched from key samples), then at most one binary
// pass.
std::vector<uint32_t> sort_fan_ins(bool pairs, uint64_t n, const Tuning &tu)
{
    std::vector<uint32_t> fi;
    if (n == 0)
        return fi;
    const uint64_t run0 = sort_run_keys(pairs, n, tu);
    const bool want4 = tu.merge_fan_in == 4 || (tu.merge_fan_in == 0 && (pairs || n >= kAutoFourWayMinKeys));
    const bool four = want4 && tu.sampled_partition;
    for (uint64_t runs = (n + run0 - 1) / run0; runs > 1;) {
        const uint32_t k = (four && runs > 2) ? 4 : 2;
        fi.push_back(k);
        runs = (runs + k - 1) / k;
    }
    return fi;
}

// kind 0: u32 keys; 1 int32, 2 float: keys are mapped in order to u32 as the
// block sort loads them and mapped back as the last pass stores them.
bcf_status sort_impl(bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                     uint64_t n, void *temp, uint64_t *temp_bytes, hipStream_t s, int kind = 0)
{
    if (!temp_bytes || n > kMaxN)
        return BCF_ERR_INVALID;
    const uint64_t tiles = tiles_of(n);
    const Tuning tu = tuning();
    const uint64_t run0 = sort_run_keys(pairs, n, tu);  // sorted run length after the block sort
    const std::vector<uint32_t> fan_in = sort_fan_ins(pairs, n, tu);
    const uint32_t passes = (uint32_t)fan_in.size();
    // temp: ping-pong keys [, values], one split per merge tile, two sets of
    // key samples (each pass reads one set and writes the other), then (keys)
    // the cut list of a four-way pass.  The layout does not depend on the
    // tuning, so a size queried before a tuning change stays valid.
    const uint64_t data = align256(n * 4) * (pairs ? 2 : 1);
    const uint64_t blocks64 = (n + kLine - 1) / kLine;
    const uint64_t set_bytes = 2 * align256(blocks64 * 4) + 2 * align256(tiles * 4);
    const uint64_t cut_bytes = align256(merge4_cut_bytes_max(n));
    const uint64_t need = passes ? data + align256(tiles * 4) + 2 * set_bytes + cut_bytes : 0;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (n == 0)
        return BCF_OK;
    if (!kin || !kout || (pairs && (!vin || !vout)))
        return BCF_ERR_INVALID;
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    uint32_t *kt = static_cast<uint32_t *>(temp);
    uint32_t *vt = pairs ? reinterpret_cast<uint32_t *>(static_cast<char *>(temp) + align256(n * 4)) : nullptr;
    uint32_t *splits = reinterpret_cast<uint32_t *>(static_cast<char *>(temp) + data);
    const bool tile_samples = tu.tile_samples;
    auto sample_set = [&](uint32_t k) {
        char *b = static_cast<char *>(temp) + data + align256(tiles * 4) + k * set_bytes;
        SampleSet ss;
        ss.f = reinterpret_cast<uint32_t *>(b);
        ss.l = reinterpret_cast<uint32_t *>(b + align256(blocks64 * 4));
        ss.cf = reinterpret_cast<uint32_t *>(b + 2 * align256(blocks64 * 4));
        ss.cl = reinterpret_cast<uint32_t *>(b + 2 * align256(blocks64 * 4) + align256(tiles * 4));
        if (!tile_samples)
            ss.cf = ss.cl = nullptr;
        return ss;
    };
    const SampleSet none{nullptr, nullptr, nullptr, nullptr};
    const bool sampled = tu.sampled_partition;  // searches start from samples
    // X_j = buffer after pass j; X_passes = out.
    auto kbuf = [&](uint32_t j) { return ((passes - j) % 2 == 0) ? kout : kt; };
    auto vbuf = [&](uint32_t j) { return ((passes - j) % 2 == 0) ? vout : vt; };
    const double elem_bytes = pairs ? 8.0 : 4.0;
    const KeyMap fwd = key_map(kind, false), inv = key_map(kind, true);
    // the pass that writes the output stores through the inverse map
    auto out_map = [&](uint32_t j) { return j == passes ? inv : KeyMap{}; };
    {
        ProfScope p(kname_block_sort(pairs, false), s, 2.0 * elem_bytes * n);
        const SampleSet smp = (passes && sampled) ? sample_set(0) : none;
        if (sort_uses_groups(n, tu) && tu.block_sort == 4 && !pairs && kind == 0)
            BCF_TRY(dev_status(launch_block_sort_shear_group(kin, kbuf(0), n, smp, s)));
        else if (sort_uses_groups(n, tu))
            BCF_TRY(dev_status(launch_block_sort_group(pairs, kin, vin, kbuf(0), pairs ? vbuf(0) : nullptr, n, smp, s,
                                                       fwd, out_map(0))));
        else
            BCF_TRY(dev_status(launch_block_sort_regular(pairs, tu.block_sort == 2, kin, vin, kbuf(0),
                                                         pairs ? vbuf(0) : nullptr, n, smp, s, fwd, out_map(0))));
    }
    void *cuts = static_cast<char *>(temp) + data + align256(tiles * 4) + 2 * set_bytes;
    uint64_t run = run0;
    for (uint32_t j = 1; j <= passes; run *= fan_in[j - 1], ++j) {
        if (fan_in[j - 1] == 4) {
            const SampleSet in_smp = sample_set((j - 1) & 1);
            const SampleSet out_smp = j < passes ? sample_set(j & 1) : none;
            for (int phase = 0; phase < 2; ++phase) {
                const bool cut = phase == 0;
                ProfScope p(cut ? (pairs ? "cuts4_pairs" : "cuts4_keys") : (pairs ? "merge4_pairs" : "merge4_keys"), s,
                            cut ? 0.0 : 2.0 * elem_bytes * n);
                BCF_TRY(dev_status(launch_merge4_regular(kbuf(j - 1), kbuf(j), n, run, cuts, in_smp, out_smp, cut,
                                                         s, out_map(j), pairs ? vbuf(j - 1) : nullptr,
                                                         pairs ? vbuf(j) : nullptr)));
            }
            continue;
        }
        // decided once per pass from this call's tuning snapshot: both launches agree
        const bool fused = merge_fuses_partition(pairs, sampled ? sample_set((j - 1) & 1) : none, tu);
        for (int phase = 0; phase < 2; ++phase) {
            const bool part = phase == 0;
            if (part && fused)
                continue;  // the merge launch searches its own splits
            ProfScope p(part ? kname_partition(pairs, false) : kname_merge(pairs, false), s,
                        part ? 0.0 : 2.0 * elem_bytes * n);
            const SampleSet in_smp = sampled ? sample_set((j - 1) & 1) : none;
            const SampleSet out_smp = (sampled && j < passes) ? sample_set(j & 1) : none;
            BCF_TRY(dev_status(launch_merge_regular(pairs, kbuf(j - 1), pairs ? vbuf(j - 1) : nullptr, kbuf(j),
                                                    pairs ? vbuf(j) : nullptr, n, run, splits, in_smp, out_smp,
                                                    part, fused, s, out_map(j))));
        }
    }
    return BCF_OK;
}

// ---------------------------------------------------- other key types

// Sort of int32 (kind 1) or float (kind 2) keys: the u32 sort with the
// order-preserving key map fused into its first and last pass (no extra pass
// over the keys).  The temp size is that of the u32 sort.
bcf_status sort_typed(int kind, bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                      uint32_t *vout, uint64_t n, void *temp, uint64_t *temp_bytes, hipStream_t s)
{
    if (kind != 1 && kind != 2)
        return BCF_ERR_INVALID;
    return sort_impl(pairs, kin, vin, kout, vout, n, temp, temp_bytes, s, kind);
}

// ---------------------------------------------------- table-driven plans

struct MergePass {
    std::vector<MergeJob> jobs;
    std::vector<uint32_t> tile_job;
    // fan-in 4 merges: the jobs, and the totals of their cut
    // searches, item slots and cut records (the maps from searches and slots
    // to jobs, and the records, are written on the device)
    std::vector<Merge4Job> jobs4;
    uint32_t tasks4 = 0, items4 = 0, records4 = 0;
    uint64_t keys4 = 0;  // keys the fan-in 4 jobs merge
};

// Add one fan-in 4 job: runs of n[0..3] keys back to back from `start`.
void add_job4(MergePass &mp, uint64_t start, const uint64_t (&n)[4], uint32_t src, uint32_t dst)
{
    const uint64_t tot = n[0] + n[1] + n[2] + n[3];
    if (tot == 0)
        return;
    Merge4Job j;
    j.start = start;
    for (int r = 0; r < 4; ++r)
        j.n[r] = (uint32_t)n[r];
    const uint32_t J = merge4_ab_segments(n[0] + n[1]), M = merge4_cd_cuts(n[2] + n[3]);
    j.cut_off = mp.records4;
    j.item_off = mp.items4;
    j.task_off = mp.tasks4;
    j.src = (uint16_t)src;
    j.dst = (uint16_t)dst;
    mp.jobs4.push_back(j);
    // searches: AB cuts 1..J-1 and CD cuts 1..M, at least one (the first
    // writes the records P[0] and P[J]); records P[0..J] and Q[0..M]
    mp.tasks4 += merge4_tasks(J, M);
    mp.items4 += merge4_items(J, M);
    mp.records4 += merge4_records(J, M);
    mp.keys4 += tot;
}

// Add one binary merge job A=[a, a+na), B=[a+na, a+na+nb) to a pass.
void add_job(MergePass &mp, uint64_t a, uint64_t na, uint64_t nb, uint32_t src, uint32_t dst)
{
    const uint64_t tot = na + nb;
    if (tot == 0)
        return;
    MergeJob j;
    j.a_start = a;
    j.na = (uint32_t)na;
    j.nb = (uint32_t)nb;
    j.first_tile = (uint32_t)mp.tile_job.size();
    j.src = (uint16_t)src;
    j.dst = (uint16_t)dst;
    const uint32_t id = (uint32_t)mp.jobs.size();
    mp.jobs.push_back(j);
    for (uint64_t t = 0; t < tiles_of(tot); ++t)
        mp.tile_job.push_back(id);
}

// Device layout of the descriptor tables inside temp, after the data buffers.
struct TableLayout {
    uint64_t block_off = 0, block_bytes = 0;    // single-wave tiles
    uint64_t group_off = 0, group_bytes = 0;    // multi-wave group tiles
    std::vector<uint64_t> jobs_off, map_off;
    std::vector<uint64_t> jobs4_off, task_off, item_off, cuts4_off;  // fan-in 4 tables of each pass
    uint64_t splits_off = 0;  // one u32 per tile of the largest pass (reused by every pass)
    uint64_t total = 0;
};

TableLayout layout_tables(uint64_t base, size_t nblock, size_t ngroup, const std::vector<MergePass> &passes)
{
    TableLayout L;
    uint64_t o = base;
    L.block_off = o;
    L.block_bytes = nblock * sizeof(BlockTile);
    o = align256(o + L.block_bytes);
    L.group_off = o;
    L.group_bytes = ngroup * sizeof(BlockTile);
    o = align256(o + L.group_bytes);
    size_t max_tiles = 0;
    for (const auto &mp : passes) {
        L.jobs_off.push_back(o);
        o = align256(o + mp.jobs.size() * sizeof(MergeJob));
        L.map_off.push_back(o);
        o = align256(o + mp.tile_job.size() * sizeof(uint32_t));
        max_tiles = std::max(max_tiles, mp.tile_job.size());
        L.jobs4_off.push_back(o);
        o = align256(o + mp.jobs4.size() * sizeof(Merge4Job));
        L.task_off.push_back(o);
        o = align256(o + (uint64_t)mp.tasks4 * sizeof(uint32_t));
        L.item_off.push_back(o);
        o = align256(o + (uint64_t)mp.items4 * sizeof(uint32_t));
        L.cuts4_off.push_back(o);
        o = align256(o + (uint64_t)mp.records4 * 4 * sizeof(uint32_t));
    }
    L.splits_off = o;
    o = align256(o + max_tiles * sizeof(uint32_t));
    L.total = o;
    return L;
}

// A host-planned launch sequence: block-sort tiles, then merge passes.
struct TablePlan {
    std::vector<BlockTile> single, group;
    std::vector<MergePass> passes;
    TableLayout L;
    bool pairs = false;
};

// Pack every table into one host image and upload it with one copy.
bcf_status upload_tables(char *temp, const TablePlan &P, hipStream_t s)
{
    const TableLayout &L = P.L;
    const uint64_t lo = L.block_off;
    const uint64_t bytes = L.splits_off - lo;  // the splits area is written on the device
    if (bytes == 0)
        return BCF_OK;
    std::vector<char> img(bytes, 0);
    if (!P.single.empty())
        std::memcpy(img.data() + (L.block_off - lo), P.single.data(), L.block_bytes);
    if (!P.group.empty())
        std::memcpy(img.data() + (L.group_off - lo), P.group.data(), L.group_bytes);
    for (size_t p = 0; p < P.passes.size(); ++p) {
        if (!P.passes[p].jobs.empty())
            std::memcpy(img.data() + (L.jobs_off[p] - lo), P.passes[p].jobs.data(),
                        P.passes[p].jobs.size() * sizeof(MergeJob));
        if (!P.passes[p].tile_job.empty())
            std::memcpy(img.data() + (L.map_off[p] - lo), P.passes[p].tile_job.data(),
                        P.passes[p].tile_job.size() * sizeof(uint32_t));
        const MergePass &mp = P.passes[p];
        if (!mp.jobs4.empty())
            std::memcpy(img.data() + (L.jobs4_off[p] - lo), mp.jobs4.data(), mp.jobs4.size() * sizeof(Merge4Job));
    }
    return upload(temp + lo, img.data(), bytes, s);
}

// Enqueue the kernels of a plan whose tables are already in temp.
bcf_status launch_tables(Bufs kb, Bufs vb, char *temp, const TablePlan &P, hipStream_t s)
{
    const bool pairs = P.pairs;
    const TableLayout &L = P.L;
    const double eb = pairs ? 8.0 : 4.0;
    if (!P.single.empty()) {
        double moved = 0;
        for (const auto &b : P.single)
            moved += 2.0 * eb * b.count;
        ProfScope p(kname_block_sort(pairs, true), s, moved);
        BCF_TRY(dev_status(launch_block_sort_table(pairs, kb, vb, reinterpret_cast<const BlockTile *>(temp + L.block_off),
                                                   (uint32_t)P.single.size(), s)));
    }
    if (!P.group.empty()) {
        double moved = 0;
        for (const auto &b : P.group)
            moved += 2.0 * eb * b.count;
        ProfScope p(kname_block_sort(pairs, true), s, moved);
        BCF_TRY(dev_status(launch_block_sort_group_table(
            pairs, kb, vb, reinterpret_cast<const BlockTile *>(temp + L.group_off), (uint32_t)P.group.size(), s)));
    }
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const auto &mp = P.passes[p];
        if (!mp.jobs4.empty()) {
            // the fan-in 4 merges of this pass (other segments than its binary
            // jobs): maps, cut searches, merges
            for (int phase = 0; phase < 3; ++phase) {
                static const char *const names[2][3] = {{"map4_keys_table", "cuts4_keys_table", "merge4_keys_table"},
                                                        {"map4_pairs_table", "cuts4_pairs_table", "merge4_pairs_table"}};
                ProfScope ps(names[pairs][phase], s, phase == 2 ? 2.0 * eb * mp.keys4 : 0.0);
                BCF_TRY(dev_status(launch_merge4_table(
                    kb, reinterpret_cast<const Merge4Job *>(temp + L.jobs4_off[p]), (uint32_t)mp.jobs4.size(),
                    reinterpret_cast<uint32_t *>(temp + L.task_off[p]), mp.tasks4,
                    reinterpret_cast<uint32_t *>(temp + L.item_off[p]), mp.items4, temp + L.cuts4_off[p], mp.keys4,
                    phase, s, nullptr, pairs ? vb : Bufs{nullptr, nullptr, nullptr})));
            }
        }
        if (mp.tile_job.empty())
            continue;
        double moved = 0;
        for (const auto &j : mp.jobs)
            moved += 2.0 * eb * (double(j.na) + j.nb);
        for (int phase = 0; phase < 2; ++phase) {
            const bool part = phase == 0;
            ProfScope ps(part ? kname_partition(pairs, true) : kname_merge(pairs, true), s, part ? 0.0 : moved);
            BCF_TRY(dev_status(launch_merge_table(pairs, kb, vb, reinterpret_cast<const MergeJob *>(temp + L.jobs_off[p]),
                                                  reinterpret_cast<const uint32_t *>(temp + L.map_off[p]),
                                                  (uint32_t)mp.tile_job.size(),
                                                  reinterpret_cast<uint32_t *>(temp + L.splits_off), part, s)));
        }
    }
    return BCF_OK;
}

// Segments at least this long are block-sorted in multi-wave group tiles
// (fewer merge passes); shorter ones in 4096-key wave tiles.  `knob` is the
// tuning's group_min_keys (0: the library default).
uint64_t group_min_keys(bool pairs, uint64_t knob)
{
    return knob ? knob : group_run_keys(pairs) / 2;
}

// Plans uploaded by bcf_segmented_upload, by temp buffer: a fingerprint of the
// offsets and flags, and the tuning the plan was made under.  The execute call
// replans on the host with that same tuning (never the tuning current at
// execute time) and refuses offsets that differ from the uploaded ones.
struct UploadedPlan {
    uint64_t fingerprint;
    uint64_t group_min_keys;
    int merge_fan_in;
};
std::mutex g_plans_mu;
std::map<const void *, UploadedPlan> g_plans;

uint64_t plan_fingerprint(const uint64_t *off, uint32_t nseg, bool pairs)
{
    uint64_t h = 0xcbf29ce484222325ull ^ (pairs ? 0x9e37u : 0u);  // FNV-1a over the offsets
    auto mix = [&h](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 0x100000001b3ull;
        }
    };
    mix(nseg);
    for (uint32_t i = 0; i <= nseg; ++i)
        mix(off[i]);
    return h;
}

// Plan of a segmented sort: every segment is block-sorted into runs that
// never cross its boundaries, then merged pairwise until one run remains.
// X_j(s), the buffer holding segment s after its pass j, alternates so that
// its last pass lands in the output.
// Merge steps of a segment of `runs` sorted runs: fan-in 4 while more than
// two runs remain (when `four`), then binary steps until one run is left.
std::vector<uint8_t> seg_fan_ins(uint64_t runs, bool four)
{
    std::vector<uint8_t> fi;
    while (runs > 1) {
        const uint8_t k = (four && runs > 2) ? 4 : 2;
        fi.push_back(k);
        runs = (runs + k - 1) / k;
    }
    return fi;
}

// Whether the merges of a segmented sort of n keys (or pairs) use fan-in 4
// steps under the tuning knob merge_fan_in (0: from 2^25 keys, where a pass
// streams more than the last-level cache holds).
bool seg_four_way(bool pairs, uint64_t n, int fan_in_knob)
{
    (void)pairs;
    return fan_in_knob == 4 || (fan_in_knob == 0 && n >= kAutoFourWayMinN);
}

bcf_status plan_segmented(const uint64_t *off, uint32_t nseg, bool pairs, uint64_t gmin_knob, int fan_in_knob,
                          TablePlan &P)
{
    P.pairs = pairs;
    const uint64_t n = off[nseg];
    const uint64_t gmin = group_min_keys(pairs, gmin_knob);
    const uint64_t grun = group_run_keys(pairs);
    const bool four = seg_four_way(pairs, n, fan_in_knob);
    std::vector<uint32_t> ps(nseg, 0);
    std::vector<uint64_t> run0(nseg, kTile);
    std::vector<std::vector<uint8_t>> fan(nseg);
    uint32_t pmax = 0;
    for (uint32_t sg = 0; sg < nseg; ++sg) {
        const uint64_t len = off[sg + 1] - off[sg];
        if (len == 0)
            continue;
        if (len > (uint64_t)kTile && len >= gmin)
            run0[sg] = grun;
        fan[sg] = seg_fan_ins((len + run0[sg] - 1) / run0[sg], four);
        ps[sg] = (uint32_t)fan[sg].size();
        pmax = std::max(pmax, ps[sg]);
    }
    auto bufsel = [&](uint32_t sg, uint32_t j) -> uint32_t { return ((ps[sg] - j) % 2 == 0) ? kBufOut : kBufTemp; };
    for (uint32_t sg = 0; sg < nseg; ++sg) {
        const uint64_t a = off[sg], len = off[sg + 1] - a;
        const uint64_t r0 = run0[sg];
        auto &dst = r0 == (uint64_t)kTile ? P.single : P.group;
        for (uint64_t o = 0; o < len; o += r0) {
            BlockTile b;
            b.start = a + o;
            b.count = (uint32_t)std::min<uint64_t>(r0, len - o);
            b.dst = bufsel(sg, 0);
            dst.push_back(b);
        }
    }
    P.passes.assign(pmax, MergePass{});
    std::vector<uint64_t> run(run0);  // run length of each segment before its next step
    for (uint32_t j = 1; j <= pmax; ++j) {
        for (uint32_t sg = 0; sg < nseg; ++sg) {
            if (ps[sg] < j)
                continue;
            const uint64_t L = run[sg];
            const uint64_t a = off[sg], len = off[sg + 1] - a;
            const uint32_t k = fan[sg][j - 1];
            if (k == 4) {
                for (uint64_t o = 0; o < len; o += 4 * L) {
                    uint64_t nr[4];
                    for (int r = 0; r < 4; ++r) {
                        const uint64_t s0 = o + r * L;
                        nr[r] = s0 < len ? std::min(L, len - s0) : 0;
                    }
                    add_job4(P.passes[j - 1], a + o, nr, bufsel(sg, j - 1), bufsel(sg, j));
                }
            } else {
                for (uint64_t o = 0; o < len; o += 2 * L) {
                    const uint64_t na = std::min(L, len - o);
                    const uint64_t nb = std::min(L, len - o - na);
                    add_job(P.passes[j - 1], a + o, na, nb, bufsel(sg, j - 1), bufsel(sg, j));
                }
            }
            run[sg] = L * k;
        }
    }
    const uint64_t data = pmax ? align256(n * 4) * (pairs ? 2 : 1) : 0;
    P.L = layout_tables(data, P.single.size(), P.group.size(), P.passes);
    return BCF_OK;
}

enum SegMode { kSegFull, kSegUpload, kSegExecute };

bcf_status segmented_impl(SegMode mode, bool pairs, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                          uint32_t *vout, const uint64_t *off, uint32_t nseg, void *temp, uint64_t *temp_bytes,
                          hipStream_t s)
{
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    if (nseg == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    if (!offsets_valid(off, nseg))
        return BCF_ERR_INVALID;
    const Tuning tu = tuning();
    uint64_t gmin = tu.group_min_keys;
    int fan_in = tu.merge_fan_in;
    if (mode == kSegExecute && temp && off[nseg] != 0) {
        // the tuning of the upload into this temp buffer, for the same offsets
        std::lock_guard<std::mutex> g(g_plans_mu);
        auto it = g_plans.find(temp);
        if (it == g_plans.end() || it->second.fingerprint != plan_fingerprint(off, nseg, pairs))
            return BCF_ERR_INVALID;
        gmin = it->second.group_min_keys;
        fan_in = it->second.merge_fan_in;
    }
    TablePlan P;
    BCF_TRY(plan_segmented(off, nseg, pairs, gmin, fan_in, P));
    const uint64_t n = off[nseg];
    if (!temp) {
        *temp_bytes = P.L.total;
        return BCF_OK;
    }
    if (n == 0)
        return BCF_OK;
    if (*temp_bytes < P.L.total)
        return BCF_ERR_TEMP_TOO_SMALL;
    char *tb = static_cast<char *>(temp);
    if (mode != kSegExecute)
        BCF_TRY(upload_tables(tb, P, s));
    if (mode == kSegUpload) {
        std::lock_guard<std::mutex> g(g_plans_mu);
        g_plans[temp] = UploadedPlan{plan_fingerprint(off, nseg, pairs), gmin, fan_in};
        return BCF_OK;
    }
    if (!kin || !kout || (pairs && (!vin || !vout)))
        return BCF_ERR_INVALID;
    Bufs kb{kin, kout, reinterpret_cast<uint32_t *>(tb)};
    Bufs vb{nullptr, nullptr, nullptr};
    if (pairs)
        vb = Bufs{vin, vout, reinterpret_cast<uint32_t *>(tb + align256(n * 4))};
    return launch_tables(kb, vb, tb, P, s);
}

}  // namespace

namespace bcf {
Tuning tuning()
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    return tuning_locked();
}

// Host services for the other translation units of the library (the
// distribution step): descriptor upload through the pinned staging buffers,
// and a profiling scope around one launch (recorded only while profiling is on).
bcf_status upload_host(void *dst, const void *src, size_t bytes, hipStream_t s) { return upload(dst, src, bytes, s); }
void *prof_begin(const char *name, hipStream_t s, double bytes) { return new ProfScope(name, s, bytes); }
ProfilingOff::ProfilingOff() { ++t_prof_off; }
ProfilingOff::~ProfilingOff() { --t_prof_off; }
void prof_end(void *scope) { delete static_cast<ProfScope *>(scope); }
}  // namespace bcf

// ======================================================================= ABI

extern "C" {

const char *bcf_status_string(bcf_status s)
{
    switch (s) {
    case BCF_OK: return "BCF_OK";
    case BCF_ERR_INVALID: return "BCF_ERR_INVALID: invalid argument";
    case BCF_ERR_TEMP_TOO_SMALL: return "BCF_ERR_TEMP_TOO_SMALL: temp buffer smaller than required";
    case BCF_ERR_NOMEM: return "BCF_ERR_NOMEM: host staging allocation failed";
    case BCF_ERR_DEVICE: return "BCF_ERR_DEVICE: HIP runtime or launch failure";
    case BCF_ERR_UNSORTED_RUN: return "BCF_ERR_UNSORTED_RUN: an input run is not sorted";
    }
    return "BCF_ERR_UNKNOWN";
}

uint32_t bcf_tile_keys(void) { return (uint32_t)kTile; }

uint32_t bcf_run_keys(int pairs) { return sort_run_keys(pairs != 0, ~0ull, tuning()); }

uint32_t bcf_sort_passes(uint64_t n, int pairs)
{
    if (n == 0)
        return 0;
    return 1 + (uint32_t)sort_fan_ins(pairs != 0, n, tuning()).size();
}

bcf_status bcf_sort_u32(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, void *temp,
                        uint64_t *temp_bytes, void *stream)
{
    return sort_impl(false, keys_in, nullptr, keys_out, nullptr, n, temp, temp_bytes,
                     static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_pairs_u32(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                              uint32_t *vals_out, uint64_t n, void *temp, uint64_t *temp_bytes, void *stream)
{
    return sort_impl(true, keys_in, vals_in, keys_out, vals_out, n, temp, temp_bytes,
                     static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_i32(const int32_t *keys_in, int32_t *keys_out, uint64_t n, void *temp, uint64_t *temp_bytes,
                        void *stream)
{
    return sort_typed(1, false, reinterpret_cast<const uint32_t *>(keys_in), nullptr,
                      reinterpret_cast<uint32_t *>(keys_out), nullptr, n, temp, temp_bytes,
                      static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_f32(const float *keys_in, float *keys_out, uint64_t n, void *temp, uint64_t *temp_bytes,
                        void *stream)
{
    return sort_typed(2, false, reinterpret_cast<const uint32_t *>(keys_in), nullptr,
                      reinterpret_cast<uint32_t *>(keys_out), nullptr, n, temp, temp_bytes,
                      static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_pairs_i32(const int32_t *keys_in, const uint32_t *vals_in, int32_t *keys_out, uint32_t *vals_out,
                              uint64_t n, void *temp, uint64_t *temp_bytes, void *stream)
{
    return sort_typed(1, true, reinterpret_cast<const uint32_t *>(keys_in), vals_in,
                      reinterpret_cast<uint32_t *>(keys_out), vals_out, n, temp, temp_bytes,
                      static_cast<hipStream_t>(stream));
}

bcf_status bcf_sort_pairs_f32(const float *keys_in, const uint32_t *vals_in, float *keys_out, uint32_t *vals_out,
                              uint64_t n, void *temp, uint64_t *temp_bytes, void *stream)
{
    return sort_typed(2, true, reinterpret_cast<const uint32_t *>(keys_in), vals_in,
                      reinterpret_cast<uint32_t *>(keys_out), vals_out, n, temp, temp_bytes,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Stable merge of groups of consecutive sorted runs, each group on its own:
// group g is runs [group_starts[g], group_starts[g+1]) (one group of all k runs
// when group_starts is NULL).  Every group takes its own number of binary
// passes, ceil(log2(its nonempty runs)), with its own buffer parity so that its
// last pass lands in the output: a group of one run is copied once (not at
// all when merging in place), and a group that finishes early is not read and
// written again by the passes other groups still need.
bcf_status merge_groups_impl(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                             uint32_t k, const uint32_t *group_starts, uint32_t ngroups, uint32_t *keys_out,
                             uint32_t *vals_out, void *temp, uint64_t *temp_bytes, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    if (k == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    if (!offsets_valid(run_offsets, k))
        return BCF_ERR_INVALID;
    if (group_starts) {
        if (ngroups == 0 || group_starts[0] != 0 || group_starts[ngroups] != k)
            return BCF_ERR_INVALID;
        for (uint32_t g = 0; g < ngroups; ++g)
            if (group_starts[g + 1] < group_starts[g])
                return BCF_ERR_INVALID;
    }
    const uint32_t ng = group_starts ? ngroups : 1;
    const bool pairs = vals_in != nullptr;
    const uint64_t n = run_offsets[k];
    // In place (keys or values), a group whose pass count is odd would make its
    // first pass read and write the same buffer; such a group takes one more
    // pass, a copy from temp into the output.
    const bool inplace = keys_in == keys_out || (pairs && vals_in == vals_out);
    // nonempty runs of every group, in order (empty runs change nothing,
    // stability included)
    std::vector<std::vector<std::pair<uint64_t, uint64_t>>> runs0(ng);
    for (uint32_t g = 0; g < ng; ++g) {
        const uint32_t r0 = group_starts ? group_starts[g] : 0, r1 = group_starts ? group_starts[g + 1] : k;
        for (uint32_t r = r0; r < r1; ++r)
            if (run_offsets[r + 1] > run_offsets[r])
                runs0[g].push_back({run_offsets[r], run_offsets[r + 1] - run_offsets[r]});
    }
    // The plan for in-place or separate buffers (worst: every extra copy pass
    // of either, so that the temp size does not depend on the pointers).
    auto plan = [&](bool in_place, bool worst, TablePlan &TP) {
        std::vector<std::vector<std::pair<uint64_t, uint64_t>>> cur = runs0;
        std::vector<uint32_t> gp(ng, 0);
        uint32_t P = 0;
        for (uint32_t g = 0; g < ng; ++g) {
            const uint32_t merges = cur[g].size() > 1 ? ceil_log2(cur[g].size()) : 0;
            if (cur[g].empty())
                gp[g] = 0;
            else if (merges == 0)
                gp[g] = (in_place && !worst) ? 0 : 1;  // one copy into the output
            else
                gp[g] = merges + ((merges % 2 == 1 && (in_place || worst)) ? 1 : 0);
            P = std::max(P, gp[g]);
        }
        std::vector<MergePass> passes(P);
        for (uint32_t g = 0; g < ng; ++g) {
            // buffer of group g after its pass j (j >= 1): its last pass lands in the output
            auto buf_after = [&](uint32_t j) -> uint32_t { return ((gp[g] - j) % 2 == 0) ? kBufOut : kBufTemp; };
            auto &runs = cur[g];
            for (uint32_t j = 1; j <= gp[g]; ++j) {
                const uint32_t src = j == 1 ? kBufIn : buf_after(j - 1);
                const uint32_t dst = buf_after(j);
                const bool copy = runs.size() == 1;  // one run left: this pass copies it
                std::vector<std::pair<uint64_t, uint64_t>> next;
                for (size_t i = 0; i < runs.size(); i += (copy ? 1 : 2)) {
                    const uint64_t a = runs[i].first, na = runs[i].second;
                    const uint64_t nb = (!copy && i + 1 < runs.size()) ? runs[i + 1].second : 0;
                    add_job(passes[j - 1], a, na, nb, src, dst);
                    next.push_back({a, na + nb});
                }
                runs.swap(next);
            }
        }
        const uint64_t data = align256(n * 4) * (pairs ? 2 : 1);
        TP.pairs = pairs;
        TP.passes = std::move(passes);
        TP.L = layout_tables(P ? data : 0, 0, 0, TP.passes);
    };
    TablePlan worst;
    plan(false, true, worst);
    // small area for the optional sortedness check: run offsets and a flag
    const uint64_t check_off = worst.L.total;
    const uint64_t need = check_off + align256((uint64_t(k) + 1) * sizeof(uint64_t)) + 256;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (n == 0)
        return BCF_OK;
    if (!keys_in || !keys_out || (pairs && !vals_out))
        return BCF_ERR_INVALID;
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    TablePlan TP;
    plan(inplace, false, TP);
    char *tb = static_cast<char *>(temp);
    uint32_t *kt = reinterpret_cast<uint32_t *>(tb);
    uint32_t *vt = pairs ? reinterpret_cast<uint32_t *>(tb + align256(n * 4)) : nullptr;

    if (tuning().check_runs) {
        // sortedness of every run (synchronises the stream)
        uint64_t *offs_d = reinterpret_cast<uint64_t *>(tb + check_off);
        uint32_t *flag_d =
            reinterpret_cast<uint32_t *>(tb + check_off + align256((uint64_t(k) + 1) * sizeof(uint64_t)));
        uint32_t flag = 0;
        BCF_TRY(upload(offs_d, run_offsets, (k + 1) * sizeof(uint64_t), s));
        if (hipMemsetAsync(flag_d, 0, sizeof(uint32_t), s) != hipSuccess ||
            launch_check_runs(keys_in, offs_d, k, n, flag_d, s) != hipSuccess ||
            hipMemcpyAsync(&flag, flag_d, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return BCF_ERR_DEVICE;
        if (flag)
            return BCF_ERR_UNSORTED_RUN;
    }

    if (TP.passes.empty())
        return BCF_OK;  // merged in place: every group is already one run
    Bufs kb{keys_in, keys_out, kt};
    Bufs vb{vals_in, vals_out, vt};
    BCF_TRY(upload_tables(tb, TP, s));
    return launch_tables(kb, vb, tb, TP, s);
}

}  // namespace

extern "C" {

bcf_status bcf_merge_runs_host(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                          uint32_t k, uint32_t *keys_out, uint32_t *vals_out, void *temp, uint64_t *temp_bytes,
                          void *stream)
{
    return merge_groups_impl(keys_in, vals_in, run_offsets, k, nullptr, 0, keys_out, vals_out, temp, temp_bytes,
                             stream);
}

bcf_status bcf_merge_run_groups(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                                uint32_t k, const uint32_t *group_starts, uint32_t ngroups, uint32_t *keys_out,
                                uint32_t *vals_out, void *temp, uint64_t *temp_bytes, void *stream)
{
    if (!group_starts)
        return BCF_ERR_INVALID;
    return merge_groups_impl(keys_in, vals_in, run_offsets, k, group_starts, ngroups, keys_out, vals_out, temp,
                             temp_bytes, stream);
}

bcf_status bcf_segmented_sort_host(const uint32_t *keys_in, uint32_t *keys_out, const uint64_t *seg_offsets,
                              uint32_t nseg, void *temp, uint64_t *temp_bytes, void *stream)
{
    return segmented_impl(kSegFull, false, keys_in, nullptr, keys_out, nullptr, seg_offsets, nseg, temp, temp_bytes,
                          static_cast<hipStream_t>(stream));
}

bcf_status bcf_segmented_sort_pairs_host(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                    uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg, void *temp,
                                    uint64_t *temp_bytes, void *stream)
{
    return segmented_impl(kSegFull, true, keys_in, vals_in, keys_out, vals_out, seg_offsets, nseg, temp, temp_bytes,
                          static_cast<hipStream_t>(stream));
}

bcf_status bcf_segmented_upload(const uint64_t *seg_offsets, uint32_t nseg, int pairs, void *temp,
                                uint64_t *temp_bytes, void *stream)
{
    return segmented_impl(kSegUpload, pairs != 0, nullptr, nullptr, nullptr, nullptr, seg_offsets, nseg, temp,
                          temp_bytes, static_cast<hipStream_t>(stream));
}

bcf_status bcf_segmented_execute(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                 uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg, void *temp,
                                 uint64_t *temp_bytes, void *stream)
{
    return segmented_impl(kSegExecute, vals_in != nullptr, keys_in, vals_in, keys_out, vals_out, seg_offsets, nseg,
                          temp, temp_bytes, static_cast<hipStream_t>(stream));
}

void bcf_get_tuning(bcf_tuning *out)
{
    if (!out)
        return;
    std::lock_guard<std::mutex> g(g_tune_mu);
    const Tuning &t = tuning_locked();
    out->merge_variant = t.merge_variant;
    out->nontemporal = t.nontemporal;
    out->sampled_partition = t.sampled_partition;
    out->tile_samples = t.tile_samples;
    out->group_min_keys = t.group_min_keys;
    out->check_runs = t.check_runs;
    out->block_sort = t.block_sort;
    out->fused_partition = t.fused_partition;
    out->merge_fan_in = t.merge_fan_in;
}

bcf_status bcf_set_tuning(const bcf_tuning *in)
{
    if (!in || in->merge_variant < 0 || in->merge_variant > 3 || in->block_sort < 0 || in->block_sort > 4 ||
        (in->merge_fan_in != 0 && in->merge_fan_in != 2 && in->merge_fan_in != 4))
        return BCF_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_tune_mu);
    Tuning &t = tuning_locked();
    t.merge_variant = in->merge_variant;
    t.nontemporal = in->nontemporal != 0;
    t.sampled_partition = in->sampled_partition != 0;
    t.tile_samples = in->tile_samples != 0;
    t.group_min_keys = in->group_min_keys;
    t.check_runs = in->check_runs != 0;
    t.block_sort = in->block_sort;
    t.fused_partition = in->fused_partition != 0;
    t.merge_fan_in = in->merge_fan_in;
    return BCF_OK;
}

void bcf_profile_enable(int on)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
}

int bcf_profile_collect(bcf_kernel_stat *out, int max)
{
    std::map<std::string, std::vector<ProfRec>> recs;
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        recs.swap(g_prof);
    }
    int n = 0;
    int rc = 0;
    for (auto &kv : recs) {
        double ms_sum = 0, bytes = 0;
        uint64_t launches = 0;
        for (auto &r : kv.second) {
            if (hipEventSynchronize(r.b) != hipSuccess)
                rc = -1;
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
                rc = -1;
            ms_sum += ms;
            bytes += r.bytes;
            ++launches;
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        if (out && n < max) {
            std::memset(&out[n], 0, sizeof(out[n]));
            std::snprintf(out[n].name, sizeof(out[n].name), "%s", kv.first.c_str());
            out[n].launches = launches;
            out[n].total_ms = ms_sum;
            out[n].bytes = bytes;
        }
        ++n;
    }
    return rc ? rc : std::min(n, max);
}

}  // extern "C"
