/*
 * bcf.h -- C ABI of the MI355X (gfx950) bank-conflict-free comparison sort.
 *
 * Operations follow the problem statements of Sitchinava & Weichert, "Bank
 * Conflict Free Comparison-based Sorting On GPUs": sort n keys ascending
 * (Sec. 3, base case plus merging phase), merge sorted sequences larger than
 * on-chip memory (Sec. 3.2, binary merging), extended to key/value pairs
 * (stable) and to many independent segments in one call.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Keys are uint32_t compared as unsigned integers; order is ascending
 *    (int32 and float keys: bcf_sort_i32 / bcf_sort_f32 and their pair forms).
 *  - Key/value arrays are device pointers (HBM) owned by the caller.  The
 *    offsets of bcf_merge_runs and bcf_segmented_sort[_pairs] are DEVICE
 *    pointers: their launch plans are computed on the device (see
 *    bcf_merge_runs).  The *_host variants, bcf_merge_run_groups,
 *    bcf_distribute_runs and bcf_segmented_upload / _execute take HOST offset
 *    arrays and plan on the host.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    call only enqueues work on that stream and returns; it never synchronises
 *    the device (except the temp queries of the calls with device offsets,
 *    which read the total from the device, and BCF_CHECK run checks).  Faults of earlier asynchronous work can surface as
 *    BCF_ERR_DEVICE on a later call.
 *  - Temporary storage: call once with temp == NULL to receive the number of
 *    bytes needed in *temp_bytes (nothing is launched, BCF_OK is returned);
 *    then pass a device buffer of at least that many bytes, 256-byte aligned,
 *    with *temp_bytes holding its size.  A smaller buffer yields
 *    BCF_ERR_TEMP_TOO_SMALL.  The library performs no device allocation.  The
 *    temp buffer must not be touched by other work until the call's kernels
 *    have finished (stream order guarantees this for same-stream users).
 *  - Inputs are never modified.  keys_out may equal keys_in (and vals_out may
 *    equal vals_in); any other overlap between inputs, outputs and temp is
 *    undefined.
 *  - n == 0 (or k == 0 / nseg == 0) is a no-op returning BCF_OK.  Sizes above
 *    2^32 - 1 elements return BCF_ERR_INVALID.
 *  - Offsets: off[0] == 0, nondecreasing, off[last] == total length.  Empty
 *    runs / segments are allowed.  Violations of host offsets return
 *    BCF_ERR_INVALID; device offsets are checked on the device (see
 *    bcf_merge_runs).
 *  - No C++ exception crosses this boundary.
 */
#ifndef BCF_H
#define BCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BCF_OK = 0,
    BCF_ERR_INVALID = 1,        /* bad argument: NULL pointer, size, offsets */
    BCF_ERR_TEMP_TOO_SMALL = 2, /* *temp_bytes smaller than required */
    BCF_ERR_NOMEM = 3,          /* host-side staging could not be allocated */
    BCF_ERR_DEVICE = 4,         /* a HIP runtime call or a kernel launch failed */
    BCF_ERR_UNSORTED_RUN = 5    /* merge_runs with BCF_CHECK=1: an input run is not sorted */
} bcf_status;

/*
 * Sort n keys ascending (the paper's BCFMergesort: base case of tile sorts in
 * LDS, Sec. 3.1, then binary merge passes over HBM, Sec. 3.2).
 *   keys_in   device, n u32, read only
 *   keys_out  device, n u32, receives the sorted keys (may equal keys_in)
 *   temp      device scratch (see conventions) or NULL to query *temp_bytes
 */
bcf_status bcf_sort_u32(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, void *temp,
                        uint64_t *temp_bytes, void *stream);

/*
 * bcf_sort_u32 for callers that cannot allocate device memory: code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation.
 * The temporary storage is a library-owned device array of 18 MiB per GPU
 * (each GPU the library runs on holds its own copy until the process ends),
 * so the call takes no temp argument and calls no allocating routine.
 *   keys_in, keys_out  device, n u32 each, as for bcf_sort_u32 (keys_out may
 *                      equal keys_in); the result is bcf_sort_u32's
 *   n                  at most BCF_NOALLOC_MAX_KEYS (else BCF_ERR_INVALID,
 *                      before anything is launched); n == 0 is a no-op
 *   stream             as for the other calls; its device must be the
 *                      current device
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads) race and give undefined results; calls
 * ordered on one stream are safe.  Nothing in the array needs to start at
 * zero.  No per-launch timing events are recorded for this call.
 */
#define BCF_NOALLOC_MAX_KEYS (1ull << 22)
bcf_status bcf_sort_u32_noalloc(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, void *stream);

/*
 * Stable sort of key/value pairs by key: equal keys keep their input order,
 * i.e. the result is ordered by (key, original index).  An extension of the
 * paper, whose data sets are keys only.
 *   keys_in, vals_in    device, n u32 each, read only
 *   keys_out, vals_out  device, n u32 each (may equal the inputs)
 */
bcf_status bcf_sort_pairs_u32(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                              uint32_t *vals_out, uint64_t n, void *temp, uint64_t *temp_bytes,
                              void *stream);

/*
 * Sorts of other 32-bit key types (an extension: the paper's keys are
 * unsigned 32-bit integers).  int32 keys ascend as signed integers; float
 * keys ascend in IEEE 754 totalOrder: -NaN < -inf < negative values < -0.0 <
 * +0.0 < positive values < +inf < +NaN (NaNs ordered by payload, negative ones
 * reversed), i.e. the order of the values with -0.0 before +0.0 and NaNs at
 * the ends by sign.  Keys are mapped to u32 by an order-preserving bit map
 * into keys_out, sorted there in place by bcf_sort_u32's path, and mapped
 * back: two more streaming passes over keys_out.  Same arguments, temp size
 * (bcf_sort_u32's / bcf_sort_pairs_u32's) and conventions as the u32 calls;
 * the pair variants are stable (equal keys keep their input order; for
 * floats, equal means the same bit pattern).
 */
bcf_status bcf_sort_i32(const int32_t *keys_in, int32_t *keys_out, uint64_t n, void *temp,
                        uint64_t *temp_bytes, void *stream);
bcf_status bcf_sort_f32(const float *keys_in, float *keys_out, uint64_t n, void *temp,
                        uint64_t *temp_bytes, void *stream);
bcf_status bcf_sort_pairs_i32(const int32_t *keys_in, const uint32_t *vals_in, int32_t *keys_out,
                              uint32_t *vals_out, uint64_t n, void *temp, uint64_t *temp_bytes,
                              void *stream);
bcf_status bcf_sort_pairs_f32(const float *keys_in, const uint32_t *vals_in, float *keys_out,
                              uint32_t *vals_out, uint64_t n, void *temp, uint64_t *temp_bytes,
                              void *stream);

/*
 * Sort of unsigned 64-bit keys (an extension: the paper's keys are 32-bit),
 * ascending, on the design of bcf_sort_u32 with a key held in a register pair
 * and compared as one 64-bit integer: the block sort of the paper's base case
 * (Sec. 3.1) into runs of 4096 keys, then binary merge passes (Sec. 3.2).
 *   keys_in, keys_out  device, n u64 each, 8-byte aligned (keys_out may equal keys_in)
 *   n                  at most 2^32 - 1 (else BCF_ERR_INVALID)
 *   temp               one array of n u64 (256-byte aligned size) when n > 4096,
 *                      none otherwise; query with temp == NULL as for the other sorts
 */
bcf_status bcf_sort_u64(const uint64_t *keys_in, uint64_t *keys_out, uint64_t n, void *temp,
                        uint64_t *temp_bytes, void *stream);

/*
 * Merge k sorted runs into one sorted sequence (the paper's binary merging of
 * sorted sequences larger than on-chip memory, Sec. 3.2, applied pairwise in
 * ceil(log2 k) passes).  Stable: among equal keys, lower run index first, then
 * earlier position.
 *   keys_in      device, run r occupies [run_offsets[r], run_offsets[r+1])
 *   vals_in      device values carried with the keys, or NULL for keys only
 *   run_offsets  DEVICE, k+1 entries (u64)
 *   keys_out     device, run_offsets[k] u32
 *   vals_out     device (ignored when vals_in is NULL)
 * The launch plan (every pass's merge jobs and tile map) is computed on the
 * device from run_offsets, so nothing is read back and the call can be
 * captured in a graph whose replays see new offsets.  Temp: the query
 * (temp == NULL) reads run_offsets[k] from the device (it synchronises the
 * stream) and returns the size for that many keys; at run time the size of
 * the buffer passed sets the capacity, the most keys the call merges with it
 * (run_offsets[k] may change between calls and replays within that).
 * Offsets that are not nondecreasing from 0, or whose total exceeds the
 * capacity, are found on the device: then nothing is written.
 * Every run must be sorted ascending (precondition).  With the tuning knob
 * check_runs set (environment BCF_CHECK=1) the library checks it and returns
 * BCF_ERR_UNSORTED_RUN (this check synchronises the stream).
 */
bcf_status bcf_merge_runs(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                          uint32_t k, uint32_t *keys_out, uint32_t *vals_out, void *temp,
                          uint64_t *temp_bytes, void *stream);

/* bcf_merge_runs with HOST offsets, planned on the host (the plan goes to the
 * device with one copy through pinned staging); empty runs are dropped from
 * the plan.  The temp size depends on the offsets, not only on their total. */
bcf_status bcf_merge_runs_host(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                               uint32_t k, uint32_t *keys_out, uint32_t *vals_out, void *temp,
                               uint64_t *temp_bytes, void *stream);

/*
 * Sort every segment [seg_offsets[s], seg_offsets[s+1]) of keys_in
 * independently (segments of up to 4096 keys in one wave tile, longer ones
 * block-sorted and then merged within the segment; all segments in one
 * block-sort launch per tile kind and one set of launches per merge level).
 * A segment's runs are merged four at a time while more than two remain
 * (bcf_tuning.merge_fan_in), then pairwise.
 *   seg_offsets  DEVICE, nseg+1 entries (u64)
 * Planned on the device, with the temp and capacity conventions of
 * bcf_merge_runs: the temp size does not depend on the tuning.
 */
bcf_status bcf_segmented_sort(const uint32_t *keys_in, uint32_t *keys_out, const uint64_t *seg_offsets,
                              uint32_t nseg, void *temp, uint64_t *temp_bytes, void *stream);

/*
 * Stable segmented sort of key/value pairs: every segment is sorted by key,
 * equal keys keeping their input order.  Same conventions as
 * bcf_segmented_sort, with values carried alongside the keys.
 */
bcf_status bcf_segmented_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                    uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg,
                                    void *temp, uint64_t *temp_bytes, void *stream);

/* The segmented sorts with HOST offsets, planned on the host. */
bcf_status bcf_segmented_sort_host(const uint32_t *keys_in, uint32_t *keys_out, const uint64_t *seg_offsets,
                                   uint32_t nseg, void *temp, uint64_t *temp_bytes, void *stream);
bcf_status bcf_segmented_sort_pairs_host(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                         uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg,
                                         void *temp, uint64_t *temp_bytes, void *stream);

/*
 * Sort by distribution: BCFMergesort with the distribution step of Sec. 3.2
 * and, with pivot_buckets, the pivot buckets of Sec. 3.3 (BCFMergesortPB).
 * Runs of run_keys keys are sorted (the segmented sort), distributed into P
 * buckets by P-1 splitters sampled from P candidates per run
 * (bcf_distribute_runs; 2P-1 buckets with pivot buckets), and every bucket's
 * pieces are merged on their own into keys_out, all buckets in the same
 * passes.  The piece offsets never leave the device: the bucket merge is
 * planned there (a pivot bucket, one key value, is copied as it is).
 *   keys_in, keys_out  device, n u32 each; keys_out must not equal keys_in
 *   n                  at most 2^32 - 1
 *   P                  1..65536; run_keys >= 1; the distribution's limits
 *                      apply (ceil(n / run_keys) runs at most 2^22, runs * P
 *                      at most 2^26, buckets * runs at most 2^24), else
 *                      BCF_ERR_INVALID
 *   temp               as for the sorts (the query needs no device access)
 */
bcf_status bcf_sort_u32_pb(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, uint32_t P, uint32_t run_keys,
                           int pivot_buckets, void *temp, uint64_t *temp_bytes, void *stream);

/*
 * The segmented sort split in two so that the device part can be captured in
 * a hipGraph and replayed.  bcf_segmented_upload plans the launches for
 * seg_offsets and copies the plan (tile and merge descriptors, a few bytes
 * per 4096 keys) into temp with one host-to-device copy on `stream`; keys are
 * not touched.  bcf_segmented_execute then only enqueues kernels that read the
 * plan from temp: it performs no copy and no allocation.  Both calls must get
 * the same seg_offsets, nseg, pairs flag (vals_in != NULL) and temp buffer,
 * and temp must keep the plan between them (and across graph replays).
 * Temp-size queries (temp == NULL) behave as in bcf_segmented_sort[_pairs].
 */
bcf_status bcf_segmented_upload(const uint64_t *seg_offsets, uint32_t nseg, int pairs, void *temp,
                                uint64_t *temp_bytes, void *stream);
bcf_status bcf_segmented_execute(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                                 uint32_t *vals_out, const uint64_t *seg_offsets, uint32_t nseg, void *temp,
                                 uint64_t *temp_bytes, void *stream);

/*
 * Colored prefix sums, the paper's demonstration that shared-memory bank
 * conflicts decide runtimes (Sec. 1.2 and its appendix): element i has a value
 * and a color below d; out[i] = the sum of values[j] over j <= i with
 * colors[j] == colors[i] (inclusive, modulo 2^32).  Colors at or above d count
 * as color d - 1.  Three phases (tile sums per color, their scan over the
 * tiles, scan of every tile page by page with per-thread, per-color counters
 * in LDS).  conflict_free = 0 keeps each thread's d counters consecutive in
 * LDS (the layout whose bank conflicts grow with d); 1 stores them
 * color-major, conflict-free for every d.  Results are identical.
 *   values, out  device, n u32 (out may equal values); colors device, n bytes;
 *                all three 16-byte aligned (else BCF_ERR_INVALID)
 *   d            1..32 (else BCF_ERR_INVALID)
 *   temp         as for the sorts (query with temp == NULL)
 */
bcf_status bcf_colored_prefix_sums(const uint32_t *values, const uint8_t *colors, uint32_t *out, uint64_t n,
                                   uint32_t d, int conflict_free, void *temp, uint64_t *temp_bytes,
                                   void *stream);

/*
 * Stable merge of groups of consecutive sorted runs, every group on its own
 * (the merge of Sec. 3.2 applied to many groups at once, e.g. the final merge
 * phase after a distribution, where each bucket's pieces are merged).  Group g
 * is runs [group_starts[g], group_starts[g+1]); its output occupies the same
 * key range as its runs and equals bcf_merge_runs of those runs.
 *   run_offsets   HOST, k+1 entries (conventions above)
 *   group_starts  HOST, ngroups+1 run indexes: group_starts[0] == 0,
 *                 nondecreasing, group_starts[ngroups] == k (else
 *                 BCF_ERR_INVALID); empty groups are allowed
 *   other arguments as for bcf_merge_runs
 */
bcf_status bcf_merge_run_groups(const uint32_t *keys_in, const uint32_t *vals_in, const uint64_t *run_offsets,
                                uint32_t k, const uint32_t *group_starts, uint32_t ngroups, uint32_t *keys_out,
                                uint32_t *vals_out, void *temp, uint64_t *temp_bytes, void *stream);

/*
 * Distribution of sorted runs into buckets by sampled splitters (Sec. 3.2,
 * "Distribution", whose bucket sizes Lemma 1 bounds for distinct keys), with
 * the optional pivot buckets of Sec. 3.3 ("Duplicate keys", BCFMergesortPB).
 * From each nonempty run of length L, t evenly spaced candidates are taken
 * (candidate j is the run's key at max(0, floor((j+1) L / t) - 1)); the
 * candidates are sorted into S and the P-1 final splitters are
 * F[c] = S[max(0, floor((c+1) |S| / P) - 1)].  Plain buckets (nb = P): bucket
 * c holds the keys x with F[c-1] < x <= F[c].  Pivot buckets (nb = 2P-1):
 * bucket 2c holds F[c-1] < x < F[c], bucket 2c+1 the keys equal to F[c] when
 * F[c-1] < F[c] (equal splitters share the first one's bucket).  The output
 * lists the pieces (bucket b, run r) in bucket-major order, each piece in its
 * run's order; a piece is a contiguous slice of its run.
 *   keys_in        device, n = run_offsets[s] u32; run r is [off[r], off[r+1])
 *                  and must be nondecreasing (not checked: an unsorted run
 *                  gives unspecified output, but no access outside the buffers)
 *   run_offsets    HOST, s+1 entries (conventions above); s <= 2^22
 *   P, t           1..65536 each; (#nonempty runs) * t <= 2^26; nb * s <= 2^24
 *   pivot_buckets  0: P buckets; nonzero: 2P-1 buckets
 *   keys_out       device, n u32; must not overlap keys_in (BCF_ERR_INVALID)
 *   piece_offsets  device, nb*s + 1 u64: piece (b, r) starts at
 *                  piece_offsets[b*s + r]; the last entry is n
 *   splitters      device, P-1 u32 (0 when n == 0), or NULL
 *   temp           as for the sorts (query with temp == NULL); s == 0 is a
 *                  no-op
 * Steps run on `stream`: candidates, their sort (bcf_sort_u32), splitters,
 * piece bounds by binary search, a prefix sum over the pieces, and one
 * scatter that reads and writes every key once.
 */
bcf_status bcf_distribute_runs(const uint32_t *keys_in, const uint64_t *run_offsets, uint32_t s, uint32_t P,
                               uint32_t t, int pivot_buckets, uint32_t *keys_out, uint64_t *piece_offsets,
                               uint32_t *splitters, void *temp, uint64_t *temp_bytes, void *stream);

/* Human-readable name of a status code (static storage). */
const char *bcf_status_string(bcf_status s);

/* Keys per wave tile: one wave sorts (block sort) or produces (merge pass)
 * 4096 = 64 x 64 keys at a time. */
uint32_t bcf_tile_keys(void);

/* Length of the sorted runs the block sort of a large bcf_sort_u32 (pairs = 0)
 * or bcf_sort_pairs_u32 (pairs = 1) hands to the merge passes under the current
 * tuning: with group tiles one work-group of several waves sorts that many keys
 * in LDS (32768 keys, 16384 pairs); with wave tiles 4096.  Under the default
 * tuning, sorts of at most 2^19 keys use wave tiles (see bcf_tuning). */
uint32_t bcf_run_keys(int pairs);

/* Passes over the data in HBM of a sort of n keys under the current tuning:
 * the block sort plus the merge passes (the paper's Lemma 2: O(1 + log(N/M))
 * scans).  With binary passes (fan-in 2, or below 2^24 keys under the
 * default) there are ceil(log2(R)) merge passes for R = ceil(n /
 * bcf_run_keys(pairs)) runs.  With fan-in 4 (keys or pairs) a pass merges
 * groups of four runs while more than two remain, two levels of the paper's
 * binary merging (Sec. 3.2) per read and write of the data, and a last binary
 * pass merges the final two runs if needed: 2^11 runs take 6 passes instead
 * of 11.  Each merge pass finds its work split by reading
 * O(log n) key samples and keys, in a small launch before it or (see
 * bcf_tuning.fused_partition) in the merge kernel. */
uint32_t bcf_sort_passes(uint64_t n, int pairs);

/*
 * Process-wide tuning knobs (read by every later call; not per stream).
 * Initial values come from environment variables read once, at the first
 * call into the library: BCF_MERGE_MODE, BCF_NT, BCF_NO_SAMPLES,
 * BCF_TILE_SAMPLES, BCF_SEG_GROUP_MIN, BCF_CHECK, BCF_BLOCK_SORT, BCF_FUSED, BCF_FAN_IN.  The autotuner sets them
 * through bcf_set_tuning.  Calls that are in flight on other threads when the
 * knobs change may use either setting; results are identical either way.
 */
typedef struct {
    int32_t merge_variant;     /* merge-pass kernel: 0 persistent waves with next-tile
                                  prefetch (keys), 1 persistent waves, 2 one tile per wave,
                                  3 (default) 2 for keys and 1 for key/value pairs */
    int32_t nontemporal;       /* 1 (default): nontemporal hints on merge-pass tile loads and
                                  stores (in the one-tile-per-wave kernel of a sort only when a
                                  pass streams more than the 256 MiB last-level cache) */
    int32_t sampled_partition; /* 1 (default): a pass's co-rank search starts from the key samples
                                  the previous pass wrote (sorts); 0: search the keys only */
    int32_t tile_samples;      /* 1 (default): keep one sample per 4096-key tile besides the
                                  64-key block samples */
    uint64_t group_min_keys;   /* segmented sorts: segments of at least this many keys are
                                  block-sorted by multi-wave work-groups; 0 = library default */
    int32_t check_runs;        /* 1: bcf_merge_runs checks that every run is sorted */
    int32_t block_sort;        /* block sort of bcf_sort_u32 / bcf_sort_pairs_u32: 0 (default)
                                  3 for sorts of more than 2^19 keys, else 1; 1 wave tiles
                                  sorted by merge rounds; 2 wave tiles sorted by the paper's
                                  ShearSort (Sec. 3.1); 3 multi-wave group tiles sorted by
                                  merge rounds; 4 group tiles of keys sorted by the paper's
                                  long ShearSort over the 8 waves of a work-group (Sec. 3.1,
                                  w^2 h keys by h warps; pairs use 3).  Wave tiles hand runs
                                  of 4096 keys to the merge passes, group tiles runs of
                                  32768 keys (16384 pairs) */
    int32_t fused_partition;   /* 1 (default): a merge pass of bcf_sort_u32 / bcf_sort_pairs_u32
                                  run by the one-tile-per-wave kernel finds each tile's split
                                  itself from the samples (one launch per pass); 0: a separate
                                  partition launch first */
    int32_t merge_fan_in;      /* runs merged per group by a merge pass of the sorts
                                  (bcf_sort_u32, bcf_sort_pairs_u32 and the int32 / float
                                  forms) and of the segmented sorts (device- or host-planned,
                                  keys or pairs).  0 (default): 4 for key/value sorts, for sorts
                                  of at least 2^24 keys and for segmented sorts of at least
                                  2^25 keys in total, else 2.  4 or 2: that fan-in at every
                                  size.  A segment takes four-way steps while more than two
                                  of its runs remain, then a binary one.  Four-way passes of the sorts need
                                  sampled_partition (else 2 is used).  bcf_merge_runs and the
                                  bucket merge of bcf_sort_u32_pb take four-way steps under 4,
                                  and under 0 when a merge (a bucket) has at least 16 runs */
} bcf_tuning;

void bcf_get_tuning(bcf_tuning *out);
/* BCF_ERR_INVALID for a NULL pointer, an out-of-range merge_variant or block_sort, or a
 * merge_fan_in other than 0, 2 or 4. */
bcf_status bcf_set_tuning(const bcf_tuning *in);

/*
 * Per-kernel timing.  While enabled, every launch the library makes is
 * bracketed by two HIP events recorded on the launch's stream.
 * bcf_profile_collect synchronises on those events, fills up to `max` records
 * (one per kernel name) and clears the accumulators.  `bytes` is the
 * algorithmic HBM traffic the launches were planned to move (inputs read once,
 * outputs written once).  Returns the number of records, or -1 on error.
 */
typedef struct {
    char name[48];
    uint64_t launches;
    double total_ms;
    double bytes;
} bcf_kernel_stat;

void bcf_profile_enable(int on);
int bcf_profile_collect(bcf_kernel_stat *out, int max);

#ifdef __cplusplus
}
#endif

#endif /* BCF_H */
