// bcf_dist.hip -- distribution of sorted runs into buckets by sampled
// splitters (paper Sec. 3.2, "Distribution", after Aggarwal and Vitter; the
// bucket bound is Lemma 1), and the pivot-bucket form of Sec. 3.3 ("Duplicate
// keys", BCFMergesortPB) in which keys equal to a splitter get a bucket of
// their own.
//
// Steps, each its own launch on the caller's stream:
//   1. k_dist_candidates  t evenly spaced candidates per nonempty run (the last
//                         key of each of t equal chunks of the run);
//   2. bcf_sort_u32       the candidates sorted (the library's own sort);
//   3. k_dist_splitters   P-1 evenly spaced final splitters from the sorted
//                         candidates (the last key of each of P equal chunks);
//   4. k_dist_bounds      upper bound of every splitter in every run (pivot
//                         buckets: lower bounds too), 8 lanes per search;
//      k_dist_pieces      per (bucket, run) piece its length and source start;
//   5. k_dist_block_sums, k_dist_scan, k_dist_offsets
//                         exclusive prefix over the pieces in bucket-major
//                         order (block sums, their scan, the scan inside each
//                         block): the output offset of every piece, and for
//                         each output tile the piece holding its first key;
//   6. k_dist_scatter     every output tile of 4096 keys walks the pieces it
//                         overlaps and copies them: reads contiguous within a
//                         piece, writes contiguous, one read and one write of
//                         every key (the HBM-bound step).
// The paper computes the splitter ranks by parallel scans and then sorts the
// subsequences by bucket and sequence number; since the runs are sorted, a
// piece is a contiguous slice of its run, so a binary search per piece end and
// a prefix sum replace both.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "bcf.h"

namespace bcf {
bcf_status upload_host(void *dst, const void *src, size_t bytes, hipStream_t s);
void *prof_begin(const char *name, hipStream_t s, double bytes);
void prof_end(void *scope);
}  // namespace bcf

namespace {

constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;
constexpr uint32_t kOutTile = 4096;  // output keys per scatter work-group
constexpr uint32_t kScanBlock = 4096;  // pieces per block of the offset scan
constexpr uint32_t kMaxP = 1u << 16, kMaxT = 1u << 16;
constexpr uint64_t kMaxSamples = 1ull << 26, kMaxPieces = 1ull << 24, kMaxRuns = 1ull << 22;

uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }

__global__ __launch_bounds__(kThreads) void k_dist_candidates(const uint32_t *__restrict__ keys,
                                                              const uint64_t *__restrict__ off,
                                                              const uint32_t *__restrict__ nonempty, uint32_t t,
                                                              uint64_t m, uint32_t *__restrict__ cand)
{
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= m)
        return;
    const uint32_t r = nonempty[i / t];
    const uint64_t j = i % t;
    const uint64_t L = off[r + 1] - off[r];
    const uint64_t e = (j + 1) * L / t;  // end of chunk j
    cand[i] = keys[off[r] + (e ? e - 1 : 0)];
}

__global__ __launch_bounds__(kThreads) void k_dist_splitters(const uint32_t *__restrict__ S, uint64_t m, uint32_t P,
                                                             uint32_t *__restrict__ F)
{
    const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c + 1 >= P)
        return;
    const uint64_t e = (uint64_t)(c + 1) * m / P;
    F[c] = m ? S[e ? e - 1 : 0] : 0u;
}

// Bounds of every splitter in every run: ub[c*s + r] = the first index of run
// r with a key > F[c], and (pivot buckets) lb[c*s + r] = the first index with
// a key >= F[c].  Each 8-lane group of a wave runs one search, narrowing the
// answer's bracket 8-fold per round with 8 probes (six rounds for a run of
// 2^18 keys): few dependent loads, and the probes of the first rounds are
// shared by all splitters of a run in the cache.  (Measured at 2^26 keys in
// 256 runs, P = 256: 8 lanes beat 16 and whole-wave searches.)
constexpr uint32_t kSearchLanes = 8;
constexpr uint64_t kSearchMask = (1ull << kSearchLanes) - 1;

__global__ __launch_bounds__(kThreads) void k_dist_bounds(const uint32_t *__restrict__ keys,
                                                          const uint64_t *__restrict__ off, uint32_t s,
                                                          const uint32_t *__restrict__ F, uint32_t nspl, int pb,
                                                          uint32_t *__restrict__ ub, uint32_t *__restrict__ lb)
{
    const uint32_t lane = threadIdx.x & 63, k = lane % kSearchLanes, shift = lane - k;
    const uint64_t task = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) / kSearchLanes;
    const uint64_t per = (uint64_t)nspl * s;
    const bool have = task < (pb ? 2 * per : per);
    const bool upper = task < per;
    const uint64_t cr = have ? (upper ? task : task - per) : 0;
    const uint32_t c = (uint32_t)(cr / s), r = (uint32_t)(cr % s);
    const uint32_t *run = keys + (have ? off[r] : 0);
    const uint32_t x = have ? F[c] : 0u;
    uint64_t lo = 0, hi = have ? off[r + 1] - off[r] : 0;  // answer in [lo, hi]
    while (__ballot(hi - lo > kSearchLanes) != 0) {
        const bool act = hi - lo > kSearchLanes;
        const uint64_t step = act ? (hi - lo + kSearchLanes - 1) / kSearchLanes : 0;
        const uint64_t q = lo + k * step;
        const bool before = act && q < hi && (upper ? run[q] <= x : run[q] < x);  // the answer lies after q
        const uint32_t cnt = (uint32_t)__popcll((__ballot(before) >> shift) & kSearchMask);
        if (act) {  // probes 0..cnt-1 lie before the answer, probe cnt (if any) not
            const uint64_t nlo = cnt ? lo + (uint64_t)(cnt - 1) * step + 1 : lo;
            hi = min(hi, lo + (uint64_t)cnt * step);
            lo = nlo;
        }
    }
    const uint64_t q = lo + k;
    const bool before = q < hi && (upper ? run[q] <= x : run[q] < x);
    const uint32_t res = (uint32_t)(lo + __popcll((__ballot(before) >> shift) & kSearchMask));
    if (have && k == 0)
        (upper ? ub : lb)[cr] = res;
}

// Piece b*s + r: its length and source start.  Plain buckets: piece b of run r
// ends at cut b = ub(F[b]), bucket b = (F[b-1], F[b]].  Pivot buckets (2P-1,
// bucket 2c = (F[c-1], F[c]), bucket 2c+1 = {F[c]}): cut 2c =
// max(lb(F[c]), ub(F[c-1])), cut 2c+1 = ub(F[c]); the max gives an empty pivot
// bucket to a splitter equal to its predecessor, whose keys are already in
// the predecessor's bucket.  The last cut is the run's end.
__device__ __forceinline__ uint64_t cut_of(const uint32_t *ub, const uint32_t *lb, uint32_t s, uint32_t r, uint32_t q,
                                           uint32_t nb, int pb, uint64_t L)
{
    if (q + 1 >= nb)
        return L;
    if (!pb)
        return ub[(uint64_t)q * s + r];
    const uint32_t c = q / 2;
    if (q & 1)
        return ub[(uint64_t)c * s + r];
    const uint64_t l = lb[(uint64_t)c * s + r];
    return c ? max(l, (uint64_t)ub[(uint64_t)(c - 1) * s + r]) : l;
}

__global__ __launch_bounds__(kThreads) void k_dist_pieces(const uint64_t *__restrict__ off, uint32_t s,
                                                          const uint32_t *__restrict__ ub,
                                                          const uint32_t *__restrict__ lb, uint32_t nb, int pb,
                                                          uint64_t *__restrict__ len, uint64_t *__restrict__ src)
{
    const uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x;  // piece b*s + r
    if (p >= (uint64_t)nb * s)
        return;
    const uint32_t b = (uint32_t)(p / s), r = (uint32_t)(p % s);
    const uint64_t L = off[r + 1] - off[r];
    const uint64_t lo = b ? cut_of(ub, lb, s, r, b - 1, nb, pb, L) : 0;
    const uint64_t hi = cut_of(ub, lb, s, r, b, nb, pb, L);
    len[p] = hi - lo;
    src[p] = off[r] + lo;
}

// Exclusive prefix of len[0, np) into out[0, np], one work-group: each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk's prefixes.
__global__ __launch_bounds__(kScanThreads) void k_dist_scan(const uint64_t *__restrict__ len, uint64_t np,
                                                            uint64_t *__restrict__ out)
{
    __shared__ uint64_t part[kScanThreads];
    const uint32_t tid = threadIdx.x;
    const uint64_t chunk = (np + kScanThreads - 1) / kScanThreads;
    const uint64_t a = min(np, tid * chunk), e = min(np, a + chunk);
    uint64_t sum = 0;
    for (uint64_t i = a; i < e; ++i)
        sum += len[i];
    part[tid] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < kScanThreads; d *= 2) {  // inclusive Hillis-Steele scan
        const uint64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t acc = part[tid] - sum;  // exclusive prefix of this chunk
    for (uint64_t i = a; i < e; ++i) {
        out[i] = acc;
        acc += len[i];
    }
    if (tid == kScanThreads - 1)
        out[np] = part[tid];
}

// largest p in [lo, np) with pos[p] <= x, for x < pos[np] (lo if none)
__device__ __forceinline__ uint64_t piece_of(const uint64_t *pos, uint64_t lo, uint64_t np, uint64_t x)
{
    uint64_t hi = np;  // pos[lo] <= x < pos[hi] when the offsets are monotone
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (pos[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Sum of the piece lengths of each block of kScanBlock pieces (coalesced).
__global__ __launch_bounds__(kThreads) void k_dist_block_sums(const uint64_t *__restrict__ len, uint64_t np,
                                                              uint64_t *__restrict__ bsum)
{
    __shared__ uint64_t red[kThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t sum = 0;
    for (uint32_t k = 0; k < kScanBlock / kThreads; ++k) {
        const uint64_t i = base + threadIdx.x + (uint64_t)k * kThreads;
        sum += i < np ? len[i] : 0;
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t d = kThreads / 2; d > 0; d /= 2) {
        if (threadIdx.x < d)
            red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        bsum[blockIdx.x] = red[0];
}

// Output offsets of the pieces of one block (its exclusive prefix boff[b] plus
// the scan inside the block: each thread takes kScanBlock / kThreads
// consecutive pieces), and for every output tile whose first key a piece
// holds, that piece's index in tile_first.
__global__ __launch_bounds__(kThreads) void k_dist_offsets(const uint64_t *__restrict__ len, uint64_t np,
                                                           const uint64_t *__restrict__ boff, uint64_t nblk,
                                                           uint64_t ntiles, uint64_t *__restrict__ pos,
                                                           uint32_t *__restrict__ tile_first)
{
    constexpr uint32_t kPer = kScanBlock / kThreads;
    __shared__ uint64_t part[kThreads];
    const uint32_t tid = threadIdx.x;
    const uint64_t a = min(np, (uint64_t)blockIdx.x * kScanBlock + (uint64_t)tid * kPer), e = min(np, a + kPer);
    uint64_t sum = 0;
    for (uint64_t i = a; i < e; ++i)
        sum += len[i];
    part[tid] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < kThreads; d *= 2) {  // inclusive Hillis-Steele scan
        const uint64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t acc = boff[blockIdx.x] + part[tid] - sum;
    for (uint64_t i = a; i < e; ++i) {
        const uint64_t l = len[i];
        pos[i] = acc;
        if (l) {  // tiles T with acc <= T * kOutTile < acc + l start in piece i
            for (uint64_t T = (acc + kOutTile - 1) / kOutTile; T < ntiles && T * kOutTile < acc + l; ++T)
                tile_first[T] = (uint32_t)i;
        }
        acc += l;
    }
    if (blockIdx.x == 0 && tid == 0)
        pos[np] = boff[nblk];
}

// Output tile [o0, o1) of kOutTile keys: starting from the piece holding o0
// (tile_first), copy each overlapped piece's share; the next piece is p + 1
// unless that one is empty, then a binary search skips the empty ones.  For
// sorted runs the piece reached for a position o below n holds it
// (pos[p] <= o < pos[p + 1]), so every copy moves at least one key.  An
// unsorted run can make the cuts non-monotone; then the walk stops early
// (unspecified output) but never reads outside the input.
__global__ __launch_bounds__(kThreads) void k_dist_scatter(const uint32_t *__restrict__ keys,
                                                           const uint64_t *__restrict__ pos,
                                                           const uint64_t *__restrict__ src,
                                                           const uint32_t *__restrict__ tile_first, uint64_t np,
                                                           uint64_t n, uint32_t *__restrict__ out)
{
    const uint64_t o0 = (uint64_t)blockIdx.x * kOutTile;
    const uint64_t o1 = min(n, o0 + kOutTile);
    uint64_t o = o0;
    uint64_t p = tile_first[blockIdx.x];
    while (o < o1 && p < np) {
        const uint64_t pp = pos[p], pn = pos[p + 1];
        if (pn <= o) {  // piece p ends before o
            p = (p + 1 < np && pos[p + 2] > o) ? p + 1 : piece_of(pos, p + 1, np, o);
            if (p < np && pos[p + 1] <= o)
                break;  // offsets not monotone: only after a run that was not sorted
            continue;
        }
        if (pp > o)
            break;  // likewise
        const uint64_t pend = min(pn, o1);
        const uint64_t cnt = pend - o;
        const uint64_t f0 = src[p] + (o - pp);
        if (f0 > n || cnt > n - f0)
            break;  // likewise: never read past the input
        const uint32_t *from = keys + f0;
        uint32_t *to = out + o;
        for (uint64_t i = threadIdx.x; i < cnt; i += 4 * kThreads) {
            uint32_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t j = i + (uint64_t)k * kThreads;
                v[k] = j < cnt ? from[j] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t j = i + (uint64_t)k * kThreads;
                if (j < cnt)
                    to[j] = v[k];
            }
        }
        o = pend;
        ++p;
    }
}

__global__ __launch_bounds__(kThreads) void k_dist_zero(uint64_t *__restrict__ a, uint64_t na, uint32_t *__restrict__ b,
                                                        uint64_t nbw)
{
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < na)
        a[i] = 0;
    if (b && i < nbw)
        b[i] = 0;
}

uint32_t blocks_for(uint64_t work) { return (uint32_t)((work + kThreads - 1) / kThreads); }

}  // namespace

extern "C" bcf_status bcf_distribute_runs(const uint32_t *keys_in, const uint64_t *run_offsets, uint32_t s,
                                          uint32_t P, uint32_t t, int pivot_buckets, uint32_t *keys_out,
                                          uint64_t *piece_offsets, uint32_t *splitters, void *temp,
                                          uint64_t *temp_bytes, void *stream)
{
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    if (s == 0) {
        if (!temp)
            *temp_bytes = 0;
        return BCF_OK;
    }
    if (!run_offsets || P == 0 || P > kMaxP || t == 0 || t > kMaxT || s > kMaxRuns)
        return BCF_ERR_INVALID;
    if (run_offsets[0] != 0)
        return BCF_ERR_INVALID;
    uint64_t nonempty = 0;
    for (uint32_t r = 0; r < s; ++r) {
        if (run_offsets[r + 1] < run_offsets[r])
            return BCF_ERR_INVALID;
        nonempty += run_offsets[r + 1] > run_offsets[r];
    }
    const uint64_t n = run_offsets[s];
    const int pb = pivot_buckets ? 1 : 0;
    const uint32_t nb = pb ? 2 * P - 1 : P;
    const uint64_t m = nonempty * t, np = (uint64_t)nb * s;
    if (n > 0xFFFFFFFFull || m > kMaxSamples || np > kMaxPieces)
        return BCF_ERR_INVALID;
    uint64_t sort_need = 0;
    bcf_status st = bcf_sort_u32(nullptr, nullptr, m, nullptr, &sort_need, stream);
    if (st != BCF_OK)
        return st;
    // temp: run offsets | nonempty run ids | candidates | sorted candidates |
    //       splitters | piece lengths | piece sources | the candidate sort's temp
    const uint64_t b_off = align256((uint64_t(s) + 1) * 8), b_nz = align256(std::max<uint64_t>(nonempty, 1) * 4);
    const uint64_t b_cand = align256(std::max<uint64_t>(m, 1) * 4), b_spl = align256(std::max<uint32_t>(P, 2) * 4);
    const uint64_t b_piece = align256(np * 8);
    const uint64_t nblk = (np + kScanBlock - 1) / kScanBlock, ntiles = (n + kOutTile - 1) / kOutTile;
    const uint64_t b_blk = align256((nblk + 1) * 8), b_tiles = align256(std::max<uint64_t>(ntiles, 1) * 4);
    const uint64_t nspl = P - 1, b_bnd = align256(std::max<uint64_t>(nspl * s, 1) * 4);
    const uint64_t need = b_off + b_nz + 2 * b_cand + b_spl + 2 * b_piece + 2 * b_blk + b_tiles + 2 * b_bnd + sort_need;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (!keys_in || !keys_out || !piece_offsets)
        return BCF_ERR_INVALID;
    if (n && keys_in < keys_out + n && keys_out < keys_in + n)
        return BCF_ERR_INVALID;  // the scatter cannot run in place
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    char *tp = static_cast<char *>(temp);
    uint64_t *off_d = reinterpret_cast<uint64_t *>(tp);
    uint32_t *nz_d = reinterpret_cast<uint32_t *>(tp + b_off);
    uint32_t *cand = reinterpret_cast<uint32_t *>(tp + b_off + b_nz);
    uint32_t *S = reinterpret_cast<uint32_t *>(tp + b_off + b_nz + b_cand);
    uint32_t *F_int = reinterpret_cast<uint32_t *>(tp + b_off + b_nz + 2 * b_cand);
    uint64_t *len = reinterpret_cast<uint64_t *>(tp + b_off + b_nz + 2 * b_cand + b_spl);
    uint64_t *srcp = reinterpret_cast<uint64_t *>(tp + b_off + b_nz + 2 * b_cand + b_spl + b_piece);
    char *tail = tp + b_off + b_nz + 2 * b_cand + b_spl + 2 * b_piece;
    uint64_t *bsum = reinterpret_cast<uint64_t *>(tail);
    uint64_t *boff = reinterpret_cast<uint64_t *>(tail + b_blk);
    uint32_t *tile_first = reinterpret_cast<uint32_t *>(tail + 2 * b_blk);
    uint32_t *ub = reinterpret_cast<uint32_t *>(tail + 2 * b_blk + b_tiles);
    uint32_t *lb = reinterpret_cast<uint32_t *>(tail + 2 * b_blk + b_tiles + b_bnd);
    void *sort_temp = tail + 2 * b_blk + b_tiles + 2 * b_bnd;
    uint32_t *F = splitters ? splitters : F_int;
    if (n == 0) {  // no keys: every piece empty, splitters 0
        const uint64_t w = std::max<uint64_t>(np + 1, P - 1);
        hipLaunchKernelGGL(k_dist_zero, dim3(blocks_for(w)), dim3(kThreads), 0, hs, piece_offsets, np + 1,
                           P > 1 ? F : nullptr, (uint64_t)(P - 1));
        return hipGetLastError() == hipSuccess ? BCF_OK : BCF_ERR_DEVICE;
    }
    std::vector<uint32_t> nz;
    nz.reserve(nonempty);
    for (uint32_t r = 0; r < s; ++r)
        if (run_offsets[r + 1] > run_offsets[r])
            nz.push_back(r);
    if ((st = bcf::upload_host(off_d, run_offsets, (uint64_t(s) + 1) * 8, hs)) != BCF_OK)
        return st;
    if ((st = bcf::upload_host(nz_d, nz.data(), nz.size() * 4, hs)) != BCF_OK)
        return st;
    hipLaunchKernelGGL(k_dist_candidates, dim3(blocks_for(m)), dim3(kThreads), 0, hs, keys_in, off_d, nz_d, t, m, cand);
    if (hipGetLastError() != hipSuccess)
        return BCF_ERR_DEVICE;
    uint64_t sb = sort_need;
    if ((st = bcf_sort_u32(cand, S, m, sort_temp, &sb, stream)) != BCF_OK)
        return st;
    if (P > 1)
        hipLaunchKernelGGL(k_dist_splitters, dim3(blocks_for(P - 1)), dim3(kThreads), 0, hs, S, m, P, F);
    {
        void *ps = bcf::prof_begin("dist_pieces", hs, 0.0);
        const uint64_t searches = nspl * s * (pb ? 2 : 1);
        if (searches)
            hipLaunchKernelGGL(k_dist_bounds, dim3(blocks_for(kSearchLanes * searches)), dim3(kThreads), 0, hs, keys_in,
                               off_d, s,
                               F, (uint32_t)nspl, pb, ub, lb);
        hipLaunchKernelGGL(k_dist_pieces, dim3(blocks_for(np)), dim3(kThreads), 0, hs, off_d, s, ub, lb, nb, pb, len,
                           srcp);
        bcf::prof_end(ps);
    }
    hipLaunchKernelGGL(k_dist_block_sums, dim3((uint32_t)nblk), dim3(kThreads), 0, hs, len, np, bsum);
    hipLaunchKernelGGL(k_dist_scan, dim3(1), dim3(kScanThreads), 0, hs, bsum, nblk, boff);
    hipLaunchKernelGGL(k_dist_offsets, dim3((uint32_t)nblk), dim3(kThreads), 0, hs, len, np, boff, nblk, ntiles,
                       piece_offsets, tile_first);
    {
        void *ps = bcf::prof_begin("dist_scatter", hs, 8.0 * n);
        hipLaunchKernelGGL(k_dist_scatter, dim3((uint32_t)ntiles), dim3(kThreads), 0, hs, keys_in, piece_offsets,
                           srcp, tile_first, np, n, keys_out);
        bcf::prof_end(ps);
    }
    return hipGetLastError() == hipSuccess ? BCF_OK : BCF_ERR_DEVICE;
}
