/*
 * CPU oracle for the bank-conflict-free sort library -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load this library; the GPU path never calls
 * it and shares no code with it.
 *
 * What it computes (Sitchinava & Weichert, "Bank Conflict Free Comparison-based
 * Sorting On GPUs", problem statement of Sec. 3 and the pseudocode appendix,
 * which sort ascending; the binary merge of Sec. 3.2):
 *   - oracle_sort_u32         the nondecreasing permutation of n u32 keys;
 *   - oracle_sort_pairs_u32   key/value pairs ordered by key, equal keys kept in
 *                             input order (stable): lexicographic order on
 *                             (key, original index);
 *   - oracle_merge_runs       the stable sort of the concatenation of k sorted
 *                             runs, i.e. a k-way merge where ties go to the
 *                             lower run index and then the earlier position;
 *   - oracle_segmented_sort   oracle_sort_u32 applied to every segment;
 *   - oracle_sort_typed       int32 keys (signed order) or float keys (IEEE 754
 *                             totalOrder), stable, values optional;
 *   - oracle_sort_u64            ascending sort of unsigned 64-bit keys.
 *   - oracle_colored_prefix_sums  per-color inclusive prefix sums (the paper's
 *                             bank-conflict example, Sec. 1.2).
 *   - oracle_distribute_runs  the distribution of sorted runs into buckets by
 *                             sampled splitters (Sec. 3.2, Lemma 1), optionally
 *                             with pivot buckets for splitter-equal keys
 *                             (BCFMergesortPB, Sec. 3.3).
 * Keys compare as unsigned 32-bit integers (the paper does not fix signedness).
 *
 * Algorithm: top-down merge sort (split in halves, sort each, merge taking the
 * left element on ties), with a scratch buffer.  No blocking, no networks.
 *
 * Also: an order-independent multiset hash used to check that an output is a
 * permutation of its input at sizes where element-wise comparison is costly.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- keys only ---------------------------------------------------------- */

/* merge src[lo,mid) and src[mid,hi) into dst[lo,hi); left wins ties */
static void merge_keys(const uint32_t *src, uint32_t *dst, size_t lo, size_t mid, size_t hi)
{
    size_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        if (src[i] <= src[j])
            dst[o++] = src[i++];
        else
            dst[o++] = src[j++];
    }
    while (i < mid)
        dst[o++] = src[i++];
    while (j < hi)
        dst[o++] = src[j++];
}

/* sort a[lo,hi) in place, using tmp[lo,hi) as scratch */
static void msort_keys(uint32_t *a, uint32_t *tmp, size_t lo, size_t hi)
{
    if (hi - lo < 2)
        return;
    size_t mid = lo + (hi - lo) / 2;
    msort_keys(a, tmp, lo, mid);
    msort_keys(a, tmp, mid, hi);
    merge_keys(a, tmp, lo, mid, hi);
    memcpy(a + lo, tmp + lo, (hi - lo) * sizeof(uint32_t));
}

/* out may alias in.  Returns 0 on success, -1 if scratch cannot be allocated. */
int oracle_sort_u32(const uint32_t *in, uint32_t *out, uint64_t n)
{
    if (n == 0)
        return 0;
    uint32_t *tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tmp)
        return -1;
    if (out != in)
        memcpy(out, in, n * sizeof(uint32_t));
    msort_keys(out, tmp, 0, n);
    free(tmp);
    return 0;
}

/* ---- key/value pairs (stable) ------------------------------------------- */

static void merge_pairs(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv,
                        size_t lo, size_t mid, size_t hi)
{
    size_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        if (sk[i] <= sk[j]) {
            dk[o] = sk[i];
            dv[o] = sv[i];
            i++;
        } else {
            dk[o] = sk[j];
            dv[o] = sv[j];
            j++;
        }
        o++;
    }
    while (i < mid) {
        dk[o] = sk[i];
        dv[o] = sv[i];
        i++;
        o++;
    }
    while (j < hi) {
        dk[o] = sk[j];
        dv[o] = sv[j];
        j++;
        o++;
    }
}

static void msort_pairs(uint32_t *k, uint32_t *v, uint32_t *tk, uint32_t *tv, size_t lo, size_t hi)
{
    if (hi - lo < 2)
        return;
    size_t mid = lo + (hi - lo) / 2;
    msort_pairs(k, v, tk, tv, lo, mid);
    msort_pairs(k, v, tk, tv, mid, hi);
    merge_pairs(k, v, tk, tv, lo, mid, hi);
    memcpy(k + lo, tk + lo, (hi - lo) * sizeof(uint32_t));
    memcpy(v + lo, tv + lo, (hi - lo) * sizeof(uint32_t));
}

int oracle_sort_pairs_u32(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                          uint32_t *vout, uint64_t n)
{
    if (n == 0)
        return 0;
    uint32_t *tk = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *tv = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tk || !tv) {
        free(tk);
        free(tv);
        return -1;
    }
    if (kout != kin)
        memcpy(kout, kin, n * sizeof(uint32_t));
    if (vout != vin)
        memcpy(vout, vin, n * sizeof(uint32_t));
    msort_pairs(kout, vout, tk, tv, 0, n);
    free(tk);
    free(tv);
    return 0;
}

/* ---- other key types ------------------------------------------------------ */

/*
 * Stable sort of 32-bit keys under a key type's order, values (when not NULL)
 * carried: kind 1 = int32 (signed order), kind 2 = IEEE 754 binary32 in
 * totalOrder (IEEE 754-2008, 5.10): values of different sign order by sign
 * (negative first); for two positive encodings the smaller magnitude field
 * (exponent and significand, which already orders +0 < subnormals < normals
 * < +inf < NaNs by payload) comes first, for two negative ones the larger.
 * The same top-down merge sort, with the comparison as a function.
 */
static int le_i32(uint32_t a, uint32_t b) { return (int32_t)a <= (int32_t)b; }

static int le_f32_total(uint32_t a, uint32_t b)
{
    const uint32_t sa = a >> 31, sb = b >> 31;
    if (sa != sb)
        return sa > sb; /* a negative, b positive */
    const uint32_t ma = a & 0x7fffffffu, mb = b & 0x7fffffffu;
    return sa ? ma >= mb : ma <= mb;
}

static void merge_typed(int (*le)(uint32_t, uint32_t), const uint32_t *sk, const uint32_t *sv, uint32_t *dk,
                        uint32_t *dv, size_t lo, size_t mid, size_t hi)
{
    size_t i = lo, j = mid, o = lo;
    while (i < mid || j < hi) {
        int take_left = j >= hi || (i < mid && le(sk[i], sk[j]));
        size_t s = take_left ? i++ : j++;
        dk[o] = sk[s];
        if (sv)
            dv[o] = sv[s];
        o++;
    }
}

static void msort_typed(int (*le)(uint32_t, uint32_t), uint32_t *k, uint32_t *v, uint32_t *tk, uint32_t *tv,
                        size_t lo, size_t hi)
{
    if (hi - lo < 2)
        return;
    size_t mid = lo + (hi - lo) / 2;
    msort_typed(le, k, v, tk, tv, lo, mid);
    msort_typed(le, k, v, tk, tv, mid, hi);
    merge_typed(le, k, v, tk, tv, lo, mid, hi);
    memcpy(k + lo, tk + lo, (hi - lo) * sizeof(uint32_t));
    if (v)
        memcpy(v + lo, tv + lo, (hi - lo) * sizeof(uint32_t));
}

int oracle_sort_typed(int kind, const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                      uint64_t n)
{
    int (*le)(uint32_t, uint32_t) = kind == 1 ? le_i32 : kind == 2 ? le_f32_total : 0;
    if (!le)
        return -2;
    if (n == 0)
        return 0;
    uint32_t *tk = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *tv = vin ? (uint32_t *)malloc(n * sizeof(uint32_t)) : 0;
    if (!tk || (vin && !tv)) {
        free(tk);
        free(tv);
        return -1;
    }
    if (kout != kin)
        memcpy(kout, kin, n * sizeof(uint32_t));
    if (vin && vout != vin)
        memcpy(vout, vin, n * sizeof(uint32_t));
    msort_typed(le, kout, vin ? vout : 0, tk, tv, 0, n);
    free(tk);
    free(tv);
    return 0;
}

/* ---- colored prefix sums ----------------------------------------------- */

/*
 * The paper's motivating problem for bank conflicts (Sec. 1.2 and its
 * appendix on colored prefix sums): every element i has a value and one of d
 * colors; out[i] is the sum of the values of the elements j <= i of the same
 * color (inclusive), modulo 2^32.  One pass with d running sums.  Colors at or
 * above d count as color d - 1.
 */
int oracle_colored_prefix_sums(const uint32_t *values, const uint8_t *colors, uint32_t *out, uint64_t n, uint32_t d)
{
    if (d == 0 || d > 256)
        return -2;
    uint32_t run[256];
    memset(run, 0, sizeof(run));
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = colors[i] < d ? colors[i] : d - 1;
        run[c] += values[i];
        out[i] = run[c];
    }
    return 0;
}

/* ---- 64-bit keys ---------------------------------------------------------- */

/* merge src[lo,mid) and src[mid,hi) of u64 keys into dst[lo,hi); left wins ties */
static void merge_u64(const uint64_t *src, uint64_t *dst, size_t lo, size_t mid, size_t hi)
{
    size_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        const uint64_t x = src[i], y = src[j];
        if (x <= y)
            dst[o++] = src[i++];
        else
            dst[o++] = src[j++];
    }
    while (i < mid)
        dst[o++] = src[i++];
    while (j < hi)
        dst[o++] = src[j++];
}

static void msort_u64(uint64_t *a, uint64_t *tmp, size_t lo, size_t hi)
{
    if (hi - lo < 2)
        return;
    const size_t mid = lo + (hi - lo) / 2;
    msort_u64(a, tmp, lo, mid);
    msort_u64(a, tmp, mid, hi);
    merge_u64(a, tmp, lo, mid, hi);
    memcpy(a + lo, tmp + lo, (hi - lo) * sizeof(uint64_t));
}

/* Ascending sort of unsigned 64-bit keys (top-down merge sort, as for u32). */
int oracle_sort_u64(const uint64_t *in, uint64_t *out, uint64_t n)
{
    memcpy(out, in, n * sizeof(uint64_t));
    if (n < 2)
        return 0;
    uint64_t *tmp = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!tmp)
        return -1;
    msort_u64(out, tmp, 0, n);
    free(tmp);
    return 0;
}

/* ---- k-way merge of sorted runs ------------------------------------------ */

/*
 * Runs r = 0..k-1 occupy [off[r], off[r+1]) of kin (and vin when not NULL).
 * Repeatedly emits the smallest head key; among equal heads the lowest run
 * index wins, and within a run elements leave in order, so the result is the
 * stable sort of the concatenation.  O(n*k).  Returns -1 on bad offsets.
 */
int oracle_merge_runs(const uint32_t *kin, const uint32_t *vin, const uint64_t *off, uint32_t k,
                      uint32_t *kout, uint32_t *vout)
{
    if (k == 0)
        return 0;
    if (off[0] != 0)
        return -1;
    for (uint32_t r = 0; r < k; r++)
        if (off[r + 1] < off[r])
            return -1;
    uint64_t n = off[k];
    uint64_t *cur = (uint64_t *)malloc((size_t)k * sizeof(uint64_t));
    if (!cur)
        return -1;
    for (uint32_t r = 0; r < k; r++)
        cur[r] = off[r];
    for (uint64_t o = 0; o < n; o++) {
        int64_t best = -1;
        for (uint32_t r = 0; r < k; r++) {
            if (cur[r] == off[r + 1])
                continue;
            if (best < 0 || kin[cur[r]] < kin[cur[best]])
                best = (int64_t)r;
        }
        kout[o] = kin[cur[best]];
        if (vin && vout)
            vout[o] = vin[cur[best]];
        cur[best]++;
    }
    free(cur);
    return 0;
}

/* ---- segmented sort -------------------------------------------------------- */

int oracle_segmented_sort(const uint32_t *kin, uint32_t *kout, const uint64_t *off, uint32_t nseg)
{
    if (nseg == 0)
        return 0;
    if (off[0] != 0)
        return -1;
    for (uint32_t s = 0; s < nseg; s++) {
        if (off[s + 1] < off[s])
            return -1;
        int rc = oracle_sort_u32(kin + off[s], kout + off[s], off[s + 1] - off[s]);
        if (rc)
            return rc;
    }
    return 0;
}

/* ---- checks ----------------------------------------------------------------- */

/* SplitMix64 output function, used only as a hash mixer */
static uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * Order-independent multiset hash of (key, value) elements (value 0 when vals is
 * NULL): sum and xor of mix64(key ^ (value * golden)), modulo 2^64.
 */
void oracle_multiset_hash(const uint32_t *keys, const uint32_t *vals, uint64_t n, uint64_t *sum_out,
                          uint64_t *xor_out)
{
    uint64_t s = 0, x = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t v = vals ? (uint64_t)vals[i] : 0;
        uint64_t h = mix64((uint64_t)keys[i] ^ (v * 0x9E3779B97F4A7C15ull));
        s += h;
        x ^= h;
    }
    *sum_out = s;
    *xor_out = x;
}

/* 1 if keys[0..n) is nondecreasing */
int oracle_is_sorted_u32(const uint32_t *keys, uint64_t n)
{
    for (uint64_t i = 1; i < n; i++)
        if (keys[i - 1] > keys[i])
            return 0;
    return 1;
}

/* ---- distribution of sorted runs into buckets (Sec. 3.2) ----------------- */

/*
 * The paper's distribution step (Sec. 3.2, "Distribution", with Lemma 1) and
 * its pivot-bucket form for duplicate keys (Sec. 3.3, "Duplicate keys",
 * BCFMergesortPB), in the paper's order:
 *   1. from each nonempty run of length L take t evenly spaced candidates:
 *      candidate j (j = 0..t-1) is the last key of the j-th of t equal chunks,
 *      run[max(0, floor((j+1) L / t) - 1)];
 *   2. sort the candidates into S (the top-down merge sort above);
 *   3. take P-1 evenly spaced final splitters from S:
 *      F[c] = S[max(0, floor((c+1) |S| / P) - 1)], c = 0..P-2;
 *   4. bucket of a key x.  Plain: c = #{F < x}, i.e. bucket c holds
 *      (F[c-1], F[c]] with F[-1] = -inf and F[P-1] = +inf (P buckets).
 *      Pivot buckets (pb != 0, 2P-1 buckets): a key equal to some splitter
 *      goes to bucket 2c+1 for the smallest c with F[c] == x, any other key to
 *      bucket 2 #{F < x};
 *   5. rearrange by (bucket, run): the output lists bucket 0's keys of run 0,
 *      of run 1, ..., then bucket 1's, each piece in its run's order.
 * piece_off gets nb*s + 1 entries: piece (b, r) starts at piece_off[b*s + r];
 * the last entry is n.  splitters gets the P-1 final splitters (may be NULL).
 * The key-to-bucket counts in step 4 use a binary search over the sorted
 * splitters (the smallest index with F[i] >= x, resp. > x).
 * Returns 0, -1 on allocation failure, -2 on bad arguments.
 */
static uint64_t count_less(const uint32_t *F, uint64_t m, uint32_t x)
{
    uint64_t lo = 0, hi = m; /* first i with F[i] >= x */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (F[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

int oracle_distribute_runs(const uint32_t *keys, const uint64_t *off, uint32_t s, uint32_t P, uint32_t t, int pb,
                           uint32_t *out, uint64_t *piece_off, uint32_t *splitters)
{
    if (s == 0 || P == 0 || t == 0 || off[0] != 0)
        return -2;
    for (uint32_t r = 0; r < s; r++)
        if (off[r + 1] < off[r])
            return -2;
    const uint64_t n = off[s];
    const uint64_t nb = pb ? 2 * (uint64_t)P - 1 : P;
    uint64_t nonempty = 0;
    for (uint32_t r = 0; r < s; r++)
        nonempty += off[r + 1] > off[r];
    const uint64_t m = nonempty * t;
    uint32_t *cand = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *S = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *F = malloc((P > 1 ? P - 1 : 1) * sizeof(uint32_t));
    uint64_t *cnt = calloc(nb * s + 1, sizeof(uint64_t));
    uint32_t *bucket = malloc((n ? n : 1) * sizeof(uint32_t));
    if (!cand || !S || !F || !cnt || !bucket) {
        free(cand), free(S), free(F), free(cnt), free(bucket);
        return -1;
    }
    /* 1. candidates */
    uint64_t k = 0;
    for (uint32_t r = 0; r < s; r++) {
        const uint64_t L = off[r + 1] - off[r];
        if (L == 0)
            continue;
        for (uint32_t j = 0; j < t; j++) {
            uint64_t e = ((uint64_t)(j + 1) * L) / t;
            cand[k++] = keys[off[r] + (e ? e - 1 : 0)];
        }
    }
    /* 2. sort them */
    if (m && oracle_sort_u32(cand, S, m) != 0) {
        free(cand), free(S), free(F), free(cnt), free(bucket);
        return -1;
    }
    /* 3. final splitters */
    for (uint32_t c = 0; c + 1 < P; c++) {
        uint64_t e = ((uint64_t)(c + 1) * m) / P;
        F[c] = m ? S[e ? e - 1 : 0] : 0;
        if (splitters)
            splitters[c] = F[c];
    }
    /* 4. bucket of every key, counted per (bucket, run) */
    for (uint32_t r = 0; r < s; r++) {
        for (uint64_t i = off[r]; i < off[r + 1]; i++) {
            const uint32_t x = keys[i];
            const uint64_t lt = count_less(F, P - 1, x);
            uint64_t b;
            if (!pb)
                b = lt;
            else if (lt < P - 1 && F[lt] == x)
                b = 2 * lt + 1; /* F[lt] is the first splitter equal to x */
            else
                b = 2 * lt;
            bucket[i] = (uint32_t)b;
            cnt[b * s + r]++;
        }
    }
    /* 5. piece offsets (bucket-major), then the keys in input order per piece */
    uint64_t acc = 0;
    for (uint64_t p = 0; p < nb * s; p++) {
        const uint64_t c = cnt[p];
        piece_off[p] = acc;
        cnt[p] = acc; /* now the next free slot of piece p */
        acc += c;
    }
    piece_off[nb * s] = acc;
    for (uint32_t r = 0; r < s; r++)
        for (uint64_t i = off[r]; i < off[r + 1]; i++)
            out[cnt[(uint64_t)bucket[i] * s + r]++] = keys[i];
    free(cand), free(S), free(F), free(cnt), free(bucket);
    return 0;
}
