"""Pins for the CPU oracle: checks against what the mathematics fixes, not
against the oracle's own formula.

* brute force over every permutation of small distinct inputs and every word
  over {0,1,2}, compared with the order-statistic definition of sorting
  (output[i] is the value v with #{x < v} <= i < #{x <= v});
* library special cases (numpy.sort, numpy.argsort(kind="stable"), Python's
  sorted on (key, index) tuples);
* invariants (nondecreasing, permutation-preserving, stability);
* merge of sorted runs == stable sort of their concatenation (the paper's
  binary merge of Sec. 3.2 generalised to k runs), k = 1 is the identity;
* planted mistakes: mutated copies of the oracle source, built here on the CPU,
  must each fail at least one of these pins.
"""

import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def order_statistics(xs):
    """Sorted output by the counting definition (no sort routine involved)."""
    xs = list(xs)
    n = len(xs)
    out = [None] * n
    for v in set(xs):
        lt = sum(1 for x in xs if x < v)
        le = sum(1 for x in xs if x <= v)
        for i in range(lt, le):
            out[i] = v
    return out


# ---------------------------------------------------------------- sort_u32


@pytest.mark.parametrize("n", range(0, 8))
def test_sort_every_permutation(oracle_mod, n):
    ident = np.arange(n, dtype=np.uint32)
    for perm in itertools.permutations(range(n)):
        got = oracle_mod.sort_u32(np.array(perm, dtype=np.uint32))
        assert np.array_equal(got, ident), perm


def test_sort_every_permutation_of_8_sampled_keys(oracle_mod):
    keys = np.array([0, 7, 0xFFFFFFFF, 3, 0x80000000, 12, 0x7FFFFFFF, 1], dtype=np.uint32)
    want = np.array(order_statistics(keys.tolist()), dtype=np.uint32)
    for perm in itertools.permutations(range(8)):
        got = oracle_mod.sort_u32(keys[list(perm)])
        assert np.array_equal(got, want)


@pytest.mark.parametrize("n", range(1, 9))
def test_sort_every_ternary_word(oracle_mod, n):
    for word in itertools.product((0, 1, 2), repeat=n):
        got = oracle_mod.sort_u32(np.array(word, dtype=np.uint32)).tolist()
        assert got == order_statistics(word), word


def test_sort_unsigned_order_extremes(oracle_mod):
    keys = np.array([0xFFFFFFFF, 0, 0x80000000, 0x7FFFFFFF, 0xFFFFFFFF, 1, 0], dtype=np.uint32)
    got = oracle_mod.sort_u32(keys).tolist()
    assert got == [0, 0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0xFFFFFFFF]


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS + workloads.PAPER_DISTRIBUTIONS)
@pytest.mark.parametrize("n", [1, 2, 3, 100, 4095, 4097, 1 << 16])
def test_sort_matches_numpy(oracle_mod, dist, n):
    keys = workloads.keys_u32(dist, n, seed=3)
    assert np.array_equal(oracle_mod.sort_u32(keys), np.sort(keys, kind="stable"))


def test_sort_matches_numpy_large(oracle_mod):
    keys = workloads.keys_u32("uniform", 1 << 20, seed=11)
    got = oracle_mod.sort_u32(keys)
    assert np.array_equal(got, np.sort(keys))
    assert oracle_mod.is_sorted_u32(got)
    assert oracle_mod.multiset_hash(got) == oracle_mod.multiset_hash(keys)


# ---------------------------------------------------------------- pairs (stable)


@pytest.mark.parametrize("n", range(0, 8))
def test_pairs_every_ternary_word_stable(oracle_mod, n):
    for word in itertools.product((0, 1, 2), repeat=n):
        keys = np.array(word, dtype=np.uint32)
        vals = np.arange(n, dtype=np.uint32) * 7 + 5
        ko, vo = oracle_mod.sort_pairs_u32(keys, vals)
        want = sorted(zip(word, range(n)))  # lexicographic (key, original index)
        assert ko.tolist() == [k for k, _ in want]
        assert vo.tolist() == [int(vals[i]) for _, i in want]


@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf", "paper_01", "paper_dups"])
def test_pairs_match_numpy_stable_argsort(oracle_mod, dist):
    keys, vals = workloads.pairs_u32(dist, 50_000, seed=5)
    vals = vals ^ np.uint32(0xA5A5A5A5)  # values need not be indices
    ko, vo = oracle_mod.sort_pairs_u32(keys, vals)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(ko, keys[order])
    assert np.array_equal(vo, vals[order])


# ---------------------------------------------------------------- merge of runs


def _stable_concat_sort(keys, vals):
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[order]


@pytest.mark.parametrize("sizes", [[5], [0], [3, 4], [0, 6], [6, 0], [1, 1, 1],
                                   [4, 0, 3, 0, 5], [2] * 17, list(range(17))])
def test_merge_runs_small(oracle_mod, sizes):
    keys, offs = workloads.sorted_runs(sizes, seed=2, dist="dups")
    vals = np.arange(keys.size, dtype=np.uint32)
    ko, vo = oracle_mod.merge_runs(keys, offs, vals)
    ek, ev = _stable_concat_sort(keys, vals)
    assert np.array_equal(ko, ek) and np.array_equal(vo, ev)


def test_merge_runs_bruteforce_two_runs(oracle_mod):
    # every pair of sorted ternary runs of lengths <= 4: result must be the
    # order-statistic sort, and equal keys must leave run 0 before run 1.
    runs = [tuple(sorted(w)) for m in range(5) for w in itertools.product((0, 1, 2), repeat=m)]
    runs = sorted(set(runs))
    for a in runs:
        for b in runs:
            keys = np.array(a + b, dtype=np.uint32)
            offs = np.array([0, len(a), len(a) + len(b)], dtype=np.uint64)
            vals = np.arange(keys.size, dtype=np.uint32)
            ko, vo = oracle_mod.merge_runs(keys, offs, vals)
            assert ko.tolist() == order_statistics(a + b)
            want = [i for _, i in sorted(zip(a + b, range(len(a + b))))]
            assert vo.tolist() == want


def test_merge_single_run_is_identity(oracle_mod):
    keys, offs = workloads.sorted_runs([1000], seed=4)
    assert np.array_equal(oracle_mod.merge_runs(keys, offs), keys)


def test_merge_runs_rejects_bad_offsets(oracle_mod):
    keys = np.arange(10, dtype=np.uint32)
    with pytest.raises(ValueError):
        oracle_mod.merge_runs(keys, np.array([0, 6, 4, 10], dtype=np.uint64))


# ---------------------------------------------------------------- segmented


def test_segmented_sort(oracle_mod):
    sizes = [0, 1, 2, 0, 37, 4096, 5000, 1]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    keys = workloads.keys_u32("uniform", int(offs[-1]), seed=9)
    got = oracle_mod.segmented_sort(keys, offs)
    for s in range(len(sizes)):
        lo, hi = int(offs[s]), int(offs[s + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi]))


# ---------------------------------------------------------------- is_sorted (a checker)


@pytest.mark.parametrize("n", range(0, 8))
def test_is_sorted_every_ternary_word(oracle_mod, n):
    # a sequence is sorted exactly when it equals its order-statistic sort
    for word in itertools.product((0, 1, 2), repeat=n):
        want = list(word) == order_statistics(word)
        assert oracle_mod.is_sorted_u32(np.array(word, dtype=np.uint32)) == want, word


def test_is_sorted_rejects_one_inversion_anywhere(oracle_mod):
    base = np.sort(workloads.keys_u32("uniform", 10_000, seed=12))
    base = np.unique(base)  # strictly increasing, so any swap is an inversion
    m = base.size
    assert oracle_mod.is_sorted_u32(base)
    for i in (0, 1, m // 2, m - 3, m - 2):  # first pair, middle, last pair
        bad = base.copy()
        bad[i], bad[i + 1] = bad[i + 1], bad[i]
        assert not oracle_mod.is_sorted_u32(bad), i
    # the last element alone out of place, and the first alone
    bad = base.copy()
    bad[-1] = 0
    assert not oracle_mod.is_sorted_u32(bad)
    bad = base.copy()
    bad[0] = 0xFFFFFFFF
    assert not oracle_mod.is_sorted_u32(bad)


def test_is_sorted_accepts_equal_neighbours_and_extremes(oracle_mod):
    assert oracle_mod.is_sorted_u32(np.array([], dtype=np.uint32))
    assert oracle_mod.is_sorted_u32(np.array([7], dtype=np.uint32))
    assert oracle_mod.is_sorted_u32(np.array([5, 5, 5, 5], dtype=np.uint32))
    assert oracle_mod.is_sorted_u32(np.array([0, 0, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0xFFFFFFFF],
                                             dtype=np.uint32))
    # unsigned order: 0x80000000 is above 0x7FFFFFFF
    assert not oracle_mod.is_sorted_u32(np.array([0x80000000, 0x7FFFFFFF], dtype=np.uint32))


# ---------------------------------------------------------------- chunked (all cores)


@pytest.mark.parametrize("threads", [1, 2, 3, 5, 8, 64])
@pytest.mark.parametrize("n", [0, 1, 2, 7, 1000, 4097, 100_003])
def test_chunked_sorts_match_numpy(oracle_mod, threads, n):
    keys = workloads.keys_u32("zipf", n, seed=n + threads)
    assert np.array_equal(oracle_mod.sort_u32_chunked(keys, threads), np.sort(keys))
    vals = np.arange(n, dtype=np.uint32) ^ np.uint32(0x5A5A5A5A)
    ko, vo = oracle_mod.sort_pairs_u32_chunked(keys, vals, threads)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(ko, keys[order]) and np.array_equal(vo, vals[order])


def test_chunked_sort_every_ternary_word(oracle_mod):
    for n in range(1, 8):
        for word in itertools.product((0, 1, 2), repeat=n):
            got = oracle_mod.sort_u32_chunked(np.array(word, dtype=np.uint32), 3).tolist()
            assert got == order_statistics(word), word


def test_segmented_threads_match_numpy(oracle_mod):
    sizes = [0, 1, 2, 0, 37, 4096, 5000, 1, 0, 20_000, 3]
    offs = workloads.segment_offsets(sizes)
    keys = workloads.keys_u32("distinct16", int(offs[-1]), seed=9)
    vals = np.arange(keys.size, dtype=np.uint32)
    for threads in (1, 3, 16):
        got = oracle_mod.segmented_sort_threads(keys, offs, threads)
        gk, gv = oracle_mod.segmented_sort_threads(keys, offs, threads, vals)
        for s in range(len(sizes)):
            lo, hi = int(offs[s]), int(offs[s + 1])
            order = np.argsort(keys[lo:hi], kind="stable")
            assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi]))
            assert np.array_equal(gk[lo:hi], keys[lo:hi][order])
            assert np.array_equal(gv[lo:hi], vals[lo:hi][order])


# ---------------------------------------------------------------- multiset hash


def test_multiset_hash_permutation_invariant_and_sensitive(oracle_mod):
    keys, vals = workloads.pairs_u32("zipf", 10_000, seed=8)
    h = oracle_mod.multiset_hash(keys, vals)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(keys.size)
    assert oracle_mod.multiset_hash(keys[perm], vals[perm]) == h
    k2 = keys.copy()
    k2[17] ^= 1
    assert oracle_mod.multiset_hash(k2, vals) != h
    v2 = vals.copy()
    v2[3], v2[4] = v2[4], v2[3]  # swapping values between different keys
    if keys[3] != keys[4]:
        assert oracle_mod.multiset_hash(keys, v2) != h


# ---------------------------------------------------- other key types


def _f32_bits(xs):
    return np.asarray(xs, dtype=np.float32).view(np.uint32)


# IEEE 754 totalOrder of binary32 (IEEE 754-2008, 5.10), written out from the
# standard's definition: negative NaNs (larger payload first), -inf, negative
# normals and subnormals by decreasing magnitude, -0, +0, positive values by
# increasing magnitude, +inf, positive NaNs (smaller payload first).
TOTAL_ORDER_F32_BITS = [
    0xFFC00001, 0xFFC00000, 0xFF800001,          # -NaN (quiet, payload 1), -qNaN, -sNaN
    0xFF800000,                                  # -inf
    0xFF7FFFFF, 0xBF800000, 0x80800000,          # -max, -1, -min normal
    0x807FFFFF, 0x80000001,                      # -max subnormal, -min subnormal
    0x80000000, 0x00000000,                      # -0, +0
    0x00000001, 0x007FFFFF, 0x00800000,          # +min subnormal, +max subnormal, +min normal
    0x3F800000, 0x7F7FFFFF, 0x7F800000,          # +1, +max, +inf
    0x7F800001, 0x7FC00000, 0x7FC00001,          # +sNaN, +qNaN, +qNaN payload 1
]


def test_sort_i32_matches_numpy(oracle_mod):
    rng = np.random.default_rng(3)
    for n in (1, 2, 17, 1000, 4099):
        keys = rng.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
        keys[: min(n, 2)] = [-2**31, 2**31 - 1][: min(n, 2)]
        assert np.array_equal(oracle_mod.sort_i32(keys), np.sort(keys))
        vals = np.arange(n, dtype=np.uint32)
        ko, vo = oracle_mod.sort_i32(keys % 7 - 3, vals)  # heavy ties: stability
        order = np.argsort(keys % 7 - 3, kind="stable")
        assert np.array_equal(ko, (keys % 7 - 3)[order]) and np.array_equal(vo, vals[order])


def test_sort_i32_ternary_words_order_statistics(oracle_mod):
    for word in itertools.product((-1, 0, 1), repeat=6):
        assert oracle_mod.sort_i32(np.array(word, dtype=np.int32)).tolist() == order_statistics(word)


def test_sort_f32_finite_matches_numpy(oracle_mod):
    rng = np.random.default_rng(4)
    for n in (1, 33, 5000):
        keys = (rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, size=n)).astype(np.float32)
        keys = keys[keys != 0]  # no zeros of either sign: numpy's order is then totalOrder
        assert np.array_equal(oracle_mod.sort_f32(keys).view(np.uint32), np.sort(keys).view(np.uint32))


def test_sort_f32_total_order_fixture(oracle_mod):
    want = np.array(TOTAL_ORDER_F32_BITS, dtype=np.uint32)
    rng = np.random.default_rng(5)
    for _ in range(20):
        perm = rng.permutation(want.size)
        got = oracle_mod.sort_f32(want[perm].view(np.float32)).view(np.uint32)
        assert got.tolist() == want.tolist()


def test_sort_f32_signed_zeros_stable(oracle_mod):
    keys = np.array([0.0, -0.0, 0.0, -0.0, -0.0, 1.0, -1.0], dtype=np.float32)
    vals = np.arange(keys.size, dtype=np.uint32)
    ko, vo = oracle_mod.sort_f32(keys, vals)
    assert ko.view(np.uint32).tolist() == _f32_bits([-1.0, -0.0, -0.0, -0.0, 0.0, 0.0, 1.0]).tolist()
    assert vo.tolist() == [6, 1, 3, 4, 0, 2, 5]


# ------------------------------------------------- colored prefix sums


def test_colored_prefix_sums_matches_numpy(oracle_mod):
    """Against numpy: per color, a cumulative sum over the elements of that
    color (uint32 wrap-around), scattered back to their positions."""
    rng = np.random.default_rng(6)
    for n, d in [(1, 1), (10, 3), (1000, 16), (5000, 32), (4097, 2)]:
        vals = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        cols = rng.integers(0, d, size=n).astype(np.uint8)
        want = np.empty(n, dtype=np.uint32)
        for c in range(d):
            idx = np.flatnonzero(cols == c)
            want[idx] = np.cumsum(vals[idx], dtype=np.uint32)
        assert np.array_equal(oracle_mod.colored_prefix_sums(vals, cols, d), want)


def test_colored_prefix_sums_special_cases(oracle_mod):
    # one color: the ordinary inclusive prefix sum
    vals = np.arange(1, 101, dtype=np.uint32)
    assert oracle_mod.colored_prefix_sums(vals, np.zeros(100, np.uint8), 1).tolist() == \
        [k * (k + 1) // 2 for k in range(1, 101)]
    # every element its own color: the values themselves
    assert oracle_mod.colored_prefix_sums(vals[:8], np.arange(8, dtype=np.uint8), 8).tolist() == list(range(1, 9))
    # brute force on tiny inputs: out[i] = sum of v[j], j <= i, same color
    for word in itertools.product((0, 1, 2), repeat=5):
        cols = np.array(word, dtype=np.uint8)
        v = np.array([3, 5, 7, 11, 13], dtype=np.uint32)
        want = [int(sum(v[j] for j in range(i + 1) if cols[j] == cols[i])) for i in range(5)]
        assert oracle_mod.colored_prefix_sums(v, cols, 3).tolist() == want
    # colors at or above d count as d - 1
    assert oracle_mod.colored_prefix_sums(np.ones(4, np.uint32), np.array([0, 5, 1, 9], np.uint8), 2).tolist() == \
        [1, 1, 2, 3]


# ------------------------------------------------------------------ u64 keys

U64_PROBES = (0, 1, 2**32 - 1, 2**32, 2**32 + 1, 2**63, 2**64 - 1)


def test_sort_u64_words_order_statistics(oracle_mod):
    """Every word of length 4 over keys that differ only in the high half, only
    in the low half, or in both, against the counting definition."""
    for word in itertools.product(U64_PROBES, repeat=4):
        assert oracle_mod.sort_u64(np.array(word, dtype=np.uint64)).tolist() == order_statistics(word)


def test_sort_u64_matches_numpy(oracle_mod):
    rng = np.random.default_rng(11)
    for n in (0, 1, 2, 1000, 4097):
        hi = rng.integers(0, 5, size=n, dtype=np.uint64)  # heavy ties in the high half
        lo = rng.integers(0, 2**32, size=n, dtype=np.uint64)
        for keys in ((hi << np.uint64(32)) | lo, (lo << np.uint64(32)) | hi,
                     rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)):
            assert np.array_equal(oracle_mod.sort_u64(keys), np.sort(keys))


# ---------------------------------------------------------------- planted mistakes

MUTANTS = {
    # ties in the pair merge taken from the right: no longer stable
    "unstable_pairs": ("if (sk[i] <= sk[j]) {", "if (sk[i] < sk[j]) {"),
    # right tail of a merge dropped: elements lost
    "drop_tail": ("    while (j < hi)\n        dst[o++] = src[j++];\n", ""),
    # merge_runs ties go to the highest run
    "merge_ties_high_run": ("kin[cur[r]] < kin[cur[best]]", "kin[cur[r]] <= kin[cur[best]]"),
    # descending comparison
    "descending": ("if (src[i] <= src[j])", "if (src[i] >= src[j])"),
    # right half sorted from one past the split: its first element is skipped
    "skip_split_element": ("msort_keys(a, tmp, mid, hi);", "msort_keys(a, tmp, mid + 1, hi);"),
    # int32 keys compared as unsigned
    "i32_unsigned": ("return (int32_t)a <= (int32_t)b;", "return a <= b;"),
    # negative floats ordered by increasing magnitude
    "f32_negatives_ascending": ("return sa ? ma >= mb : ma <= mb;", "return ma <= mb;"),
    # u64 keys compared by their low halves only
    "u64_low_half_only": ("        if (x <= y)\n", "        if ((uint32_t)x <= (uint32_t)y)\n"),
    # u64 keys compared by their high halves only
    "u64_high_half_only": ("        if (x <= y)\n", "        if ((x >> 32) <= (y >> 32))\n"),
    # sortedness check that accepts everything
    "is_sorted_always_true": ("        if (keys[i - 1] > keys[i])\n            return 0;\n",
                              "        if (keys[i - 1] > keys[i])\n            return 1;\n"),
    # sortedness check that never looks at the last pair
    "is_sorted_skips_last_pair": ("for (uint64_t i = 1; i < n; i++)\n        if (keys[i - 1] > keys[i])",
                                  "for (uint64_t i = 1; i + 1 < n; i++)\n        if (keys[i - 1] > keys[i])"),
    # sortedness check that never looks at the first pair
    "is_sorted_skips_first_pair": ("for (uint64_t i = 1; i < n; i++)\n        if (keys[i - 1] > keys[i])",
                                   "for (uint64_t i = 2; i < n; i++)\n        if (keys[i - 1] > keys[i])"),
    # colored prefix sums made exclusive (each output misses its own value)
    "cps_exclusive": ("        run[c] += values[i];\n        out[i] = run[c];\n",
                      "        out[i] = run[c];\n        run[c] += values[i];\n"),
    # colors out of range folded into color 0 instead of d - 1
    "cps_clamp_to_zero": ("colors[i] < d ? colors[i] : d - 1", "colors[i] < d ? colors[i] : 0"),
    # one running total shared by every color
    "cps_one_total": ("        run[c] += values[i];\n", "        run[0] += values[i];\n"),
}


def _pins_pass(lib) -> bool:
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)

    def p(a):
        return a.ctypes.data_as(u32p)

    ok = True
    # sort pin: ternary words of length 6 against order statistics
    for word in itertools.product((0, 1, 2), repeat=6):
        k = np.array(word, dtype=np.uint32)
        o = np.empty_like(k)
        lib.oracle_sort_u32(p(k), p(o), ctypes.c_uint64(k.size))
        if o.tolist() != order_statistics(word):
            ok = False
            break
    # stability pin
    if ok:
        keys, vals = workloads.pairs_u32("distinct16", 2000, seed=1)
        ko, vo = np.empty_like(keys), np.empty_like(vals)
        lib.oracle_sort_pairs_u32(p(keys), p(vals), p(ko), p(vo), ctypes.c_uint64(keys.size))
        order = np.argsort(keys, kind="stable")
        ok = np.array_equal(ko, keys[order]) and np.array_equal(vo, vals[order])
    # merge pin
    if ok:
        keys, offs = workloads.sorted_runs([7, 0, 9, 4], seed=3, dist="dups")
        vals = np.arange(keys.size, dtype=np.uint32)
        ko, vo = np.empty_like(keys), np.empty_like(vals)
        lib.oracle_merge_runs(p(keys), p(vals), offs.ctypes.data_as(u64p), ctypes.c_uint32(4), p(ko), p(vo))
        ek, ev = _stable_concat_sort(keys, vals)
        ok = np.array_equal(ko, ek) and np.array_equal(vo, ev)
    # typed pins: int32 against numpy, float32 against the totalOrder fixture
    if ok:
        keys = np.array([5, -3, 2**31 - 1, -2**31, 0, -1, 7], dtype=np.int32).view(np.uint32)
        ko = np.empty_like(keys)
        lib.oracle_sort_typed(1, p(keys), None, p(ko), None, ctypes.c_uint64(keys.size))
        ok = np.array_equal(ko.view(np.int32), np.sort(keys.view(np.int32)))
    if ok:
        want = np.array(TOTAL_ORDER_F32_BITS, dtype=np.uint32)
        keys = want[::-1].copy()
        ko = np.empty_like(keys)
        lib.oracle_sort_typed(2, p(keys), None, p(ko), None, ctypes.c_uint64(keys.size))
        ok = np.array_equal(ko, want)
    # u64 keys: words over keys differing in either half
    if ok:
        u64 = ctypes.POINTER(ctypes.c_uint64)
        for word in itertools.product((1, 2**32, 2**32 + 2, 3), repeat=4):
            k = np.array(word, dtype=np.uint64)
            o = np.empty_like(k)
            lib.oracle_sort_u64(k.ctypes.data_as(u64), o.ctypes.data_as(u64), ctypes.c_uint64(4))
            if o.tolist() != order_statistics(word):
                return False
    # sortedness check: ternary words against the order-statistic definition,
    # and one inversion at the first, a middle and the last pair
    if ok:
        for word in itertools.product((0, 1, 2), repeat=5):
            k = np.array(word, dtype=np.uint32)
            if bool(lib.oracle_is_sorted_u32(p(k), ctypes.c_uint64(5))) != (list(word) == order_statistics(word)):
                return False
        inc = np.arange(10, 20, dtype=np.uint32)
        for i in (0, 4, 8):
            bad = inc.copy()
            bad[i], bad[i + 1] = bad[i + 1], bad[i]
            if lib.oracle_is_sorted_u32(p(bad), ctypes.c_uint64(bad.size)):
                return False
    # colored prefix sums: brute force over ternary color words, with colors
    # 2 and 3 folded into the last color of d = 2 half the time
    if ok:
        u8p = ctypes.POINTER(ctypes.c_uint8)
        v = np.array([3, 5, 7, 11, 13], dtype=np.uint32)
        for word in itertools.product((0, 1, 3), repeat=5):
            cols = np.array(word, dtype=np.uint8)
            for d in (2, 4):
                eff = np.minimum(cols, d - 1)
                want = [int(sum(v[j] for j in range(i + 1) if eff[j] == eff[i])) for i in range(5)]
                o = np.empty_like(v)
                lib.oracle_colored_prefix_sums(p(v), cols.ctypes.data_as(u8p), p(o), ctypes.c_uint64(5),
                                               ctypes.c_uint32(d))
                if o.tolist() != want:
                    return False
    return ok


def _build_variant(tmp_path, name, src_text):
    import oracle.build as ob

    src = tmp_path / f"{name}.c"
    src.write_text(src_text)
    out = tmp_path / f"lib{name}.so"
    ob.build(out=str(out), src=str(src))
    lib = ctypes.CDLL(str(out))
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_sort_u32.argtypes = [u32p, u32p, ctypes.c_uint64]
    lib.oracle_sort_pairs_u32.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_uint64]
    lib.oracle_merge_runs.argtypes = [u32p, u32p, u64p, ctypes.c_uint32, u32p, u32p]
    lib.oracle_sort_typed.argtypes = [ctypes.c_int, u32p, u32p, u32p, u32p, ctypes.c_uint64]
    lib.oracle_colored_prefix_sums.argtypes = [u32p, ctypes.POINTER(ctypes.c_uint8), u32p, ctypes.c_uint64,
                                               ctypes.c_uint32]
    lib.oracle_sort_u64.argtypes = [u64p, u64p, ctypes.c_uint64]
    lib.oracle_is_sorted_u32.argtypes = [u32p, ctypes.c_uint64]
    lib.oracle_is_sorted_u32.restype = ctypes.c_int
    return lib


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_planted_mistakes_are_caught(tmp_path):
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bcf_oracle.c")
    text = open(here).read()
    assert _pins_pass(_build_variant(tmp_path, "pristine", text))
    for name, (old, new) in MUTANTS.items():
        assert old in text, f"mutant {name} no longer applies"
        lib = _build_variant(tmp_path, name, text.replace(old, new, 1))
        assert not _pins_pass(lib), f"planted mistake {name!r} was not caught"
