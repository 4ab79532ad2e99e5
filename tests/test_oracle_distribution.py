"""Pins for the oracle of the distribution step (Sec. 3.2 "Distribution",
Lemma 1; Sec. 3.3 "Duplicate keys", BCFMergesortPB).

The oracle is checked against what the paper and the mathematics fix, not
against its own formula:

* a hand-worked example from the paper's description (two runs, t = 2, P = 2,
  with and without pivot buckets), stored under tests/golden/;
* exact quantiles: with every key of equal-length runs a candidate (t = run
  length), the splitters are order statistics and P buckets of distinct keys
  hold exactly n / P keys each;
* Lemma 1's bound on the bucket size for distinct keys;
* invariants: a permutation of the input, buckets in increasing key order,
  every piece a contiguous slice of its run in run order, pivot buckets
  holding only their splitter's key;
* special cases: P = 1 and s = 1 are the identity, all-equal keys fill one
  bucket (plain) or one pivot bucket (PB);
* planted mistakes in copies of the oracle source must each fail a pin.
"""

import ctypes
import json
import math
import os
import shutil

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "distribution_small.json")


def _check_invariants(keys, off, P, pb, out, piece, spl):
    """Invariants every correct distribution satisfies (independent of how
    buckets are found): returns a list of violated properties."""
    bad = []
    s = len(off) - 1
    nb = 2 * P - 1 if pb else P
    n = int(off[-1])
    if piece.size != nb * s + 1 or int(piece[0]) != 0 or int(piece[-1]) != n or np.any(np.diff(piece.astype(np.int64)) < 0):
        return ["piece offsets"]
    if sorted(out.tolist()) != sorted(keys.tolist()):
        bad.append("permutation")
    # pieces: run r is tiled in order by its pieces of buckets 0..nb-1
    for r in range(s):
        pos = int(off[r])
        for b in range(nb):
            a, e = int(piece[b * s + r]), int(piece[b * s + r + 1])
            if not np.array_equal(out[a:e], keys[pos:pos + (e - a)]):
                bad.append(f"piece ({b},{r}) not the next slice of its run")
                break
            pos += e - a
        if pos != int(off[r + 1]):
            bad.append(f"run {r} not covered by its pieces")
    # buckets in strictly increasing key order (every key of a bucket is below
    # every key of any later nonempty bucket)
    prev_max = None
    for b in range(nb):
        seg = out[int(piece[b * s]):int(piece[(b + 1) * s])]
        if seg.size == 0:
            continue
        if prev_max is not None and int(seg.min()) <= prev_max:
            bad.append(f"bucket {b} overlaps an earlier bucket")
        prev_max = int(seg.max())
    # bucket contents against the splitters
    F = [int(x) for x in spl]
    if F != sorted(F):
        bad.append("splitters not sorted")
    for b in range(nb):
        seg = out[int(piece[b * s]):int(piece[(b + 1) * s])].tolist()
        if not pb:
            lo = F[b - 1] if b > 0 else None
            hi = F[b] if b < P - 1 else None
            if any((lo is not None and x <= lo) or (hi is not None and x > hi) for x in seg):
                bad.append(f"bucket {b} outside (F[b-1], F[b]]")
        elif b % 2 == 1:
            c = b // 2
            if any(x != F[c] for x in seg):
                bad.append(f"pivot bucket {b} holds a key other than F[{c}]")
        else:
            c = b // 2
            lo = F[c - 1] if c > 0 else None
            hi = F[c] if c < P - 1 else None
            if any((lo is not None and x <= lo) or (hi is not None and x >= hi) for x in seg):
                bad.append(f"bucket {b} outside (F[c-1], F[c])")
    return bad


def test_golden_hand_example():
    with open(GOLDEN) as f:
        g = json.load(f)
    keys = np.array(g["keys"], dtype=np.uint32)
    off = np.array(g["run_offsets"], dtype=np.uint64)
    for case in g["cases"]:
        out, piece, spl = oracle.distribute_runs(keys, off, case["P"], case["t"], case["pivot_buckets"])
        assert spl.tolist() == case["splitters"], case["name"]
        assert out.tolist() == case["out"], case["name"]
        assert piece.tolist() == case["piece_offsets"], case["name"]


@pytest.mark.parametrize("s,L,P", [(4, 64, 4), (8, 32, 16), (3, 96, 6), (16, 16, 8), (1, 128, 32)])
def test_exact_quantiles_when_every_key_is_a_candidate(s, L, P):
    rng = np.random.default_rng(s * 1000 + L + P)
    n = s * L
    assert n % P == 0
    vals = rng.choice(1 << 32, size=n, replace=False).astype(np.uint32)  # distinct keys
    keys = np.concatenate([np.sort(vals[r * L:(r + 1) * L]) for r in range(s)])
    off = np.arange(0, n + 1, L, dtype=np.uint64)
    out, piece, spl = oracle.distribute_runs(keys, off, P, L, False)
    srt = np.sort(keys)
    # splitter c is the ((c+1) n / P)-th smallest key
    assert spl.tolist() == [int(srt[(c + 1) * n // P - 1]) for c in range(P - 1)]
    sizes = np.diff(piece[::s].astype(np.int64))
    assert sizes.tolist() == [n // P] * P
    assert _check_invariants(keys, off, P, False, out, piece, spl) == []


@pytest.mark.parametrize("s,L,P,t", [(8, 4096, 8, 8), (16, 1024, 32, 32), (32, 512, 16, 16), (4, 8192, 64, 64),
                                     (64, 256, 8, 8), (16, 1000, 16, 4)])
def test_lemma1_bucket_bound_distinct_keys(s, L, P, t):
    """Lemma 1: with distinct keys each bucket holds at most
    s*ceil(N/(st)) + ceil(st/P)*ceil(N/(st)) keys."""
    rng = np.random.default_rng(7 * s + L + P + t)
    n = s * L
    vals = rng.choice(1 << 32, size=n, replace=False).astype(np.uint32)
    keys = np.concatenate([np.sort(vals[r * L:(r + 1) * L]) for r in range(s)])
    off = np.arange(0, n + 1, L, dtype=np.uint64)
    out, piece, spl = oracle.distribute_runs(keys, off, P, t, False)
    bound = s * math.ceil(n / (s * t)) + math.ceil(s * t / P) * math.ceil(n / (s * t))
    sizes = np.diff(piece[::s].astype(np.int64))
    assert sizes.max() <= bound
    assert sizes.sum() == n
    assert _check_invariants(keys, off, P, False, out, piece, spl) == []


@pytest.mark.parametrize("pb", [False, True])
@pytest.mark.parametrize("dist", ["uniform", "dups"])
def test_invariants_uneven_and_empty_runs(pb, dist):
    sizes = [0, 1, 7, 300, 0, 2048, 33, 5, 0, 999]
    keys, off = workloads.sorted_runs(sizes, seed=3, dist=dist)
    for P, t in [(1, 1), (2, 3), (5, 4), (16, 16), (40, 7)]:
        out, piece, spl = oracle.distribute_runs(keys, off, P, t, pb)
        assert _check_invariants(keys, off, P, pb, out, piece, spl) == [], (P, t)


def test_identity_cases():
    keys, off = workloads.sorted_runs([100, 0, 57, 300], seed=5)
    out, piece, spl = oracle.distribute_runs(keys, off, 1, 8, False)
    assert np.array_equal(out, keys) and piece.tolist() == off.tolist() and spl.size == 0
    one = np.sort(workloads.draws_u32(9, 1000))
    for pb in (False, True):
        out, piece, _ = oracle.distribute_runs(one, np.array([0, 1000], dtype=np.uint64), 8, 8, pb)
        assert np.array_equal(out, one)


def test_all_equal_keys_one_bucket_or_one_pivot_bucket():
    keys = np.full(4 * 50, 77, dtype=np.uint32)
    off = np.arange(0, 201, 50, dtype=np.uint64)
    s, P = 4, 8
    out, piece, spl = oracle.distribute_runs(keys, off, P, 8, False)
    sizes = np.diff(piece[::s].astype(np.int64))
    assert sizes.tolist() == [200] + [0] * (P - 1)  # x <= F[0] = x: all in bucket 0
    out, piece, spl = oracle.distribute_runs(keys, off, P, 8, True)
    sizes = np.diff(piece[::s].astype(np.int64))
    assert sizes.tolist() == [0, 200] + [0] * (2 * P - 3)  # all in the pivot bucket of F[0]


def test_zero_one_keys_pivot_buckets():
    """The paper's 0-1 input: with pivot buckets every key lands in the pivot
    bucket of its value once both values are splitters."""
    rng = np.random.default_rng(11)
    s, L, P = 8, 256, 4
    keys = np.concatenate([np.sort(rng.integers(0, 2, L)).astype(np.uint32) for _ in range(s)])
    off = np.arange(0, s * L + 1, L, dtype=np.uint64)
    out, piece, spl = oracle.distribute_runs(keys, off, P, P, True)
    assert _check_invariants(keys, off, P, True, out, piece, spl) == []
    assert np.array_equal(out, np.sort(keys))  # two distinct values: buckets alone sort them


# ---------------------------------------------------------------- planted mistakes

MUTANTS = {
    # candidate at the first key of each chunk instead of the last
    "candidate_index": ("cand[k++] = keys[off[r] + (e ? e - 1 : 0)];",
                        "cand[k++] = keys[off[r] + ((uint64_t)j * L) / t];"),
    # splitter one place later in S
    "splitter_index": ("F[c] = m ? S[e ? e - 1 : 0] : 0;", "F[c] = m ? S[e < m ? e : m - 1] : 0;"),
    # bucket c as [F[c-1], F[c]) (ties to the upper bucket)
    "bucket_ties": ("        if (F[mid] < x)\n", "        if (F[mid] <= x)\n"),
    # pivot bucket placed before its open bucket
    "pivot_order": ("b = 2 * lt + 1; /* F[lt]", "b = 2 * lt; /* F[lt]"),
    # pieces ordered run-major instead of bucket-major
    "run_major": ("cnt[b * s + r]++;", "cnt[(uint64_t)r * nb + b]++;"),
}


def _variant_distribute(tmp_path, name, text):
    import oracle.build as ob

    src = tmp_path / f"{name}.c"
    src.write_text(text)
    out = tmp_path / f"lib{name}.so"
    ob.build(out=str(out), src=str(src))
    lib = ctypes.CDLL(str(out))
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_distribute_runs.argtypes = [u32p, u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_int, u32p, u64p, u32p]

    def run(keys, off, P, t, pb):
        s = off.size - 1
        nb = 2 * P - 1 if pb else P
        o = np.empty_like(keys)
        piece = np.empty(nb * s + 1, dtype=np.uint64)
        spl = np.empty(max(P - 1, 1), dtype=np.uint32)
        p32 = lambda a: a.ctypes.data_as(u32p)  # noqa: E731
        lib.oracle_distribute_runs(p32(keys), off.ctypes.data_as(u64p), s, P, t, int(pb), p32(o),
                                   piece.ctypes.data_as(u64p), p32(spl))
        return o, piece, spl[: P - 1]

    return run


def _pins_pass(run):
    with open(GOLDEN) as f:
        g = json.load(f)
    keys = np.array(g["keys"], dtype=np.uint32)
    off = np.array(g["run_offsets"], dtype=np.uint64)
    for case in g["cases"]:
        out, piece, spl = run(keys, off, case["P"], case["t"], case["pivot_buckets"])
        if out.tolist() != case["out"] or piece.tolist() != case["piece_offsets"] or spl.tolist() != case["splitters"]:
            return False
    rng = np.random.default_rng(5)
    s, L, P = 4, 64, 4
    vals = rng.choice(1 << 32, size=s * L, replace=False).astype(np.uint32)
    keys = np.concatenate([np.sort(vals[r * L:(r + 1) * L]) for r in range(s)])
    off = np.arange(0, s * L + 1, L, dtype=np.uint64)
    out, piece, spl = run(keys, off, P, L, False)
    if np.diff(piece[::s].astype(np.int64)).tolist() != [s * L // P] * P:
        return False
    for pb in (False, True):
        k2, o2 = workloads.sorted_runs([0, 7, 300, 33, 999], seed=3, dist="dups")
        out, piece, spl = run(k2, o2, 5, 4, pb)
        if _check_invariants(k2, o2, 5, pb, out, piece, spl):
            return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_planted_mistakes_are_caught(tmp_path):
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bcf_oracle.c")
    text = open(here).read()
    assert _pins_pass(_variant_distribute(tmp_path, "pristine", text))
    for name, (old, new) in MUTANTS.items():
        assert old in text, f"mutant {name} no longer applies"
        run = _variant_distribute(tmp_path, name, text.replace(old, new, 1))
        assert not _pins_pass(run), f"planted mistake {name!r} was not caught"
