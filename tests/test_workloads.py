"""Seeded generators: deterministic, slice-consistent, and shaped as stated."""

import numpy as np
import pytest

import workloads


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: the first outputs of the published reference
    # generator (state += gamma; mix) are 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4.
    x = np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64)
    got = workloads.splitmix64(x)
    assert int(got[0]) == 0xE220A8397B1DCDAF
    assert int(got[1]) == 0x6E789E6AA1B965F4


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS + workloads.PAPER_DISTRIBUTIONS)
def test_deterministic(dist):
    a = workloads.keys_u32(dist, 5000, seed=7)
    b = workloads.keys_u32(dist, 5000, seed=7)
    c = workloads.keys_u32(dist, 5000, seed=8)
    assert a.dtype == np.uint32 and a.shape == (5000,)
    assert np.array_equal(a, b)
    if dist not in ("paper_01",):
        assert not np.array_equal(a, c)


def test_slices_consistent():
    full = workloads.draws_u32(3, 10000)
    part = workloads.draws_u32(3, 100, start=5000)
    assert np.array_equal(full[5000:5100], part)


def test_shapes_of_distributions():
    n = 1 << 16
    s = workloads.keys_u32("sorted", n)
    assert np.all(s[1:] >= s[:-1])
    # the uniform sample itself, in order: same multiset and ties
    assert np.array_equal(np.sort(workloads.keys_u32("uniform", n)), s)
    r = workloads.keys_u32("reverse", n)
    assert np.array_equal(r, s[::-1])
    assert len(np.unique(workloads.keys_u32("distinct16", n))) == 16
    z = workloads.keys_u32("zipf", n)
    _, counts = np.unique(z, return_counts=True)
    # rank 1 has probability 1/H(1.2, 2^20) ~ 0.20
    assert 0.15 < counts.max() / n < 0.25
    assert set(np.unique(workloads.keys_u32("paper_01", n)).tolist()) == {0, 1}
    d = workloads.keys_u32("paper_distinct", n)
    assert np.array_equal(np.sort(d), np.arange(1, n + 1, dtype=np.uint32))
    assert workloads.keys_u32("paper_random", n).max() <= 10**6


def test_segment_sizes_and_runs():
    sz = workloads.segment_sizes(10000)
    assert sz.min() >= 32 and sz.max() <= 1 << 20
    keys, offs = workloads.sorted_runs([5, 0, 7], seed=1)
    assert offs.tolist() == [0, 5, 5, 12]
    assert np.all(np.diff(keys[:5].astype(np.int64)) >= 0)
    assert np.all(np.diff(keys[5:].astype(np.int64)) >= 0)


def test_torch_twin_bit_identical():
    import torch

    for seed, n, start in [(1, 1000, 0), (7, 4097, 123), (2**31 + 5, 333, 10**9)]:
        a = workloads.draws_u32(seed, n, start=start)
        b = workloads.draws_u32_torch(seed, n, "cpu", start=start, chunk=1000).numpy()
        assert np.array_equal(a, b)
    assert np.array_equal(workloads.segment_offsets([3, 0, 2]), np.array([0, 3, 3, 5], dtype=np.uint64))
    for dist in ("uniform", "zipf"):
        a = workloads.keys_u32(dist, 5000, seed=4)
        b = workloads.keys_u32_torch(dist, 5000, "cpu", seed=4, chunk=1024).numpy()
        assert np.array_equal(a, b), dist


@pytest.mark.parametrize("m", [1, 5, 32, 40, 256])
def test_colored_inputs_twins_and_range(m):
    v, c = workloads.colored_u32(70001, m, seed=9)
    assert v.dtype == np.uint32 and c.dtype == np.uint8
    assert int(c.max()) < m
    if m <= 40:  # every color drawn
        assert np.unique(c).size == m
    tv, tc = workloads.colored_u32_torch(70001, m, "cpu", seed=9, chunk=30000)
    assert np.array_equal(tv.numpy(), v) and np.array_equal(tc.numpy(), c)


def test_u64_keys_distributions():
    n = 50_000
    for dist in workloads.U64_DISTRIBUTIONS:
        k = workloads.keys_u64(dist, n, seed=4)
        assert k.dtype == np.uint64 and k.size == n
        assert np.array_equal(k, workloads.keys_u64(dist, n, seed=4))  # reproducible
    hi = lambda a: a >> np.uint64(32)
    lo = lambda a: a & np.uint64(0xFFFFFFFF)
    assert np.unique(hi(workloads.keys_u64("hi16", n))).size == 16
    assert np.unique(lo(workloads.keys_u64("lo16", n))).size == 16
    s = workloads.keys_u64("sorted", n)
    assert np.all(np.diff(hi(s).astype(np.int64)) >= 0)
    assert np.array_equal(hi(workloads.keys_u64("reverse", n)), hi(s)[::-1])
    assert set(workloads.keys_u64("extremes", n).tolist()) == {0, 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1}
