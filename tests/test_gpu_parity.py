"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact equality.  Every configuration up to
its full size (2^26 keys in five distributions, 2^28 stable pairs) is compared
element by element with the oracle (at full size the oracle runs its chunked
form on the host cores).  Only the largest size the ABI takes (2^32 - 1) is
checked by properties that determine the result completely, computed on the
device: nondecreasing keys, equal multiset, sampled order statistics and, for
pairs, stability.
"""

import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

T = 4096
EDGE_SIZES = [1, 2, 3, 63, 64, 65, 127, 4095, 4096, 4097, 8191, 8192, 8193, 3 * 4096 + 123,
              5 * 4096, 65535, 65536, 65537, 100_003]


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def bcf():
    import paper_1306_5076_amd as bcf
    from paper_1306_5076_amd import _native

    _native.load()
    return bcf


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def first_diff(got, want):
    idx = np.flatnonzero(got != want)
    return None if idx.size == 0 else (int(idx[0]), int(got[idx[0]]), int(want[idx[0]]))


# ------------------------------------------------------------------ sort_u32


@pytest.mark.parametrize("n", EDGE_SIZES)
def test_sort_edge_sizes(torch_dev, bcf, n):
    torch, dev = torch_dev
    keys = workloads.keys_u32("uniform", n, seed=n)
    got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
    assert first_diff(got, oracle.sort_u32(keys)) is None


def test_sort_empty(torch_dev, bcf):
    torch, dev = torch_dev
    out = bcf.sort_u32(torch.empty(0, dtype=torch.uint32, device=dev))
    assert out.numel() == 0


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_sort_2p16_uniform(torch_dev, bcf, seed):
    torch, dev = torch_dev
    keys = workloads.keys_u32("uniform", 1 << 16, seed=seed)
    got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
    assert first_diff(got, oracle.sort_u32(keys)) is None


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS + workloads.PAPER_DISTRIBUTIONS)
def test_sort_distributions_1m(torch_dev, bcf, dist):
    torch, dev = torch_dev
    keys = workloads.keys_u32(dist, (1 << 20) + 77, seed=2)
    got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
    assert first_diff(got, oracle.sort_u32(keys)) is None


def test_sort_keys_equal_to_padding_value(torch_dev, bcf):
    torch, dev = torch_dev
    keys = workloads.keys_u32("uniform", 3 * T + 17, seed=4)
    keys[::3] = 0xFFFFFFFF
    keys[1::7] = 0
    got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
    assert first_diff(got, oracle.sort_u32(keys)) is None


def test_sort_in_place(torch_dev, bcf):
    torch, dev = torch_dev
    for n in (T - 1, 9 * T + 5, 1 << 18):
        keys = workloads.keys_u32("zipf", n, seed=6)
        t = to_dev(torch, dev, keys)
        bcf.sort_u32(t, out=t)
        assert first_diff(t.cpu().numpy(), oracle.sort_u32(keys)) is None


def test_sort_on_side_stream(torch_dev, bcf):
    torch, dev = torch_dev
    keys = workloads.keys_u32("uniform", 300_000, seed=9)
    s = torch.cuda.Stream(device=dev)
    src = to_dev(torch, dev, keys)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        out = bcf.sort_u32(src, stream=s)
    torch.cuda.current_stream(dev).wait_stream(s)
    assert first_diff(out.cpu().numpy(), oracle.sort_u32(keys)) is None


# host threads for the oracle at full sizes (chunk sorts + pairwise merge tree)
ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_sort_2p26_full_size(torch_dev, bcf, dist):
    """The headline configuration, element by element against the oracle, in
    the launch configuration the benchmark times (default tuning)."""
    torch, dev = torch_dev
    n = 1 << 26
    print(f"sort_u32 2^26 {dist}", flush=True)
    keys = workloads.keys_u32(dist, n, seed=1)
    got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
    assert first_diff(got, oracle.sort_u32_chunked(keys, ORACLE_THREADS)) is None


# ------------------------------------------------------------------ pairs


@pytest.mark.parametrize("n", [1, 5, 4095, 4096, 4097, 3 * 4096 + 123, 65536 + 3])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "paper_01"])
def test_pairs_vs_oracle(torch_dev, bcf, n, dist):
    torch, dev = torch_dev
    keys = workloads.keys_u32(dist, n, seed=n + 1)
    vals = workloads.draws_u32(77, n)  # arbitrary values
    ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, keys), to_dev(torch, dev, vals))
    wk, wv = oracle.sort_pairs_u32(keys, vals)
    assert first_diff(ko.cpu().numpy(), wk) is None
    assert first_diff(vo.cpu().numpy(), wv) is None


@pytest.mark.parametrize("dist", ["uniform", "zipf", "distinct16", "paper_dups"])
def test_pairs_1m_stable(torch_dev, bcf, dist):
    torch, dev = torch_dev
    keys, vals = workloads.pairs_u32(dist, (1 << 20) + 5, seed=3)
    ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, keys), to_dev(torch, dev, vals))
    wk, wv = oracle.sort_pairs_u32(keys, vals)
    assert first_diff(ko.cpu().numpy(), wk) is None
    assert first_diff(vo.cpu().numpy(), wv) is None


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_pairs_2p28_full_size(torch_dev, bcf, dist):
    torch, dev = torch_dev
    n = 1 << 28
    keys, vals = workloads.pairs_u32(dist, n, seed=1)
    ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, keys), to_dev(torch, dev, vals))
    ko, vo = ko.cpu().numpy(), vo.cpu().numpy()
    # element by element against the oracle's stable pair sort
    wk, wv = oracle.sort_pairs_u32_chunked(keys, vals, ORACLE_THREADS)
    assert first_diff(ko, wk) is None
    assert first_diff(vo, wv) is None
    # stability: value = original index, so within equal keys values increase
    same = ko[1:] == ko[:-1]
    assert np.all(vo[1:][same] > vo[:-1][same])


# --------------------------------------------------- the largest size the ABI takes
#
# n = 2^32 - 1 keys (16 GiB; pairs 32 GiB) fits in the GPU's HBM with the
# output and the scratch.  The oracle cannot sort this many keys on the host
# in a test, so the checks are properties that fix the result, computed on the
# device chunk by chunk: the output is nondecreasing; it is a permutation of the
# input (per-bucket counts of the top 16 bits, sum and sum of squares modulo
# 2^64); sampled outputs equal the order statistics of the input by their
# definition (count of smaller and of not-larger keys); for pairs, every output
# key is the input key at the output value's index (value = original index)
# and equal keys keep increasing values (stability).

N_MAX = (1 << 32) - 1
CH = 1 << 28


def _signed(x, torch):
    """uint32 -> int32 with the unsigned order (flip the sign bit)."""
    return x.view(torch.int32) ^ torch.tensor(-(1 << 31), dtype=torch.int32, device=x.device)


def _chunks(n):
    return [(lo, min(n, lo + CH)) for lo in range(0, n, CH)]


def _multiset_digest(x, torch):
    hist = torch.zeros(65536, dtype=torch.int64, device=x.device)
    s1 = torch.zeros((), dtype=torch.int64, device=x.device)
    s2 = torch.zeros((), dtype=torch.int64, device=x.device)
    for lo, hi in _chunks(x.numel()):
        v = x[lo:hi].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        hist += torch.bincount(v >> 16, minlength=65536)
        s1 += v.sum()
        s2 += (v * v).sum()  # wraps modulo 2^64
    return hist.cpu().numpy(), int(s1), int(s2)


def _need_bytes(torch, nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")


def test_max_size_keys(torch_dev, bcf):
    torch, dev = torch_dev
    n = N_MAX
    _need_bytes(torch, 3 * 4 * n + (4 << 30))
    keys = workloads.draws_u32_torch(7, n, dev)
    out = bcf.sort_u32(keys)
    torch.cuda.synchronize()
    for lo, hi in _chunks(n):
        s = _signed(out[lo:min(n, hi + 1)], torch)
        assert bool((s[1:] >= s[:-1]).all()), lo
    assert [np.array_equal(a, b) if isinstance(a, np.ndarray) else a == b
            for a, b in zip(_multiset_digest(out, torch), _multiset_digest(keys, torch))] == [True] * 3
    # order statistics at sampled ranks, by definition
    sk = _signed(keys, torch)
    for i in (0, 1, 12345, n // 3, n // 2 + 7, n - 2, n - 1):
        v = _signed(out[i:i + 1], torch)
        less = int((sk < v).sum())
        not_larger = int((sk <= v).sum())
        assert less <= i < not_larger, i


def test_max_size_pairs(torch_dev, bcf):
    torch, dev = torch_dev
    n = N_MAX
    _need_bytes(torch, 6 * 4 * n + (4 << 30))
    keys = workloads.keys_u32_torch("zipf", n, dev, seed=5)  # heavy duplicates: stability matters
    vals = torch.empty(n, dtype=torch.int32, device=dev)
    for lo, hi in _chunks(n):  # value = original index
        vals[lo:hi] = torch.arange(lo, hi, dtype=torch.int64, device=dev).to(torch.int32)
    vals = vals.view(torch.uint32)
    ko, vo = bcf.sort_pairs_u32(keys, vals)
    torch.cuda.synchronize()
    sk_in = keys.view(torch.int32)
    for lo, hi in _chunks(n):
        k = _signed(ko[lo:min(n, hi + 1)], torch)
        v = vo[lo:min(n, hi + 1)].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert bool((k[1:] >= k[:-1]).all()), lo
        same = k[1:] == k[:-1]
        assert bool((v[1:][same] > v[:-1][same]).all()), lo  # stable
        # output pair (k, v) is input element v
        assert bool((sk_in.index_select(0, v) == ko[lo:min(n, hi + 1)].view(torch.int32)).all()), lo
    # the values are a permutation of 0 .. n-1: counts per top-16-bit bucket, sums
    hist, s1, s2 = _multiset_digest(vo, torch)
    assert np.all(hist[:-1] == 65536) and hist[-1] == 65535
    assert s1 == n * (n - 1) // 2
    assert s2 == ((n - 1) * n * (2 * n - 1) // 6 + (1 << 63)) % (1 << 64) - (1 << 63)


# ------------------------------------------------------------------ merge_runs


@pytest.mark.parametrize(
    "sizes",
    [[5000], [0, 0, 7], [4096, 4096], [1, 10000], [10000, 1], [3, 0, 9000, 0, 4097],
     [700] * 17, [8192, 123, 5000, 4096 * 3 + 1, 0, 77, 4096], list(range(0, 3400, 200))],
)
@pytest.mark.parametrize("pairs", [False, True])
def test_merge_runs_vs_oracle(torch_dev, bcf, sizes, pairs):
    torch, dev = torch_dev
    keys, offs = workloads.sorted_runs(sizes, seed=len(sizes), dist="dups")
    vals = workloads.draws_u32(5, keys.size) if pairs else None
    kd = to_dev(torch, dev, keys)
    if pairs:
        ko, vo = bcf.merge_runs(kd, offs, vals=to_dev(torch, dev, vals))
        wk, wv = oracle.merge_runs(keys, offs, vals)
        assert first_diff(ko.cpu().numpy(), wk) is None
        assert first_diff(vo.cpu().numpy(), wv) is None
    else:
        ko = bcf.merge_runs(kd, offs)
        assert first_diff(ko.cpu().numpy(), oracle.merge_runs(keys, offs)) is None


def test_merge_runs_in_place(torch_dev, bcf):
    torch, dev = torch_dev
    for sizes in ([3000, 4000], [100, 200, 300], [5000] * 5):
        keys, offs = workloads.sorted_runs(sizes, seed=2)
        t = to_dev(torch, dev, keys)
        bcf.merge_runs(t, offs, keys_out=t)
        assert first_diff(t.cpu().numpy(), oracle.merge_runs(keys, offs)) is None


@pytest.mark.parametrize("alias", ["keys", "vals", "both"])
def test_merge_runs_pairs_in_place(torch_dev, bcf, alias):
    """Key/value merges where the keys, the values or both are merged in place;
    2 and 5 runs take an odd number of passes, 3 runs an even number."""
    torch, dev = torch_dev
    for sizes in ([3000, 4000], [100, 200, 300], [5000] * 5):
        keys, offs = workloads.sorted_runs(sizes, seed=3, dist="dups")
        vals = workloads.draws_u32(11, keys.size)
        kd, vd = to_dev(torch, dev, keys), to_dev(torch, dev, vals)
        ko = kd if alias in ("keys", "both") else torch.empty_like(kd)
        vo = vd if alias in ("vals", "both") else torch.empty_like(vd)
        bcf.merge_runs(kd, offs, vals=vd, keys_out=ko, vals_out=vo)
        wk, wv = oracle.merge_runs(keys, offs, vals)
        assert first_diff(ko.cpu().numpy(), wk) is None
        assert first_diff(vo.cpu().numpy(), wv) is None


def test_merge_runs_large(torch_dev, bcf):
    torch, dev = torch_dev
    sizes = workloads.segment_sizes(64, lo=1 << 10, hi=1 << 20, seed=4)
    keys, offs = workloads.sorted_runs(sizes, seed=8)
    got = bcf.merge_runs(to_dev(torch, dev, keys), offs).cpu().numpy()
    assert first_diff(got, oracle.merge_runs(keys, offs)) is None


# ------------------------------------------------------------------ segmented


@pytest.mark.parametrize(
    "sizes",
    [[0], [1], [0, 1, 2, 0, 3], [4096, 4097, 1, 0, 8192], [12345], [31, 4096 * 5 + 3, 64, 100000, 0, 2],
     [64] * 200],
)
def test_segmented_vs_oracle(torch_dev, bcf, sizes):
    torch, dev = torch_dev
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    keys = workloads.keys_u32("uniform", int(offs[-1]), seed=len(sizes))
    got = bcf.segmented_sort(to_dev(torch, dev, keys), offs).cpu().numpy()
    assert first_diff(got, oracle.segmented_sort(keys, offs)) is None


def test_segmented_log_uniform_batch(torch_dev, bcf):
    torch, dev = torch_dev
    sizes = workloads.segment_sizes(1000, lo=32, hi=1 << 16, seed=1)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    keys = workloads.keys_u32("uniform", int(offs[-1]), seed=1)
    got = bcf.segmented_sort(to_dev(torch, dev, keys), offs).cpu().numpy()
    assert first_diff(got, oracle.segmented_sort(keys, offs)) is None


# ------------------------------------------------------------------ profiling / errors


@pytest.mark.parametrize("fused", [1, 0])
def test_profile_records_every_launch(torch_dev, bcf, fused):
    torch, dev = torch_dev
    n = 1 << 20
    keys = to_dev(torch, dev, workloads.keys_u32("uniform", n))
    with bcf.tuning(fused_partition=fused, merge_fan_in=2):
        bcf.profile_collect()
        bcf.profile_enable(True)
        bcf.sort_u32(keys)
        bcf.profile_enable(False)
        st = bcf.profile_collect()
        merges = bcf.sort_passes(n) - 1
    assert st["block_sort_keys"]["launches"] == 1
    assert st["merge_keys"]["launches"] == merges
    # keys take the one-tile-per-wave merge by default: with fused partitions
    # it searches its own splits and there is no partition launch
    assert st.get("partition_keys", {"launches": 0})["launches"] == (0 if fused else merges)
    assert st["merge_keys"]["bytes"] == pytest.approx(merges * 8.0 * n)
    assert all(v["total_ms"] > 0 for v in st.values())


def test_profile_records_four_way_passes(torch_dev, bcf):
    # 2^20 keys in 32 runs of 32768: four-way passes to 8 and 2 runs, then one binary pass
    torch, dev = torch_dev
    n = 1 << 20
    keys = to_dev(torch, dev, workloads.keys_u32("uniform", n))
    with bcf.tuning(merge_fan_in=4):
        bcf.profile_collect()
        bcf.profile_enable(True)
        bcf.sort_u32(keys)
        bcf.profile_enable(False)
        st = bcf.profile_collect()
        assert bcf.sort_passes(n) == 4
    assert st["block_sort_keys"]["launches"] == 1
    assert st["cuts4_keys"]["launches"] == 2 and st["merge4_keys"]["launches"] == 2
    assert st["merge_keys"]["launches"] == 1
    assert st["merge4_keys"]["bytes"] == pytest.approx(2 * 8.0 * n)


# run counts around the four-way grouping: 3 runs (the fourth empty), 4, 5
# (a four-way pass, then a binary one), ragged last groups of 1..4 runs, many
# passes; with wave tiles (runs of 4096) and group tiles (runs of 32768)
FOUR_WAY_CASES = [(3 * 4096, 1), (3 * 4096 - 7, 1), (4 * 4096, 1), (5 * 4096 + 1, 1), (16 * 4096 + 4095, 1),
                  (17 * 4096, 1), (61 * 4096 + 100, 1), (300007, 1), (3 * 32768 + 5, 3), (9 * 32768, 3),
                  ((1 << 20) + 3, 0), (5 * (1 << 19) + 77, 0), ((1 << 22) + 12345, 0)]


@pytest.mark.parametrize("n,block_sort", FOUR_WAY_CASES)
def test_four_way_merge_passes(torch_dev, bcf, n, block_sort):
    """Sorts whose merge passes take four runs at a time (the default for keys)
    against the oracle, over distributions with many, few and no ties."""
    torch, dev = torch_dev
    with bcf.tuning(block_sort=block_sort, merge_fan_in=4):
        for dist in ("uniform", "distinct16", "sorted", "reverse", "zipf"):
            keys = workloads.keys_u32(dist, n, seed=n % 1000 + 3)
            got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
            assert first_diff(got, oracle.sort_u32(keys)) is None, (n, block_sort, dist)


@pytest.mark.parametrize("knobs", [{"tile_samples": 0}, {"sampled_partition": 0}, {"merge_variant": 1},
                                   {"merge_variant": 0}, {"fused_partition": 0}, {"block_sort": 2}])
def test_four_way_with_other_knobs(torch_dev, bcf, knobs):
    """Fan-in 4 forced together with other knobs: without tile samples the cut
    searches start from block samples; without samples the passes are binary;
    the last (binary) pass under every merge kernel; ShearSort runs of 4096."""
    torch, dev = torch_dev
    n = 5 * (1 << 18) + 4097  # 41 runs of 32768: four-way 41 -> 11 -> 3 -> 1
    with bcf.tuning(merge_fan_in=4, **knobs):
        passes = bcf.sort_passes(n)
        for dist in ("uniform", "distinct16"):
            keys = workloads.keys_u32(dist, n, seed=17)
            got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
            assert first_diff(got, oracle.sort_u32(keys)) is None, (knobs, dist)
    if knobs.get("sampled_partition") == 0:
        assert passes == 1 + 6  # binary: 41 runs -> 6 passes
    elif knobs.get("block_sort") == 2:
        assert passes == 1 + 5  # 322 runs of 4096 -> 81 -> 21 -> 6 -> 2 -> 1
    else:
        assert passes == 1 + 3


@pytest.mark.parametrize("nt", [0, 1])
def test_four_way_same_as_binary(torch_dev, bcf, nt):
    """Four-way and binary merge passes give the same bytes (keys, all equal
    keys, two values, and a sort large enough for nontemporal traffic)."""
    torch, dev = torch_dev
    for n, make in [((1 << 21) + 999, lambda n: workloads.keys_u32("uniform", n, seed=9)),
                    (400000, lambda n: np.full(n, 7, dtype=np.uint32)),
                    (700001, lambda n: (workloads.draws_u32(4, n) & 1).astype(np.uint32)),
                    ((1 << 26) + 4097, None)]:
        if make is None:
            kd = workloads.draws_u32_torch(12, n, dev)
        else:
            kd = to_dev(torch, dev, make(n))
        with bcf.tuning(merge_fan_in=4, nontemporal=nt):
            a = bcf.sort_u32(kd)
        with bcf.tuning(merge_fan_in=2, nontemporal=nt):
            b = bcf.sort_u32(kd)
        assert bool(torch.equal(a, b)), n
        if make is not None:
            assert first_diff(a.cpu().numpy(), oracle.sort_u32(make(n))) is None, n


# key/value sorts: runs of 4096 (wave tiles) or 16384 (group tiles of four waves)
FOUR_WAY_PAIR_CASES = [(3 * 4096, 1), (3 * 4096 - 7, 1), (5 * 4096 + 1, 1), (17 * 4096, 1), (61 * 4096 + 100, 1),
                       (3 * 16384 + 5, 3), (9 * 16384, 3), ((1 << 20) + 3, 0), ((1 << 22) + 12345, 0)]


@pytest.mark.parametrize("n,block_sort", FOUR_WAY_PAIR_CASES)
def test_four_way_pair_passes(torch_dev, bcf, n, block_sort):
    """Stable key/value sorts whose merge passes take four runs at a time
    against the oracle; the value is the input index, so equal keys must leave
    in input order (many, few and no ties)."""
    torch, dev = torch_dev
    print(f"four-way pairs: n={n} block_sort={block_sort}", flush=True)
    with bcf.tuning(block_sort=block_sort, merge_fan_in=4):
        for dist in ("uniform", "distinct16", "sorted", "reverse", "zipf"):
            keys, vals = workloads.pairs_u32(dist, n, seed=n % 1000 + 5)
            ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, keys), to_dev(torch, dev, vals))
            wk, wv = oracle.sort_pairs_u32(keys, vals)
            assert first_diff(ko.cpu().numpy(), wk) is None, (n, block_sort, dist)
            assert first_diff(vo.cpu().numpy(), wv) is None, (n, block_sort, dist)


@pytest.mark.parametrize("nt", [0, 1])
def test_four_way_pairs_same_as_binary(torch_dev, bcf, nt):
    """Four-way and binary key/value passes give the same bytes (random values;
    all keys equal; two key values; a sort large enough for nontemporal
    traffic)."""
    torch, dev = torch_dev
    for n, kmake in [((1 << 21) + 999, lambda n: workloads.keys_u32("uniform", n, seed=9)),
                     (400000, lambda n: np.full(n, 7, dtype=np.uint32)),
                     (700001, lambda n: (workloads.draws_u32(4, n) & 1).astype(np.uint32)),
                     ((1 << 25) + 4097, None)]:
        print(f"four-way pairs vs binary: n={n} nt={nt}", flush=True)
        if kmake is None:
            kd = workloads.draws_u32_torch(12, n, dev)
        else:
            kd = to_dev(torch, dev, kmake(n))
        vd = workloads.draws_u32_torch(13, n, dev)
        with bcf.tuning(merge_fan_in=4, nontemporal=nt):
            ak, av = bcf.sort_pairs_u32(kd, vd)
        with bcf.tuning(merge_fan_in=2, nontemporal=nt):
            bk, bv = bcf.sort_pairs_u32(kd, vd)
        assert bool(torch.equal(ak, bk)) and bool(torch.equal(av, bv)), n
        if kmake is not None:
            wk, wv = oracle.sort_pairs_u32(kmake(n), vd.cpu().numpy())
            assert first_diff(ak.cpu().numpy(), wk) is None and first_diff(av.cpu().numpy(), wv) is None, n


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("variant", [2, 3])
def test_fused_partition_parity(torch_dev, bcf, fused, variant):
    """Merge passes with in-kernel split searches against the oracle (keys and
    pairs, duplicates, ragged sizes spanning many passes)."""
    torch, dev = torch_dev
    with bcf.tuning(fused_partition=fused, merge_variant=variant):
        for n, dist in [((1 << 21) + 4097, "uniform"), ((1 << 20) + 3, "distinct16"), (600001, "zipf")]:
            keys = workloads.keys_u32(dist, n, seed=n)
            got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
            assert first_diff(got, oracle.sort_u32(keys)) is None, (n, dist)
            kk, vv = workloads.pairs_u32(dist, n, seed=n + 1)
            ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, kk), to_dev(torch, dev, vv))
            wk, wv = oracle.sort_pairs_u32(kk, vv)
            assert first_diff(ko.cpu().numpy(), wk) is None and first_diff(vo.cpu().numpy(), wv) is None


@pytest.mark.parametrize("pairs", [False, True])
def test_group_tile_boundaries(torch_dev, bcf, pairs):
    # sizes around one and several block-sort runs (group tiles)
    torch, dev = torch_dev
    R = bcf.run_keys(pairs)
    for n in (R - 1, R, R + 1, 2 * R - 4096, 3 * R + 4097, 5 * R + 1):
        keys, vals = workloads.pairs_u32("zipf", n, seed=n)
        if pairs:
            ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, keys), to_dev(torch, dev, vals))
            wk, wv = oracle.sort_pairs_u32(keys, vals)
            assert first_diff(ko.cpu().numpy(), wk) is None and first_diff(vo.cpu().numpy(), wv) is None
        else:
            got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
            assert first_diff(got, oracle.sort_u32(keys)) is None


def test_errors_raise(torch_dev, bcf):
    torch, dev = torch_dev
    from paper_1306_5076_amd import BcfError

    keys = to_dev(torch, dev, np.arange(10, dtype=np.uint32))
    with pytest.raises(ValueError):
        bcf.merge_runs(keys, [0, 5, 11])
    with pytest.raises(TypeError):
        bcf.sort_u32(torch.zeros(4, dtype=torch.float32, device=dev))
    with bcf.tuning(check_runs=1):
        bad = to_dev(torch, dev, np.array([1, 2, 3, 9, 4, 5, 6], dtype=np.uint32))
        with pytest.raises(BcfError) as ei:
            bcf.merge_runs(bad, [0, 3, 7])  # second run 9,4,5,6 is not sorted
            torch.cuda.synchronize()
        assert ei.value.status == 5
        good = to_dev(torch, dev, np.array([1, 2, 3, 9, 4, 5, 6], dtype=np.uint32))
        got = bcf.merge_runs(good, [0, 4, 7]).cpu().numpy()
        assert list(got) == [1, 2, 3, 4, 5, 6, 9]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("nt", [0, 1])
def test_merge_kernel_variants(torch_dev, bcf, mode, nt):
    torch, dev = torch_dev
    with bcf.tuning(merge_variant=mode, nontemporal=nt):
        _check_sorts(torch, dev, bcf)


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_block_sort_variants(torch_dev, bcf, variant):
    """Block sorts (wave tiles by merge rounds, wave tiles by the paper's
    ShearSort, group tiles by merge rounds, group tiles of keys by the paper's
    long ShearSort over 8 waves) against the oracle: single partial tile,
    exact tile, ragged multi-tile, partial and full groups, many passes, keys
    and stable pairs (pairs take merge rounds under variant 4)."""
    torch, dev = torch_dev
    with bcf.tuning(block_sort=variant):
        assert bcf.run_keys() == (32768 if variant >= 3 else 4096)
        for n in (1, 100, 4095, 4096, 4097, 3 * 4096 + 17, 32768, 40000, 5 * 32768 + 4099):
            for dist in ("uniform", "distinct16", "reverse"):
                keys = workloads.keys_u32(dist, n, seed=n)
                got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
                assert first_diff(got, oracle.sort_u32(keys)) is None, (n, dist)
                kk, vv = workloads.pairs_u32(dist, n, seed=n + 1)
                ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, kk), to_dev(torch, dev, vv))
                wk, wv = oracle.sort_pairs_u32(kk, vv)
                assert first_diff(ko.cpu().numpy(), wk) is None and first_diff(vo.cpu().numpy(), wv) is None
        _check_sorts(torch, dev, bcf)


def _check_sorts(torch, dev, bcf):
    for n, dist in [((1 << 20) + 3, "uniform"), (7 * 4096 + 5, "zipf")]:
        keys = workloads.keys_u32(dist, n, seed=11)
        got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
        assert first_diff(got, oracle.sort_u32(keys)) is None
        kk, vv = workloads.pairs_u32(dist, n, seed=12)
        ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, kk), to_dev(torch, dev, vv))
        wk, wv = oracle.sort_pairs_u32(kk, vv)
        assert first_diff(ko.cpu().numpy(), wk) is None and first_diff(vo.cpu().numpy(), wv) is None


# ------------------------------------------------------------------ segmented pairs / plans / graphs


@pytest.mark.parametrize(
    "sizes",
    [[0, 1, 2, 0, 3], [4096, 4097, 1, 0, 8192], [31, 4096 * 5 + 3, 64, 100000, 0, 2], [20000, 40000, 70000]],
)
def test_segmented_pairs_vs_oracle(torch_dev, bcf, sizes):
    torch, dev = torch_dev
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    n = int(offs[-1])
    keys = workloads.keys_u32("distinct16", n, seed=3)
    vals = workloads.draws_u32(9, n)
    ko, vo = bcf.segmented_sort(to_dev(torch, dev, keys), offs, vals=to_dev(torch, dev, vals))
    ko, vo = ko.cpu().numpy(), vo.cpu().numpy()
    for s in range(len(sizes)):
        lo, hi = int(offs[s]), int(offs[s + 1])
        wk, wv = oracle.sort_pairs_u32(keys[lo:hi], vals[lo:hi])
        assert first_diff(ko[lo:hi], wk) is None and first_diff(vo[lo:hi], wv) is None


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("sizes", [[3000, 16384 + 100], [20000, 40000, 3 * 16384 + 1]])
def test_segmented_tail_at_allocation_end(torch_dev, bcf, sizes, pairs):
    """Inputs that end exactly where their 16 MiB device allocations end, with
    the last segment's last group tile only partly filled: the waves whose
    sub-tiles lie past the end of the input must not read past it."""
    torch, dev = torch_dev
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    n = int(offs[-1])
    keys = workloads.keys_u32("uniform", n, seed=21)
    vals = workloads.draws_u32(22, n)
    cap = 1 << 22
    kbuf = torch.zeros(cap, dtype=torch.int32, device=dev)
    kbuf[cap - n:].copy_(torch.from_numpy(keys.view(np.int32)))
    kd = kbuf.view(torch.uint32)[cap - n:]
    if pairs:
        vbuf = torch.zeros(cap, dtype=torch.int32, device=dev)
        vbuf[cap - n:].copy_(torch.from_numpy(vals.view(np.int32)))
        ko, vo = bcf.segmented_sort(kd, offs, vals=vbuf.view(torch.uint32)[cap - n:])
        ko, vo = ko.cpu().numpy(), vo.cpu().numpy()
    else:
        ko = bcf.segmented_sort(kd, offs).cpu().numpy()
    for sg in range(len(sizes)):
        lo, hi = int(offs[sg]), int(offs[sg + 1])
        if pairs:
            wk, wv = oracle.sort_pairs_u32(keys[lo:hi], vals[lo:hi])
            assert first_diff(ko[lo:hi], wk) is None and first_diff(vo[lo:hi], wv) is None
        else:
            assert first_diff(ko[lo:hi], oracle.sort_u32(keys[lo:hi])) is None


@pytest.mark.parametrize("sizes", [
    [4096 * 3 + 5], [4096 * 5 + 1], [4096 * 9, 7, 0, 4096 * 17 + 100], [32768 * 3 + 11, 32768 * 5, 1 << 20],
    [1 << 18, 1 << 18, 3, 200000], [12345] * 40 + [4096 * 4 + 1] * 5])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf"])
def test_segmented_four_way_vs_oracle(torch_dev, bcf, sizes, dist):
    """Host-planned segmented sort with fan-in 4 merge steps (groups of four
    runs of a segment merged per pass, the last step binary when two runs are
    left): segments of 3, 5, 9, 17, ... runs, wave and group tiles, ties."""
    torch, dev = torch_dev
    offs = workloads.segment_offsets(sizes)
    keys = workloads.keys_u32(dist, int(offs[-1]), seed=len(sizes) + 3)
    for gmin in (0, 1 << 40):  # group tiles for long segments, or wave tiles only
        with bcf.tuning(merge_fan_in=4, group_min_keys=gmin):
            got = bcf.segmented_sort(to_dev(torch, dev, keys), offs).cpu().numpy()
        assert first_diff(got, oracle.segmented_sort(keys, offs)) is None, (sizes, dist, gmin)


@pytest.mark.parametrize("sizes", [
    [4096 * 3 + 5], [4096 * 9, 7, 0, 4096 * 17 + 100], [16384 * 3 + 11, 16384 * 5, 1 << 20],
    [12345] * 20 + [4096 * 4 + 1] * 3])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf"])
def test_segmented_pairs_four_way_vs_oracle(torch_dev, bcf, sizes, dist):
    """Host-planned stable key/value segmented sort with fan-in 4 steps: the
    value is the input index, so equal keys must keep their order."""
    torch, dev = torch_dev
    print(f"segmented pairs four-way: sizes={sizes[:4]} dist={dist}", flush=True)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    keys = workloads.keys_u32(dist, n, seed=len(sizes) + 13)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.segmented_sort_threads(keys, offs, ORACLE_THREADS, vals=vals)
    for gmin in (0, 1 << 40):
        with bcf.tuning(merge_fan_in=4, group_min_keys=gmin):
            ko, vo = bcf.segmented_sort(to_dev(torch, dev, keys), offs, vals=to_dev(torch, dev, vals))
        assert first_diff(ko.cpu().numpy(), wk) is None, (sizes[:4], dist, gmin)
        assert first_diff(vo.cpu().numpy(), wv) is None, (sizes[:4], dist, gmin)


def test_segmented_four_way_plan_graph_and_tuning(torch_dev, bcf):
    """A plan uploaded with fan-in 4 steps replays in a graph on new data and
    keeps its fan-in when executed under another tuning."""
    torch, dev = torch_dev
    sizes = workloads.segment_sizes(200, lo=32, hi=1 << 18, seed=7)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    with bcf.tuning(merge_fan_in=4):
        plan = bcf.SegmentedPlan(offs, dev)
    kin = torch.empty(n, dtype=torch.uint32, device=dev)
    kout = torch.empty_like(kin)
    with bcf.tuning(merge_fan_in=2):
        graph = plan.capture(kin, kout)
    for rep in range(3):
        keys = workloads.keys_u32("zipf" if rep % 2 else "uniform", n, seed=40 + rep)
        kin.copy_(torch.from_numpy(keys))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert first_diff(kout.cpu().numpy(), oracle.segmented_sort(keys, offs)) is None, rep


@pytest.mark.parametrize("group_min", [4097, 1000000000, 0])
def test_segmented_group_threshold(torch_dev, bcf, group_min):
    # the same segments block-sorted in group tiles or in wave tiles
    torch, dev = torch_dev
    sizes = [5000, 40000, 100000, 4096, 32768, 32769]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    keys = workloads.keys_u32("zipf", int(offs[-1]), seed=2)
    with bcf.tuning(group_min_keys=group_min):
        got = bcf.segmented_sort(to_dev(torch, dev, keys), offs).cpu().numpy()
    assert first_diff(got, oracle.segmented_sort(keys, offs)) is None


@pytest.mark.parametrize("pairs", [False, True])
def test_segmented_plan_graph_replay(torch_dev, bcf, pairs):
    torch, dev = torch_dev
    sizes = workloads.segment_sizes(300, lo=32, hi=1 << 16, seed=5)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    n = int(offs[-1])
    plan = bcf.SegmentedPlan(offs, dev, pairs=pairs)
    kin = torch.empty(n, dtype=torch.uint32, device=dev)
    kout = torch.empty_like(kin)
    vin = torch.empty_like(kin) if pairs else None
    vout = torch.empty_like(kin) if pairs else None
    graph = plan.capture(kin, kout, vin, vout)
    for rep in range(3):  # new data each replay, eager work in between
        keys = workloads.keys_u32("uniform", n, seed=100 + rep)
        vals = workloads.draws_u32(200 + rep, n)
        kin.copy_(torch.from_numpy(keys))
        if pairs:
            vin.copy_(torch.from_numpy(vals))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        eager = bcf.segmented_sort(kin, offs, vals=vin) if pairs else bcf.segmented_sort(kin, offs)
        torch.cuda.synchronize()
        if pairs:
            assert torch.equal(kout, eager[0]) and torch.equal(vout, eager[1])
            wk = np.concatenate([oracle.sort_pairs_u32(keys[int(offs[s]):int(offs[s + 1])],
                                                       vals[int(offs[s]):int(offs[s + 1])])[1]
                                 for s in range(len(sizes))])
            assert first_diff(vout.cpu().numpy(), wk) is None
        else:
            assert torch.equal(kout, eager)
            assert first_diff(kout.cpu().numpy(), oracle.segmented_sort(keys, offs)) is None


@pytest.mark.parametrize("gmin_upload,gmin_run", [(4097, 1_000_000_000), (1_000_000_000, 4097)])
def test_segmented_plan_keeps_its_tuning(torch_dev, bcf, gmin_upload, gmin_run):
    """A plan uploaded under one group threshold and executed under another
    runs the plan it uploaded (group or wave tiles as at upload time)."""
    torch, dev = torch_dev
    sizes = [5000, 40000, 100000, 4096, 32768, 32769, 7]
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    keys = workloads.keys_u32("uniform", n, seed=31)
    with bcf.tuning(group_min_keys=gmin_upload):
        plan = bcf.SegmentedPlan(offs, dev)
    kin = to_dev(torch, dev, keys)
    kout = torch.empty_like(kin)
    with bcf.tuning(group_min_keys=gmin_run):
        plan.run(kin, kout)
        torch.cuda.synchronize()
    assert first_diff(kout.cpu().numpy(), oracle.segmented_sort(keys, offs)) is None


@pytest.mark.parametrize("knobs", [{"tile_samples": 0}, {"nontemporal": 0}, {"sampled_partition": 0}])
def test_sort_switches(torch_dev, bcf, knobs):
    torch, dev = torch_dev
    with bcf.tuning(**knobs):
        _check_sorts_2(torch, dev, bcf)


def _check_sorts_2(torch, dev, bcf):
    for n, dist in [((1 << 21) + 3, "uniform"), (9 * 32768 + 5, "zipf"), (1 << 20, "distinct16")]:
        keys = workloads.keys_u32(dist, n, seed=21)
        got = bcf.sort_u32(to_dev(torch, dev, keys)).cpu().numpy()
        assert first_diff(got, oracle.sort_u32(keys)) is None
        kk, vv = workloads.pairs_u32(dist, n, seed=22)
        ko, vo = bcf.sort_pairs_u32(to_dev(torch, dev, kk), to_dev(torch, dev, vv))
        wk, wv = oracle.sort_pairs_u32(kk, vv)
        assert first_diff(ko.cpu().numpy(), wk) is None and first_diff(vo.cpu().numpy(), wv) is None


# ------------------------------------------------------------ other key types

F32_SPECIAL_BITS = np.array([0xFFC00000, 0xFF800000, 0xFF7FFFFF, 0xBF800000, 0x80000001, 0x80000000, 0x00000000,
                             0x00000001, 0x3F800000, 0x7F7FFFFF, 0x7F800000, 0x7FC00000], dtype=np.uint32)


def _typed_keys(kind, n, dist, seed):
    bits = workloads.draws_u32(seed, n)
    if dist == "special":  # special values only: heavy ties across -NaN .. +NaN, both zeros
        bits = F32_SPECIAL_BITS[bits % F32_SPECIAL_BITS.size] if kind == "f32" else (bits % 9).astype(np.uint32) - 4
    return bits.view(np.float32 if kind == "f32" else np.int32)


@pytest.mark.parametrize("kind", ["i32", "f32"])
@pytest.mark.parametrize("n", [1, 4096, 4097, 100003, (1 << 20) + 7, 1 << 25, (1 << 25) + 5])
def test_typed_sorts_vs_oracle(torch_dev, bcf, kind, n):
    torch, dev = torch_dev
    sort = bcf.sort_f32 if kind == "f32" else bcf.sort_i32
    ref = oracle.sort_f32 if kind == "f32" else oracle.sort_i32
    for dist in ("bits", "special"):
        keys = _typed_keys(kind, n, dist, seed=n % 977)
        got = sort(torch.from_numpy(keys).to(dev)).cpu().numpy()
        assert first_diff(got.view(np.uint32), ref(keys).view(np.uint32)) is None, (kind, n, dist)


@pytest.mark.parametrize("kind", ["i32", "f32"])
@pytest.mark.parametrize("n", [3, 4096 * 3 + 1, (1 << 20) + 7])
def test_typed_pairs_stable_vs_oracle(torch_dev, bcf, kind, n):
    torch, dev = torch_dev
    sort = bcf.sort_pairs_f32 if kind == "f32" else bcf.sort_pairs_i32
    ref = oracle.sort_f32 if kind == "f32" else oracle.sort_i32
    keys = _typed_keys(kind, n, "special", seed=7)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = sort(torch.from_numpy(keys).to(dev), to_dev(torch, dev, vals))
    wk, wv = ref(keys, vals)
    assert first_diff(ko.cpu().numpy().view(np.uint32), wk.view(np.uint32)) is None
    assert first_diff(vo.cpu().numpy(), wv) is None


@pytest.mark.parametrize("knobs", [
    {"block_sort": 1}, {"block_sort": 3, "merge_fan_in": 4}, {"merge_fan_in": 2, "fused_partition": 0},
    {"merge_fan_in": 2, "merge_variant": 1}, {"block_sort": 2}, {"block_sort": 4, "merge_fan_in": 4}])
def test_typed_sorts_under_tunings(torch_dev, bcf, knobs):
    """The key maps are fused into the first and the last pass: every block
    sort and merge kernel that can be either (wave or group tiles, binary or
    four-way last pass, fused or separate split search) maps correctly."""
    torch, dev = torch_dev
    n = 3 * (1 << 18) + 11
    for kind in ("i32", "f32"):
        keys = _typed_keys(kind, n, "bits", seed=5)
        ref = oracle.sort_f32 if kind == "f32" else oracle.sort_i32
        sort = bcf.sort_f32 if kind == "f32" else bcf.sort_i32
        with bcf.tuning(**knobs):
            got = sort(torch.from_numpy(keys).to(dev)).cpu().numpy()
        assert first_diff(got.view(np.uint32), ref(keys).view(np.uint32)) is None, (kind, knobs)
        psort = bcf.sort_pairs_f32 if kind == "f32" else bcf.sort_pairs_i32
        vals = np.arange(n, dtype=np.uint32)
        with bcf.tuning(**knobs):
            ko, vo = psort(torch.from_numpy(keys).to(dev), to_dev(torch, dev, vals))
        wk, wv = ref(keys, vals)
        assert first_diff(ko.cpu().numpy().view(np.uint32), wk.view(np.uint32)) is None, (kind, knobs)
        assert first_diff(vo.cpu().numpy(), wv) is None, (kind, knobs)


def test_typed_sort_in_place_and_errors(torch_dev, bcf):
    torch, dev = torch_dev
    keys = _typed_keys("f32", 50000, "bits", seed=3)
    t = torch.from_numpy(keys).to(dev)
    bcf.sort_f32(t, out=t)
    assert first_diff(t.cpu().numpy().view(np.uint32), oracle.sort_f32(keys).view(np.uint32)) is None
    # a view that is not 16-byte aligned (scalar map kernel) and a size with a tail
    base = torch.from_numpy(_typed_keys("i32", 70003, "bits", seed=4)).to(dev)
    view = base[1:]
    want = oracle.sort_i32(view.cpu().numpy())
    out = torch.empty(70005, dtype=torch.int32, device=dev)[3:]  # 70002, like the view
    bcf.sort_i32(view, out=out)
    assert first_diff(out.cpu().numpy(), want) is None
    with pytest.raises(TypeError):
        bcf.sort_f32(torch.zeros(10, dtype=torch.int32, device=dev))
    with pytest.raises(TypeError):
        bcf.sort_i32(torch.zeros(10, dtype=torch.float32, device=dev))
