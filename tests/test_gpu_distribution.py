"""GPU parity of the distribution step (Sec. 3.2 "Distribution"; pivot
buckets of Sec. 3.3, BCFMergesortPB) through the C ABI against the CPU oracle.

Integer work: the rearranged keys, the piece offsets and the splitters must
equal the oracle's bit for bit.  Inputs are seeded sorted runs: uneven and
empty runs, uniform keys, heavy duplicates, the paper's 0-1 and
defined-duplicates sets, and the full size of 2^26 keys in 256 runs.
"""

import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "distribution_small.json")


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


def _run_both(bcf, torch_dev, keys, off, P, t, pb):
    torch, dev = torch_dev
    print(f"distribute n={int(off[-1])} s={off.size - 1} P={P} t={t} pb={pb}", flush=True)
    kd = torch.from_numpy(np.ascontiguousarray(keys)).to(dev)
    out, pieces, spl = bcf.distribute_runs(kd, off, P, t, pivot_buckets=pb)
    torch.cuda.synchronize()
    got = (out.cpu().numpy(), pieces.cpu().numpy().astype(np.uint64), spl.cpu().numpy())
    want = oracle.distribute_runs(keys, off, P, t, pb)
    return got, want


def _assert_same(got, want):
    (go, gp, gs), (wo, wp, ws) = got, want
    assert np.array_equal(gs, ws), "splitters differ"
    assert np.array_equal(gp, wp), f"piece offsets differ at {np.flatnonzero(gp != wp)[:5]}"
    bad = np.flatnonzero(go != wo)
    assert bad.size == 0, f"keys differ at {bad[:5]}"


def test_golden_example(bcf, torch_dev):
    with open(GOLDEN) as f:
        g = json.load(f)
    keys = np.array(g["keys"], dtype=np.uint32)
    off = np.array(g["run_offsets"], dtype=np.uint64)
    for case in g["cases"]:
        got, want = _run_both(bcf, torch_dev, keys, off, case["P"], case["t"], case["pivot_buckets"])
        _assert_same(got, want)
        assert got[0].tolist() == case["out"]


@pytest.mark.parametrize("pb", [False, True])
@pytest.mark.parametrize("dist", ["uniform", "dups"])
@pytest.mark.parametrize("P,t", [(1, 1), (2, 3), (7, 5), (64, 64), (300, 17)])
def test_uneven_and_empty_runs(bcf, torch_dev, dist, P, t, pb):
    sizes = [0, 1, 7, 4095, 0, 4096, 4097, 33, 5, 0, 12345, 999, 65536]
    keys, off = workloads.sorted_runs(sizes, seed=11, dist=dist)
    _assert_same(*_run_both(bcf, torch_dev, keys, off, P, t, pb))


@pytest.mark.parametrize("pb", [False, True])
def test_paper_duplicate_sets(bcf, torch_dev, pb):
    rng = np.random.default_rng(2)
    s, L = 32, 5000
    # 0-1 keys
    keys = np.concatenate([np.sort(rng.integers(0, 2, L)).astype(np.uint32) for _ in range(s)])
    off = np.arange(0, s * L + 1, L, dtype=np.uint64)
    _assert_same(*_run_both(bcf, torch_dev, keys, off, 16, 16, pb))
    # defined duplicates: k copies of n/k distinct keys
    vals = workloads.draws_u32(4, (s * L) // 8)
    keys = np.repeat(vals, 8)
    perm = rng.permutation(keys.size)
    keys = np.concatenate([np.sort(keys[perm[r * L:(r + 1) * L]]) for r in range(s)])
    _assert_same(*_run_both(bcf, torch_dev, keys, off, 32, 32, pb))
    # all keys equal
    keys = np.full(s * L, 0xFFFFFFFF, dtype=np.uint32)
    _assert_same(*_run_both(bcf, torch_dev, keys, off, 8, 8, pb))


def test_no_keys_and_single_run(bcf, torch_dev):
    torch, dev = torch_dev
    off = np.zeros(5, dtype=np.uint64)  # four empty runs
    kd = torch.empty(0, dtype=torch.uint32, device=dev)
    out, pieces, spl = bcf.distribute_runs(kd, off, 4, 4, pivot_buckets=True)
    torch.cuda.synchronize()
    assert out.numel() == 0 and pieces.cpu().tolist() == [0] * (7 * 4 + 1) and spl.cpu().tolist() == [0, 0, 0]
    keys = np.sort(workloads.draws_u32(3, 100_003))
    one = np.array([0, keys.size], dtype=np.uint64)
    got, want = _run_both(bcf, torch_dev, keys, one, 128, 128, False)
    _assert_same(got, want)
    assert np.array_equal(got[0], keys)


@pytest.mark.parametrize("pb", [False, True])
def test_full_size_2p26_in_256_runs(bcf, torch_dev, pb):
    """2^26 uniform keys in 256 sorted runs of 2^18, P = t = 256: every output
    key, piece offset and splitter against the oracle."""
    keys, off = workloads.sorted_runs([1 << 18] * 256, seed=1)
    got, want = _run_both(bcf, torch_dev, keys, off, 256, 256, pb)
    _assert_same(got, want)


@pytest.mark.parametrize("dist", ["uniform", "dups"])
@pytest.mark.parametrize("in_place", [False, True])
def test_merge_run_groups_matches_per_group_merge(bcf, torch_dev, dist, in_place):
    """Batched merge of groups of runs == the oracle's merge of each group.
    Groups of 3, 1, 0, 5, 5, 2 and 1 runs (one with only empty runs) take 2,
    0, 0, 3, 3, 1 and 0 merge passes of their own (in place, odd counts take
    one more pass, a copy out of the scratch buffer)."""
    torch, dev = torch_dev
    sizes = [0, 5, 4096, 4097, 1, 0, 12345, 300, 65536, 7, 0, 0, 999, 2048, 70000, 3, 0, 0, 40000]
    keys, off = workloads.sorted_runs(sizes, seed=21, dist=dist)
    starts = [0, 3, 4, 4, 9, 14, 16, 17, 19]
    print(f"merge_run_groups {dist} n={keys.size} in_place={in_place}", flush=True)
    kd = torch.from_numpy(keys).to(dev)
    got = bcf.merge_run_groups(kd, off, starts, keys_out=kd if in_place else None).cpu().numpy()
    want = np.empty_like(keys)
    for g in range(len(starts) - 1):
        a, b = starts[g], starts[g + 1]
        lo, hi = int(off[a]), int(off[b])
        want[lo:hi] = oracle.merge_runs(keys[lo:hi], (off[a:b + 1] - off[a]).astype(np.uint64))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pb", [False, True])
@pytest.mark.parametrize("dist,n", [("uniform", 1_000_003), ("distinct16", 1 << 22), ("zipf", 1 << 22),
                                    ("uniform", 1 << 26)])
def test_sort_by_distribution_equals_oracle_sort(bcf, torch_dev, dist, n, pb):
    """Runs, distribution, batched merge of every bucket: the sorted keys."""
    torch, dev = torch_dev
    keys = workloads.keys_u32(dist, n, seed=2)
    print(f"sort_u32_pb {dist} n={n} pb={pb}", flush=True)
    got = bcf.sort_u32_pb(torch.from_numpy(keys).to(dev), P=256, run_keys=1 << 16 if n < (1 << 24) else 1 << 18,
                          pivot_buckets=pb).cpu().numpy()
    assert np.array_equal(got, oracle.sort_u32(keys))
