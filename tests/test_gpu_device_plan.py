"""GPU parity of the calls whose offsets live in device memory and whose launch
plans are computed on the device: bcf_merge_runs, bcf_segmented_sort[_pairs]
and the sort by distribution bcf_sort_u32_pb, against the oracle; graph
replays with offsets changed between replays; invalid device offsets."""

import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1306_5076_amd as bcf
    from paper_1306_5076_amd import _native

    _native.load()
    return torch, torch.device("cuda:0"), bcf


def _dev_offsets(torch, dev, offs):
    return torch.from_numpy(np.asarray(offs, dtype=np.int64)).to(dev)


@pytest.mark.parametrize("sizes", [[5000], [1, 1], [0, 7, 0, 4096, 4097, 0], [4096] * 9,
                                   [100000, 3, 70000, 8192, 1, 65536, 12345],
                                   [1] * 37, [300000, 250000]])
@pytest.mark.parametrize("pairs", [False, True])
def test_merge_runs_device_offsets(env, sizes, pairs):
    torch, dev, bcf = env
    print(f"merge_runs device offsets: sizes={sizes[:8]} pairs={pairs}", flush=True)
    keys, offs = workloads.sorted_runs(sizes, seed=len(sizes) + 7)
    n = keys.size
    kin = torch.from_numpy(keys).to(dev)
    doff = _dev_offsets(torch, dev, offs)
    if pairs:
        vals = np.arange(n, dtype=np.uint32)
        ko, vo = bcf.merge_runs(kin, doff, vals=torch.from_numpy(vals).to(dev))
        wk, wv = oracle.merge_runs(keys, offs, vals=vals)
        assert np.array_equal(ko.cpu().numpy(), wk) and np.array_equal(vo.cpu().numpy(), wv)
    else:
        out = bcf.merge_runs(kin, doff)
        assert np.array_equal(out.cpu().numpy(), oracle.merge_runs(keys, offs))


@pytest.mark.parametrize("sizes", [[5000], [3000, 2000, 9000], [1, 1, 1, 1, 1], [70000, 0, 30000, 4096]])
def test_merge_runs_device_offsets_in_place(env, sizes):
    """In place: an odd number of merge passes takes one more, a copy."""
    torch, dev, bcf = env
    keys, offs = workloads.sorted_runs(sizes, seed=3)
    kin = torch.from_numpy(keys).to(dev)
    doff = _dev_offsets(torch, dev, offs)
    want = oracle.merge_runs(keys, offs)
    bcf.merge_runs(kin, doff, keys_out=kin)
    assert np.array_equal(kin.cpu().numpy(), want)
    vals = np.arange(keys.size, dtype=np.uint32)
    kin = torch.from_numpy(keys).to(dev)
    vin = torch.from_numpy(vals).to(dev)
    wk, wv = oracle.merge_runs(keys, offs, vals=vals)
    bcf.merge_runs(kin, doff, vals=vin, keys_out=kin, vals_out=vin)
    assert np.array_equal(kin.cpu().numpy(), wk) and np.array_equal(vin.cpu().numpy(), wv)


@pytest.mark.parametrize("fan_in", [2, 4])
@pytest.mark.parametrize("k", [3, 4, 5, 16, 17, 64, 200, 1000])
def test_merge_runs_device_offsets_fan_in(env, fan_in, k):
    """bcf_merge_runs under either fan-in (four-way steps over runs of uneven
    length, some empty, ties across runs; then binary ones), keys and stable
    pairs, out of place and in place (an odd level count takes a final copy)."""
    torch, dev, bcf = env
    print(f"merge_runs fan_in={fan_in} k={k}", flush=True)
    rng = np.random.default_rng(k * 10 + fan_in)
    sizes = [int(x) for x in rng.integers(0, 9000, size=k)]
    sizes[k // 2] = 0
    keys, offs = workloads.sorted_runs(sizes, seed=k + 31, dist="dups")
    n = keys.size
    vals = np.arange(n, dtype=np.uint32)
    doff = _dev_offsets(torch, dev, offs)
    wk, wv = oracle.merge_runs(keys, offs, vals=vals)
    with bcf.tuning(merge_fan_in=fan_in):
        out = bcf.merge_runs(torch.from_numpy(keys).to(dev), doff)
        ko, vo = bcf.merge_runs(torch.from_numpy(keys).to(dev), doff, vals=torch.from_numpy(vals).to(dev))
        kin = torch.from_numpy(keys).to(dev)
        vin = torch.from_numpy(vals).to(dev)
        bcf.merge_runs(kin, doff, vals=vin, keys_out=kin, vals_out=vin)
    assert np.array_equal(out.cpu().numpy(), wk)
    assert np.array_equal(ko.cpu().numpy(), wk) and np.array_equal(vo.cpu().numpy(), wv)
    assert np.array_equal(kin.cpu().numpy(), wk) and np.array_equal(vin.cpu().numpy(), wv)


@pytest.mark.parametrize("sizes", [[0], [1], [4096], [4097], [100, 0, 5000, 16384, 16385, 40000, 3],
                                   [70000, 200000, 1, 0, 4096 * 3 + 5], [32768 * 3 + 7]])
@pytest.mark.parametrize("pairs", [False, True])
def test_segmented_device_offsets(env, sizes, pairs):
    torch, dev, bcf = env
    print(f"segmented device offsets: sizes={sizes} pairs={pairs}", flush=True)
    offs = workloads.segment_offsets(np.asarray(sizes))
    n = int(offs[-1])
    keys = workloads.keys_u32("uniform", n, seed=n + 1)
    kin = torch.from_numpy(keys).to(dev)
    doff = _dev_offsets(torch, dev, offs)
    if pairs:
        vals = np.arange(n, dtype=np.uint32)
        ko, vo = bcf.segmented_sort(kin, doff, vals=torch.from_numpy(vals).to(dev))
        wk, wv = oracle.segmented_sort_threads(keys, offs, THREADS, vals=vals)
        assert np.array_equal(ko.cpu().numpy(), wk) and np.array_equal(vo.cpu().numpy(), wv)
    else:
        out = bcf.segmented_sort(kin, doff)
        assert np.array_equal(out.cpu().numpy(), oracle.segmented_sort(keys, offs))


@pytest.mark.parametrize("sizes", [
    [4096 * 3 + 5], [4096 * 5 + 1], [4096 * 9, 7, 0, 4096 * 17 + 100], [32768 * 3 + 11, 32768 * 5, 1 << 20],
    [1 << 18, 1 << 18, 3, 200000], [12345] * 40 + [4096 * 4 + 1] * 5])
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf"])
@pytest.mark.parametrize("pairs", [False, True])
def test_segmented_device_offsets_four_way(env, sizes, dist, pairs):
    """Device-planned segmented sort with fan-in 4 merge steps (four runs of a
    segment per job while more than two remain, then binary): segments of 3,
    5, 9, 17, ... runs, wave and group tiles, ties; equal to the oracle and to
    the host-planned sort under the same tuning."""
    torch, dev, bcf = env
    print(f"segmented device offsets four-way: sizes={sizes[:6]} dist={dist} pairs={pairs}", flush=True)
    offs = workloads.segment_offsets(np.asarray(sizes))
    n = int(offs[-1])
    keys = workloads.keys_u32(dist, n, seed=len(sizes) + 5)
    kin = torch.from_numpy(keys).to(dev)
    doff = _dev_offsets(torch, dev, offs)
    if pairs:
        vals = np.arange(n, dtype=np.uint32)  # value = input index: ties must keep their order
        vin = torch.from_numpy(vals).to(dev)
        wk, wv = oracle.segmented_sort_threads(keys, offs, THREADS, vals=vals)
    else:
        want = oracle.segmented_sort(keys, offs)
    for gmin in (0, 1 << 40):  # group tiles for long segments, or wave tiles only
        with bcf.tuning(merge_fan_in=4, group_min_keys=gmin):
            if pairs:
                dk, dv = bcf.segmented_sort(kin, doff, vals=vin)
                hk, hv = bcf.segmented_sort(kin, offs, vals=vin)
                for gk, gv in ((dk, dv), (hk, hv)):
                    assert np.array_equal(gk.cpu().numpy(), wk), (sizes[:6], dist, gmin)
                    assert np.array_equal(gv.cpu().numpy(), wv), (sizes[:6], dist, gmin)
                continue
            got = bcf.segmented_sort(kin, doff).cpu().numpy()
            host = bcf.segmented_sort(kin, offs).cpu().numpy()
        assert np.array_equal(got, want), (sizes[:6], dist, gmin)
        assert np.array_equal(host, want), (sizes[:6], dist, gmin)


def test_segmented_device_offsets_full_size(env):
    """The configured batch: 10,000 arrays of 32..2^20 keys (log-uniform), keys,
    segment by segment against the oracle."""
    torch, dev, bcf = env
    sizes = workloads.segment_sizes(10_000, lo=32, hi=1 << 20, seed=1)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    print(f"segmented device offsets full size: {n} keys", flush=True)
    kin = workloads.keys_u32_torch("uniform", n, dev, seed=4)
    out = bcf.segmented_sort(kin, _dev_offsets(torch, dev, offs))
    torch.cuda.synchronize()
    want = oracle.segmented_sort_threads(kin.cpu().numpy(), offs, THREADS)
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("pairs,fan_in", [(False, 0), (False, 4), (True, 0), (True, 4)])
def test_segmented_graph_replay_with_new_offsets(env, pairs, fan_in):
    """One captured graph of the device-planned segmented sort, replayed with
    new segment offsets (same total) written into the same device tensor:
    every replay equals the oracle for its own segmentation.  Fan-in 4 keeps
    its per-segment step counts on the device too (segments of 1 to ~60 runs)."""
    torch, dev, bcf = env
    n = 300_000 if fan_in != 4 else 1_500_000
    from paper_1306_5076_amd import _native

    lib = _native.load()
    import ctypes

    kin = torch.empty(n, dtype=torch.uint32, device=dev)
    kout = torch.empty_like(kin)
    vin = torch.arange(n, dtype=torch.int32, device=dev).view(torch.uint32) if pairs else None
    vout = torch.empty_like(kin) if pairs else None
    nseg = 64
    doff = torch.zeros(nseg + 1, dtype=torch.int64, device=dev)
    rng = np.random.default_rng(9)

    def new_offsets():
        cuts = np.sort(rng.integers(0, n + 1, size=nseg - 1))
        return np.concatenate([[0], cuts, [n]]).astype(np.int64)

    offs = new_offsets()
    doff.copy_(torch.from_numpy(offs))
    need = ctypes.c_uint64(0)
    vp = ctypes.c_void_p
    stream = torch.cuda.current_stream(dev)
    if pairs:
        assert lib.bcf_segmented_sort_pairs(None, None, None, None, vp(doff.data_ptr()), nseg, None,
                                            ctypes.byref(need), vp(stream.cuda_stream)) == 0
    else:
        assert lib.bcf_segmented_sort(None, None, vp(doff.data_ptr()), nseg, None, ctypes.byref(need),
                                      vp(stream.cuda_stream)) == 0
    temp = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    tb = ctypes.c_uint64(temp.numel())

    def run(st):
        sh = vp(st.cuda_stream)
        if pairs:
            return lib.bcf_segmented_sort_pairs(vp(kin.data_ptr()), vp(vin.data_ptr()), vp(kout.data_ptr()),
                                                vp(vout.data_ptr()), vp(doff.data_ptr()), nseg, vp(temp.data_ptr()),
                                                ctypes.byref(tb), sh)
        return lib.bcf_segmented_sort(vp(kin.data_ptr()), vp(kout.data_ptr()), vp(doff.data_ptr()), nseg,
                                      vp(temp.data_ptr()), ctypes.byref(tb), sh)

    kin.copy_(workloads.keys_u32_torch("uniform", n, dev, seed=1))
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    # fan-in 4 with wave tiles only: segments of up to ~60 runs of 4096 keys
    with bcf.tuning(merge_fan_in=fan_in, group_min_keys=(1 << 40) if fan_in == 4 else 0):
        with torch.cuda.stream(side):
            assert run(side) == 0  # warm-up outside capture
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            assert run(torch.cuda.current_stream(dev)) == 0
    for rep in range(3):
        offs = new_offsets()
        doff.copy_(torch.from_numpy(offs))
        kin.copy_(workloads.keys_u32_torch("uniform", n, dev, seed=10 + rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        keys = kin.cpu().numpy()
        if pairs:
            vals = np.arange(n, dtype=np.uint32)
            wk, wv = oracle.segmented_sort_threads(keys, offs.astype(np.uint64), THREADS, vals=vals)
            assert np.array_equal(kout.cpu().numpy(), wk), rep
            assert np.array_equal(vout.cpu().numpy(), wv), rep
        else:
            assert np.array_equal(kout.cpu().numpy(), oracle.segmented_sort(keys, offs.astype(np.uint64))), rep


@pytest.mark.parametrize("fan_in", [2, 4])
def test_invalid_device_offsets_write_nothing(env, fan_in):
    """Decreasing device offsets, or a total past the capacity, are found by the
    planner on the device: nothing is written (binary or fan-in 4 steps)."""
    torch, dev, bcf = env
    n = 50_000
    kin = workloads.keys_u32_torch("uniform", n, dev, seed=2)
    out = torch.full_like(kin, 7)
    good = _dev_offsets(torch, dev, [0, 20_000, n])
    from paper_1306_5076_amd import _native
    import ctypes

    lib = _native.load()
    vp = ctypes.c_void_p
    need = ctypes.c_uint64(0)
    assert lib.bcf_segmented_sort(None, None, vp(good.data_ptr()), 2, None, ctypes.byref(need), None) == 0
    temp = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    tb = ctypes.c_uint64(temp.numel())
    for bad in ([0, 30_000, 20_000], [0, 20_000, 10 * n]):
        doff = _dev_offsets(torch, dev, bad)
        sh = vp(torch.cuda.current_stream(dev).cuda_stream)
        with bcf.tuning(merge_fan_in=fan_in):
            assert lib.bcf_segmented_sort(vp(kin.data_ptr()), vp(out.data_ptr()), vp(doff.data_ptr()), 2,
                                          vp(temp.data_ptr()), ctypes.byref(tb), sh) == 0
        torch.cuda.synchronize()
        assert bool((out == 7).all()), bad


@pytest.mark.parametrize("dist", ["uniform", "distinct16", "zipf", "sorted"])
@pytest.mark.parametrize("pivot", [True, False])
@pytest.mark.parametrize("fan_in", [0, 2])
def test_sort_pb_c_abi(env, dist, pivot, fan_in):
    """The sort by distribution through the C ABI (device-planned bucket merge,
    four-way steps over each bucket's 33 pieces by default, or binary ones)
    equals the oracle sort."""
    torch, dev, bcf = env
    n = (1 << 21) + 12345
    keys = workloads.keys_u32(dist, n, seed=5)
    with bcf.tuning(merge_fan_in=fan_in):
        out = bcf.sort_u32_pb(torch.from_numpy(keys).to(dev), P=64, run_keys=1 << 16, pivot_buckets=pivot)
    assert np.array_equal(out.cpu().numpy(), oracle.sort_u32(keys))


def test_sort_pb_c_abi_full_size(env):
    torch, dev, bcf = env
    n = 1 << 26
    kin = workloads.keys_u32_torch("uniform", n, dev, seed=1)
    out = bcf.sort_u32_pb(kin, P=256, run_keys=1 << 18, pivot_buckets=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.sort_u32_chunked(kin.cpu().numpy(), THREADS))
