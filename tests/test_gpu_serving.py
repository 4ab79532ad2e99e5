"""Serving loop (continuous batching) on the GPU: results are the same alone and
in the mix (tolerance 0: integer sort), admission never exceeds the HBM
budget, and requests that arrive while a batch is on the device are batched."""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch

    assert torch.cuda.is_available()
    from paper_1306_5076_amd import serve

    return serve


def _requests(count, seed, hi=1 << 18):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(count):
        n = int(rng.integers(0, hi))
        keys = workloads.keys_u32("zipf" if i % 3 == 0 else "uniform", n, seed=seed * 1000 + i)
        vals = workloads.draws_u32(seed * 7 + i, n) if i % 2 else None
        reqs.append((0.0, keys, vals))
    return reqs


def test_mix_equals_alone(serve):
    reqs = _requests(40, seed=3)
    alone, _, _ = serve.serve_serial(reqs, realtime=False)
    # requests of 2^16 keys and more take the single-sort path, smaller ones share segmented sorts
    with serve.SortServer(hbm_budget=1 << 30, solo_keys=1 << 16) as srv:
        with srv.held():  # everything queues first, then is admitted as one mixed batch
            futs = [srv.submit(k, v) for _, k, v in reqs]
        mixed = [f.result(timeout=120) for f in futs]
        batches = srv.batches
    assert batches == 1
    for (_, k, v), a, m in zip(reqs, alone, mixed):
        if v is None:
            assert np.array_equal(a, m)
            assert np.array_equal(m, oracle.sort_u32(k))
        else:
            assert np.array_equal(a[0], m[0]) and np.array_equal(a[1], m[1])
            wk, wv = oracle.sort_pairs_u32(k, v)
            assert np.array_equal(m[0], wk) and np.array_equal(m[1], wv)


def test_admission_budget(serve):
    budget = 48 << 20
    reqs = _requests(30, seed=5, hi=1 << 20)
    with serve.SortServer(hbm_budget=budget) as srv:
        futs = [srv.submit(k, v) for _, k, v in reqs]
        big = srv.submit(np.zeros(budget, dtype=np.uint32))  # larger than the whole budget
        results = [f.result(timeout=120) for f in futs]
        peak = srv.peak_used
    assert 0 < peak <= budget
    with pytest.raises(MemoryError):
        big.result(timeout=10)
    for (_, k, v), m in zip(reqs, results):
        want = oracle.sort_u32(k) if v is None else oracle.sort_pairs_u32(k, v)[0]
        got = m if v is None else m[0]
        assert np.array_equal(got, want)


def test_serving_benchmark_small(serve):
    out = serve.run_serving_benchmark(count=40, fracs=(0.8,), lo=1 << 10, hi=1 << 18)
    run = out["runs"][0]
    assert run["batched"]["p99_ms"] > 0 and run["serial"]["p99_ms"] > 0
    assert run["batched"]["peak_hbm_bytes"] <= out["hbm_budget_bytes"]


def test_device_requests_mixed_with_host(serve):
    """Device-resident requests (CUDA tensors in, CUDA tensors out) batched
    together with host requests; every result equals the oracle's."""
    import torch

    dev = torch.device("cuda:0")
    reqs = _requests(24, seed=9)
    with serve.SortServer(hbm_budget=1 << 30, solo_keys=1 << 16) as srv:
        with srv.held():
            futs = []
            for i, (_, k, v) in enumerate(reqs):
                if i % 2:
                    kd = torch.from_numpy(k).to(dev)
                    vd = torch.from_numpy(v).to(dev) if v is not None else None
                    futs.append(srv.submit(kd, vd))
                else:
                    futs.append(srv.submit(k, v))
        got = [f.result(timeout=120) for f in futs]
        assert srv.batches == 1
    for i, ((_, k, v), g) in enumerate(zip(reqs, got)):
        if v is None:
            g = g.cpu().numpy() if i % 2 else g
            assert np.array_equal(g, oracle.sort_u32(k))
        else:
            gk, gv = (g[0].cpu().numpy(), g[1].cpu().numpy()) if i % 2 else g
            wk, wv = oracle.sort_pairs_u32(k, v)
            assert np.array_equal(gk, wk) and np.array_equal(gv, wv)


def test_device_serving_benchmark_small(serve):
    out = serve.run_serving_benchmark(count=40, fracs=(0.8,), lo=1 << 10, hi=1 << 18, resident="device")
    run = out["runs"][0]
    assert run["batched"]["p99_ms"] > 0 and run["serial"]["p99_ms"] > 0


def _merge_requests(count, seed, hi=1 << 17):
    """Merge requests: k sorted runs of uneven length (some empty), keys with
    heavy ties every third request so that the stable order by run matters."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(count):
        k = int(rng.integers(1, 12))
        lens = rng.integers(0, hi // k + 1, size=k)
        if i % 4 == 0:
            lens[0] = 0  # an empty run
        runs = []
        for j, ln in enumerate(lens):
            dist = "distinct16" if i % 3 == 0 else "uniform"
            runs.append(np.sort(workloads.keys_u32(dist, int(ln), seed=seed * 1000 + 17 * i + j)))
        keys = np.concatenate(runs).astype(np.uint32)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
        vals = workloads.draws_u32(seed * 11 + i, keys.size) if i % 2 else None
        reqs.append((0.0, keys, vals, offs))
    return reqs


def test_merge_requests_mixed_with_sorts(serve):
    """Merge requests (host and device, keys and pairs) batched together with
    sort requests: each result equals the serial path's and the oracle's
    (tolerance 0)."""
    import torch

    dev = torch.device("cuda:0")
    reqs = _requests(12, seed=21) + _merge_requests(12, seed=22)
    order = np.random.Generator(np.random.PCG64(23)).permutation(len(reqs))
    reqs = [reqs[i] for i in order]
    alone, _, _ = serve.serve_serial(reqs, realtime=False)
    with serve.SortServer(hbm_budget=1 << 30, solo_keys=1 << 16) as srv:
        with srv.held():
            futs = []
            for i, (_, k, v, *runs) in enumerate(reqs):
                on_dev = i % 3 == 1
                if on_dev:
                    k = torch.from_numpy(k).to(dev)
                    v = torch.from_numpy(v).to(dev) if v is not None else None
                futs.append(srv.submit_merge(k, runs[0], v) if runs else srv.submit(k, v))
        got = [f.result(timeout=120) for f in futs]
        assert srv.batches == 1
    for i, ((_, k, v, *runs), a, g) in enumerate(zip(reqs, alone, got)):
        host = lambda x: x.cpu().numpy() if isinstance(x, torch.Tensor) else x
        if runs:
            want = oracle.merge_runs(k, runs[0], v)
        else:
            want = oracle.sort_u32(k) if v is None else oracle.sort_pairs_u32(k, v)
        if v is None:
            assert np.array_equal(host(g), want) and np.array_equal(a, want), i
        else:
            assert np.array_equal(host(g[0]), want[0]) and np.array_equal(host(g[1]), want[1]), i
            assert np.array_equal(a[0], want[0]) and np.array_equal(a[1], want[1]), i


def test_merge_request_offsets_validated(serve):
    with serve.SortServer(hbm_budget=1 << 30) as srv:
        keys = np.arange(10, dtype=np.uint32)
        with pytest.raises(ValueError):
            srv.submit_merge(keys, [0, 5, 9])      # does not end at n
        with pytest.raises(ValueError):
            srv.submit_merge(keys, [0, 6, 5, 10])  # not monotone
        with pytest.raises(ValueError):
            srv.submit_merge(keys, [1, 10])        # does not start at 0
        assert np.array_equal(srv.submit_merge(keys, [0, 10]).result(timeout=60), keys)


def test_admission_by_free_hbm(serve):
    """Admission takes the smaller of the budget and the HBM free on the
    device: with the free figure pinned low, a request that fits the budget
    but not the free HBM is rejected while nothing is in flight, a smaller one
    is served, and the real figure is within the device's memory."""
    import torch

    with serve.SortServer(hbm_budget=1 << 40, hbm_headroom=0) as srv:
        real = srv._free_hbm()
        assert 0 < real <= torch.cuda.get_device_properties(0).total_memory
        srv._free_hbm = lambda: 4 << 20  # 4 MiB "free"
        big = workloads.keys_u32("uniform", 1 << 19, seed=4)     # 6 MiB + margin: does not fit
        small = workloads.keys_u32("uniform", 1 << 16, seed=5)   # 0.8 MiB: fits
        with pytest.raises(MemoryError):
            srv.submit(big).result(timeout=60)
        assert np.array_equal(srv.submit(small).result(timeout=60), oracle.sort_u32(small))
        assert srv.min_free_hbm == 4 << 20


def test_inline_launch_when_idle(serve):
    """A lone request on an idle server is launched on the submitting thread:
    its admission and launch timestamps fall inside the submit call."""
    import time

    keys = workloads.keys_u32("uniform", 3000, seed=8)
    with serve.SortServer(hbm_budget=1 << 30) as srv:
        srv.submit(keys).result(timeout=60)  # warm-up
        t0 = time.perf_counter()
        f = srv.submit(keys)
        t1 = time.perf_counter()
        assert np.array_equal(f.result(timeout=60), oracle.sort_u32(keys))
        tm = f.timing
        assert t0 <= tm["admitted"] <= tm["launched"] <= t1
    with serve.SortServer(hbm_budget=1 << 30, inline=False) as srv:
        assert np.array_equal(srv.submit(keys).result(timeout=60), oracle.sort_u32(keys))


@pytest.mark.parametrize("inline", [True, False])
def test_device_request_from_side_stream(serve, inline):
    """Device keys (and values) written on a side stream right before submit:
    the server reads them after that work, whether the request is launched
    inline on the submitting stream or queued for the launch thread (sorts,
    key/value sorts and merges)."""
    import torch

    dev = torch.device("cuda:0")
    side = torch.cuda.Stream(dev)
    n = 200_000
    keys = workloads.keys_u32("uniform", n, seed=21)
    vals = workloads.draws_u32(22, n)
    runs, offs = workloads.sorted_runs([70_000, 1, 90_000, 39_999], seed=23)
    with serve.SortServer(hbm_budget=1 << 30, inline=inline) as srv:
        for rep in range(3):
            hk = torch.from_numpy(keys).pin_memory()
            hv = torch.from_numpy(vals).pin_memory()
            hr = torch.from_numpy(runs).pin_memory()
            with torch.cuda.stream(side):
                kd = torch.empty(n, dtype=torch.uint32, device=dev)
                vd = torch.empty(n, dtype=torch.uint32, device=dev)
                rd = torch.empty(runs.size, dtype=torch.uint32, device=dev)
                kd.copy_(hk, non_blocking=True)
                vd.copy_(hv, non_blocking=True)
                rd.copy_(hr, non_blocking=True)
                f1 = srv.submit(kd)
                f2 = srv.submit(kd, vd)
                f3 = srv.submit_merge(rd, offs)
            g1 = f1.result(timeout=120).cpu().numpy()
            gk, gv = f2.result(timeout=120)
            g3 = f3.result(timeout=120).cpu().numpy()
            assert np.array_equal(g1, oracle.sort_u32(keys)), rep
            wk, wv = oracle.sort_pairs_u32(keys, vals)
            assert np.array_equal(gk.cpu().numpy(), wk) and np.array_equal(gv.cpu().numpy(), wv), rep
            assert np.array_equal(g3, oracle.merge_runs(runs, offs)), rep
