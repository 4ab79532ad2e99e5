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
