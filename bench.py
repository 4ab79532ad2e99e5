#!/usr/bin/env python3
"""Benchmark: sort throughput of 2^26 u32 keys on one MI355X.

One step = one full sort (block sort + every merge pass) of a 2^26-key array
resident in HBM; the timed steps cycle through the five seeded distributions
(uniform, sorted, reverse, 16 distinct values, Zipf(1.2) over 2^20 ranks).
Inputs, outputs and scratch are allocated before timing; no host transfer is
inside the timed region.

Prints ONE JSON line with the headline value (Gkeys/s), the roofline of the
dominant kernel (merge pass, HBM bound) measured live with HIP events on the
launch stream, and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
N_KEYS = 1 << 26


def _source_hash():
    from paper_1306_5076_amd.counters import kernel_source_hash

    return kernel_source_hash()


def committed_counters(name: str):
    """Counter summary committed under profiles/ for the current kernel sources, else None."""
    from paper_1306_5076_amd.counters import kernel_source_hash

    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def counted_kernel(rec, prefix: str):
    """The per-kernel counter record of the most-dispatched kernel named prefix..."""
    if not rec:
        return None, None
    cands = [(v.get("dispatches", 0), k) for k, v in rec["per_kernel"].items() if k.startswith(prefix)]
    if not cands:
        return None, None
    _, name = max(cands)
    return name, rec["per_kernel"][name]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Worker threads of the all-cores leg: the host cores this process may run on,
# at most 16 (the host-core share of one GPU on a shared GPU node).
CPU_THREADS_MAX = 16


def cpu_baseline(keys_np, reps=3):
    """The CPU oracle on one full 2^26-key uniform array, median of `reps` runs:
    its plain top-down merge sort pinned to one core (the calling thread's
    affinity set to a single core, as `taskset -c` would), and its chunked form
    on all allowed host cores (one chunk sort per thread, then a pairwise merge
    tree), each checked against the other."""
    import numpy as np

    import oracle

    allowed = sorted(os.sched_getaffinity(0))
    threads = max(1, min(CPU_THREADS_MAX, len(allowed)))
    pin = allowed[0]
    single = []
    os.sched_setaffinity(0, {pin})
    try:
        for _ in range(reps):
            t0 = time.perf_counter()
            ref = oracle.sort_u32(keys_np)
            single.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, set(allowed))
    multi = []
    for _ in range(reps):
        t0 = time.perf_counter()
        got = oracle.sort_u32_chunked(keys_np, threads)
        multi.append(time.perf_counter() - t0)
    if not np.array_equal(got, ref):
        raise RuntimeError("chunked oracle disagrees with the plain oracle")
    t1 = sorted(single)[len(single) // 2]
    tm = sorted(multi)[len(multi) // 2]
    return {
        "value": round(keys_np.size / t1 / 1e9, 4),
        "unit": "Gkeys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one {keys_np.size}-key uniform u32 array (seed 1), the oracle's top-down merge sort "
        f"pinned to host core {pin}, median of {reps} runs = {t1:.2f} s (runs {', '.join(f'{x:.2f}' for x in single)} s)",
        "all_cores": {
            "value": round(keys_np.size / tm / 1e9, 4),
            "unit": "Gkeys/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"the same array cut into {threads} chunks, each sorted by the oracle in its own thread, "
            f"then a pairwise merge tree of the oracle's stable merge; median of {reps} runs = {tm:.2f} s",
        },
        "nproc": os.cpu_count(),
        "allowed_cores": len(allowed),
        "cpu_model": _cpu_model(),
    }


def _kernel_table(stats):
    return {
        k: {
            "launches": v["launches"],
            "avg_us": round(1e3 * v["total_ms"] / v["launches"], 2),
            "GB_per_s": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1),
        }
        for k, v in stats.items()
    }


def bench_small(bcf, workloads, torch, dev, n=1 << 16, reps=100, warmup=10):
    """2^16 uniform u32 (fits in L2: latency-bound): median device time of one
    sort over `reps` runs, each bracketed by HIP events."""
    keys = workloads.keys_u32_torch("uniform", n, dev, seed=1)
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    for _ in range(warmup):
        bcf.sort_u32(keys, out=out, workspace=ws)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        bcf.sort_u32(keys, out=out, workspace=ws)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e3)
    times.sort()
    med = times[len(times) // 2]
    return {"n": n, "median_us": round(med, 2), "p10_us": round(times[reps // 10], 2),
            "Gkeys_per_s": round(n / med / 1e3, 3), "passes": bcf.sort_passes(n)}


def bench_block_sorts(bcf, workloads, torch, dev, n=1 << 26, reps=5):
    """Ablation of the block sort at 2^26 uniform keys: group tiles sorted by
    merge rounds (default), wave tiles sorted by merge rounds, wave tiles sorted
    by the paper's ShearSort (Sec. 3.1), group tiles sorted by the paper's long
    ShearSort over 8 waves; whole sort and the block-sort kernel."""
    from paper_1306_5076_amd import autotune

    keys = workloads.keys_u32_torch("uniform", n, dev, seed=1)
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    res = {"n": n}
    names = {3: "group_merge_rounds", 1: "wave_merge_rounds", 2: "wave_shearsort", 4: "group_long_shearsort"}
    for v, name in names.items():
        with bcf.tuning(block_sort=v):
            fn = lambda: bcf.sort_u32(keys, out=out, workspace=ws)
            ms = autotune.time_ms(fn, reps=reps, warmup=1)
            bcf.profile_collect()
            bcf.profile_enable(True)
            fn()
            bcf.profile_enable(False)
            st = bcf.profile_collect()
            bs = st.get("block_sort_keys", {"total_ms": 0.0, "launches": 1})
            res[name] = {"sort_ms": round(ms, 4), "Gkeys_per_s": round(n / ms / 1e6, 3),
                         "run_keys": bcf.run_keys(), "passes": bcf.sort_passes(n),
                         "block_sort_us": round(bs["total_ms"] * 1e3 / max(1, bs["launches"]), 1)}
    return res


def bench_fan_in(bcf, workloads, torch, dev, n=1 << 26, reps=5):
    """Merge fan-in at 2^26 uniform keys: four-way passes (default) against
    binary passes; whole sort and the per-launch time of each merge kernel."""
    from paper_1306_5076_amd import autotune

    keys = workloads.keys_u32_torch("uniform", n, dev, seed=1)
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    res = {"n": n}
    for k in (4, 2):
        with bcf.tuning(merge_fan_in=k):
            fn = lambda: bcf.sort_u32(keys, out=out, workspace=ws)
            ms = autotune.time_ms(fn, reps=reps, warmup=1)
            bcf.profile_collect()
            bcf.profile_enable(True)
            fn()
            bcf.profile_enable(False)
            st = bcf.profile_collect()
            res[f"fan_in_{k}"] = {"sort_ms": round(ms, 4), "Gkeys_per_s": round(n / ms / 1e6, 3),
                                  "passes": bcf.sort_passes(n), "kernels": _kernel_table(st)}
    return res


def bench_u64(bcf, workloads, torch, dev, n=1 << 26, reps=5):
    """Unsigned 64-bit keys at 2^26 (uniform 64-bit draws), inputs in HBM."""
    from paper_1306_5076_amd import autotune

    keys = workloads.draws_u64_torch(1, n, dev).view(torch.uint64)
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    fn = lambda: bcf.sort_u64(keys, out=out, workspace=ws)  # noqa: E731
    ms = autotune.time_ms(fn, reps=reps, warmup=1)
    bcf.profile_collect()
    bcf.profile_enable(True)
    fn()
    bcf.profile_enable(False)
    return {"n": n, "ms": round(ms, 4), "Gkeys_per_s": round(n / ms / 1e6, 3),
            "method": "keys in register pairs: group block sort into runs of 16384, binary merge passes",
            "kernels": _kernel_table(bcf.profile_collect())}


def bench_distribution(bcf, workloads, torch, dev, runs=256, run_len=1 << 18, P=256, t=256, reps=10):
    """The distribution step (Sec. 3.2; pivot buckets of Sec. 3.3) on 2^26 keys
    in 256 sorted runs of 2^18 (uniform keys), P = t = 256: whole call and the
    scatter kernel (one read and one write of every key) against HBM peak."""
    from paper_1306_5076_amd import autotune

    def autotime(fn):
        return autotune.time_ms(fn, reps=5, warmup=1)

    keys_np, off = workloads.sorted_runs([run_len] * runs, seed=1)
    keys = torch.from_numpy(keys_np).to(dev)
    n = keys.numel()
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    res = {"n": n, "runs": runs, "P": P, "t": t}
    for pb in (False, True):
        fn = lambda: bcf.distribute_runs(keys, off, P, t, pivot_buckets=pb, keys_out=out, workspace=ws)  # noqa: E731
        ms = autotune.time_ms(fn, reps=reps, warmup=2)
        bcf.profile_collect()
        bcf.profile_enable(True)
        for _ in range(3):
            fn()
        bcf.profile_enable(False)
        st = bcf.profile_collect()
        sc = st.get("dist_scatter")
        rec = {"ms": round(ms, 4), "Gkeys_per_s": round(n / ms / 1e6, 3), "kernels": _kernel_table(st)}
        if sc:
            gbs = sc["bytes"] / (sc["total_ms"] * 1e-3) / 1e9
            rec["scatter_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(gbs / HBM_PEAK_GBS, 4),
                                       "avg_launch_us": round(1e3 * sc["total_ms"] / sc["launches"], 2)}
        res["pivot_buckets" if pb else "plain"] = rec
    # whole sorts through the distribution (runs of 2^18, distribution, one
    # batched merge of every bucket's pieces; one host read-back of the piece
    # offsets in between) against the regular sort, same keys
    del keys, out
    srt = {}
    for dist in ("uniform", "distinct16", "zipf"):
        k = torch.from_numpy(workloads.keys_u32(dist, n, seed=1)).to(dev)
        o = torch.empty_like(k)
        row = {"bcf_sort_u32_ms": round(autotime(lambda: bcf.sort_u32(k, out=o, workspace=ws)), 4)}
        for pb in (False, True):
            row["pivot_buckets_ms" if pb else "plain_buckets_ms"] = round(autotime(
                lambda: bcf.sort_u32_pb(k, P=P, run_keys=run_len, pivot_buckets=pb, out=o, workspace=ws)), 4)
        srt[dist] = row
        del k, o
    res["sort_by_distribution_ms"] = srt
    return res


def bench_pairs(bcf, workloads, torch, dev, n=1 << 28, steps=5, warmup=2):
    """2^28 stable key/value sorts (value = original index), uniform and Zipf keys."""
    from paper_1306_5076_amd import autotune

    out = {}
    vals = torch.arange(n, dtype=torch.int32, device=dev).view(torch.uint32)
    ko = torch.empty(n, dtype=torch.uint32, device=dev)
    vo = torch.empty_like(ko)
    ws = bcf.Workspace(dev)
    for dist in ("uniform", "zipf"):
        keys = workloads.keys_u32_torch(dist, n, dev, seed=1)
        fn = lambda: bcf.sort_pairs_u32(keys, vals, ko, vo, workspace=ws)
        ms = autotune.time_ms(fn, reps=steps, warmup=warmup)
        bcf.profile_collect()
        bcf.profile_enable(True)
        fn()
        bcf.profile_enable(False)
        out[dist] = {"ms": round(ms, 3), "Gpairs_per_s": round(n / ms / 1e6, 3),
                     "kernels": _kernel_table(bcf.profile_collect())}
        del keys
    return {"n": n, "value": "original index", "stable": True, **out}


def bench_segmented(bcf, workloads, torch, dev, count=10000, lo=32, hi=1 << 20, seed=1, reps=3):
    """One batched segmented sort (eager and graph-replayed, autotuned knobs)
    against one bcf_sort_u32 call per array, same arrays, same stream."""
    from paper_1306_5076_amd import autotune

    sizes = workloads.segment_sizes(count, lo=lo, hi=hi, seed=seed)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    keys = workloads.draws_u32_torch(seed, n, dev)
    out = torch.empty_like(keys)
    ws = bcf.Workspace(dev)
    eager = lambda: bcf.segmented_sort(keys, offs, keys_out=out, workspace=ws)
    sig = autotune.signature("segmented", n, extra=f"{count}x[{lo},{hi}]")
    knobs, table = autotune.tuned(sig, eager, autotune.SEGMENTED_SPACE, path=None)
    res = {"arrays": count, "sizes": [lo, hi], "total_keys": n, "autotuned": knobs,
           "autotune_table": table}
    with bcf.tuning(**knobs):
        ms_eager = autotune.time_ms(eager, reps=reps)
        plan = bcf.SegmentedPlan(offs, dev)
        graph = plan.capture(keys, out)
        ms_graph = autotune.time_ms(graph.replay, reps=reps)
        views = [(int(offs[i]), int(offs[i + 1])) for i in range(count)]
        wsa = bcf.Workspace(dev)

        def per_array():
            for a, b in views:
                bcf.sort_u32(keys[a:b], out=out[a:b], workspace=wsa)

        ms_per = autotune.time_ms(per_array, reps=1, warmup=1)
        del plan, graph
        # the same sort through the device-offset entry point: planned on the
        # device from offsets in HBM (eager, and one captured graph)
        ms_dev, ms_dev_graph = _segmented_device_offsets(bcf, torch, dev, keys, out, offs, reps)
    res["per_array_calls"] = {"ms": round(ms_per, 3), "Gkeys_per_s": round(n / ms_per / 1e6, 3)}
    res["batched_eager"] = {"ms": round(ms_eager, 3), "Gkeys_per_s": round(n / ms_eager / 1e6, 3)}
    res["batched_graph"] = {"ms": round(ms_graph, 3), "Gkeys_per_s": round(n / ms_graph / 1e6, 3)}
    res["device_offsets_eager"] = {"ms": round(ms_dev, 3), "Gkeys_per_s": round(n / ms_dev / 1e6, 3)}
    res["device_offsets_graph"] = {"ms": round(ms_dev_graph, 3), "Gkeys_per_s": round(n / ms_dev_graph / 1e6, 3)}
    res["speedup_graph_vs_per_array"] = round(ms_per / ms_graph, 2)
    del keys, out
    return res


def bench_segmented_device(bcf, workloads, torch, dev, count=10000, lo=32, hi=1 << 20, seed=1, reps=3):
    """The segmented workload of bench_segmented (same arrays) through the
    device-offset entry point only, under the default tuning: eager calls and
    graph replays, for a kernel trace of that sort alone."""
    sizes = workloads.segment_sizes(count, lo=lo, hi=hi, seed=seed)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    keys = workloads.draws_u32_torch(seed, n, dev)
    out = torch.empty_like(keys)
    ms_dev, ms_graph = _segmented_device_offsets(bcf, torch, dev, keys, out, offs, reps)
    del keys, out
    return {"arrays": count, "sizes": [lo, hi], "total_keys": n, "reps": reps,
            "device_offsets_eager": {"ms": round(ms_dev, 3), "Gkeys_per_s": round(n / ms_dev / 1e6, 3)},
            "device_offsets_graph": {"ms": round(ms_graph, 3), "Gkeys_per_s": round(n / ms_graph / 1e6, 3)}}


def _segmented_device_offsets(bcf, torch, dev, keys, out, offs, reps):
    """Device time of bcf_segmented_sort with its offsets in device memory
    (temp sized once by a query), eager and replayed from one graph."""
    import ctypes

    from paper_1306_5076_amd import _native, autotune

    lib = _native.load()
    vp = ctypes.c_void_p
    nseg = len(offs) - 1
    doff = torch.from_numpy(offs.astype("int64")).to(dev)
    stream = torch.cuda.current_stream(dev)
    need = ctypes.c_uint64(0)
    _native.check("bcf_segmented_sort", lib.bcf_segmented_sort(None, None, vp(doff.data_ptr()), nseg, None,
                                                                ctypes.byref(need), vp(stream.cuda_stream)))
    temp = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    tb = ctypes.c_uint64(temp.numel())

    def run():
        _native.check("bcf_segmented_sort", lib.bcf_segmented_sort(
            vp(keys.data_ptr()), vp(out.data_ptr()), vp(doff.data_ptr()), nseg, vp(temp.data_ptr()),
            ctypes.byref(tb), vp(torch.cuda.current_stream(dev).cuda_stream)))

    ms_eager = autotune.time_ms(run, reps=reps)
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        run()  # warm-up outside capture
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    ms_graph = autotune.time_ms(g.replay, reps=reps)
    del g, temp, doff
    return ms_eager, ms_graph


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=N_KEYS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-per-dist", action="store_true", help="skip the per-distribution timing")
    ap.add_argument("--quick", action="store_true",
                    help="headline only: skip the pairs, segmented and serving sections")
    ap.add_argument("--distribution", action="store_true",
                    help="only the distribution step at 2^26 keys in 256 runs (one JSON object)")
    ap.add_argument("--block-sort-ablation", action="store_true",
                    help="only the block-sort ablation at 2^26 keys (one JSON object)")
    ap.add_argument("--pairs", action="store_true",
                    help="only the 2^28 stable key/value sorts, uniform and Zipf keys (one JSON object)")
    ap.add_argument("--segmented", action="store_true",
                    help="only the segmented sort (10000 arrays of 32 .. 2^20 keys) through the "
                         "device-offset entry point (one JSON object)")
    ap.add_argument("--u64", action="store_true", help="only the 2^26 u64 key sort (one JSON object)")
    ap.add_argument("--reps", type=int, default=5, help="repetitions of the ablation timings")
    ap.add_argument(
        "--copy-calibration",
        action="store_true",
        help="first copy one n-key array device-to-device 3 times (a plain copy of known size, "
        "used to scale HBM traffic counters)",
    )
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(
            "bench.py measures one GPU only: this build has no multi-GPU path "
            "(the sort of one array runs on one MI355X); run with --gpus 1.",
            file=sys.stderr,
        )
        sys.exit(2)
    if args.distribution:
        import torch

        import paper_1306_5076_amd as bcf
        import workloads

        dev = torch.device("cuda:0")
        if args.copy_calibration:  # a plain copy of n u32 keys, 3 times, for the traffic counters
            a = torch.zeros(args.n, dtype=torch.int32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        print(json.dumps(bench_distribution(bcf, workloads, torch, dev)), flush=True)
        return
    if args.pairs:
        import torch

        import paper_1306_5076_amd as bcf
        import workloads

        rec = bench_pairs(bcf, workloads, torch, torch.device("cuda:0"), steps=args.steps, warmup=args.warmup)
        print(json.dumps(rec), flush=True)
        return
    if args.segmented or args.u64:
        import torch

        import paper_1306_5076_amd as bcf
        import workloads

        dev = torch.device("cuda:0")
        if args.copy_calibration:  # a plain copy of n u32 keys, 3 times, for the traffic counters
            a = torch.zeros(args.n, dtype=torch.int32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        if args.segmented:
            rec = bench_segmented_device(bcf, workloads, torch, dev, reps=args.reps)
        else:
            rec = bench_u64(bcf, workloads, torch, dev, reps=args.reps)
        print(json.dumps(rec), flush=True)
        return
    if args.block_sort_ablation:
        import torch

        import paper_1306_5076_amd as bcf
        import workloads

        print(json.dumps(bench_block_sorts(bcf, workloads, torch, torch.device("cuda:0"), reps=args.reps)), flush=True)
        return

    import numpy as np
    import torch

    import paper_1306_5076_amd as bcf
    import workloads

    dev = torch.device("cuda:0")
    n = args.n
    dists = list(workloads.DISTRIBUTIONS)
    host = {d: workloads.keys_u32(d, n, seed=1) for d in dists}
    src = {d: torch.from_numpy(host[d]).to(dev) for d in dists}
    out = torch.empty(n, dtype=torch.uint32, device=dev)
    ws = bcf.Workspace(dev)
    stream = torch.cuda.current_stream(dev)

    def step(i):
        bcf.sort_u32(src[dists[i % len(dists)]], out=out, stream=stream, workspace=ws)

    if args.copy_calibration:
        for _ in range(3):
            out.copy_(src["uniform"])
        torch.cuda.synchronize()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed / 1e9

    # per-distribution time (events on the launch stream)
    per_dist = {}
    for d in ([] if args.no_per_dist else dists):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            bcf.sort_u32(src[d], out=out, stream=stream, workspace=ws)
        e1.record(stream)
        e1.synchronize()
        per_dist[d] = round(e0.elapsed_time(e1) / reps, 4)

    # the same sorts replayed from a captured graph (one graph per distribution)
    graph_ms = {}
    try:
        ws.get(1, dev)  # scratch allocated before capture
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            for d in dists:
                bcf.sort_u32(src[d], out=out, stream=side, workspace=ws)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graphs = {}
        for d in dists:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                bcf.sort_u32(src[d], out=out, workspace=ws)
            graphs[d] = g
        for d in dists:
            graphs[d].replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            graphs[dists[i % len(dists)]].replay()
        torch.cuda.synchronize()
        graph_ms = {"ms_per_step": round((time.perf_counter() - t0) * 1e3 / args.steps, 4)}
        graph_ms["value_gkeys_per_s"] = round(n / graph_ms["ms_per_step"] / 1e6, 4)
        del graphs
    except Exception as e:  # reported, never fatal for the headline
        graph_ms = {"error": repr(e)[:200]}

    # roofline of the dominant kernel: per-launch HIP events around each launch
    bcf.profile_collect()
    bcf.profile_enable(True)
    for i in range(max(1, args.profile_steps)):
        step(i)
    bcf.profile_enable(False)
    stats = bcf.profile_collect()
    dominant = max(stats, key=lambda k: stats[k]["total_ms"])
    st = stats[dominant]
    avg_ms = st["total_ms"] / st["launches"]
    bytes_per_launch = st["bytes"] / st["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernels = _kernel_table(stats)
    # the rocprofv3 name of the dominant launch record
    prefix = {"merge_keys": "bcf::k_merge<false, bcf::RegularMergeSrc", "merge4_keys": "bcf::k_merge4<",
              "block_sort_keys": "bcf::k_block_sort"}.get(dominant, "-")
    traffic_name, traffic_rec = counted_kernel(committed_counters("traffic_sort_keys_2p26.json"), prefix)
    conflicts_rec = committed_counters("lds_sort_keys_2p26.json")

    rec = {
        "metric": "Gkeys/s + HBM GB/s frac at 2^26 uint32; LDS bank conflicts; p99 served latency",
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "sort 2^26 uint32 keys (one array per step, cycling uniform / sorted / reverse / "
            "16-distinct / zipf1.2 over 2^20 ranks, seed 1)",
            "n": n,
            "distributions": dists,
            "tile_keys": bcf.tile_keys(),
            "run_keys": bcf.run_keys(),
            "passes_per_sort": bcf.sort_passes(n),
        },
        "per_distribution_ms": per_dist,
        "graph_replay": graph_ms,
        "roofline": {
            "kernel": dominant,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_rec["read_bytes"] + traffic_rec["write_bytes"] if traffic_rec else None,
            "traffic_kernel": traffic_name,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_ms * 1e3, 2),
        },
        "kernels": kernels,
        "overall_hbm_frac": round(
            sum(v["bytes"] for v in stats.values()) / (sum(v["total_ms"] for v in stats.values()) * 1e-3) / 1e9
            / HBM_PEAK_GBS,
            4,
        ),
        "lds_bank_conflicts": conflicts_rec["per_kernel"] if conflicts_rec else None,
        "kernel_source_hash": _source_hash(),
    }
    rec["tuning"] = bcf.get_tuning()
    if not args.quick:
        del src, out
        torch.cuda.empty_cache()
        t0s = time.perf_counter()
        rec["small_2p16"] = bench_small(bcf, workloads, torch, dev)
        rec["block_sort_ablation"] = bench_block_sorts(bcf, workloads, torch, dev)
        rec["fan_in_ablation"] = bench_fan_in(bcf, workloads, torch, dev)
        rec["pairs_2p28"] = bench_pairs(bcf, workloads, torch, dev)
        torch.cuda.empty_cache()
        rec["u64_2p26"] = bench_u64(bcf, workloads, torch, dev)
        torch.cuda.empty_cache()
        rec["distribution_2p26"] = bench_distribution(bcf, workloads, torch, dev)
        torch.cuda.empty_cache()
        from paper_1306_5076_amd import cps_demo

        rec["colored_prefix_sums_2p29"] = cps_demo.sweep(reps=3, device=str(dev))
        torch.cuda.empty_cache()
        rec["segmented"] = bench_segmented(bcf, workloads, torch, dev)
        rec["segmented_2p17"] = bench_segmented(bcf, workloads, torch, dev, hi=1 << 17)
        rec["segmented_2p17"].pop("autotune_table", None)
        torch.cuda.empty_cache()
        from paper_1306_5076_amd import serve

        rec["serving"] = serve.run_serving_benchmark(count=400, device=str(dev))
        rec["serving_device"] = serve.run_serving_benchmark(count=2000, device=str(dev), resident="device")
        rec["sections_s"] = round(time.perf_counter() - t0s, 1)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(host["uniform"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
