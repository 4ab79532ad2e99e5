"""Autotuner for the library's tuning knobs (bcf_tuning in include/bcf.h).

For a workload (a callable that enqueues one sort on the current stream) it
times every combination of candidate knob values with HIP events, keeps the
fastest, and caches the winner in a JSON file keyed by a workload signature
(kind, size bucket, key/value or keys only).  The knobs it searches are the
ones the kernels expose at run time:

* block_sort        -- (sorts) the block size: wave tiles of 4096 keys (one
                       wave, E = 64 keys per lane) or group tiles of 32768
                       keys (8 waves; 16384 pairs by 4 waves), both sorted by
                       merge rounds;
* group_min_keys    -- (segmented sorts) the same block-size choice per
                       segment: the segment length from which a segment is
                       block-sorted in group tiles instead of wave tiles;
* merge_fan_in      -- (sorts and segmented sorts, keys or pairs) runs merged per
                       pass: 2 (binary passes), 4 (four-way passes, two merge
                       levels per read and write of the data), or 0 for the
                       size-based default;
* merge_variant     -- persistent waves with / without next-tile prefetch, one
                       tile per wave, or the per-kind default;
* nontemporal       -- nontemporal hints on the merge passes' tile traffic;
* fused_partition   -- whether one-tile-per-wave merge passes search their
                       own splits (one launch per pass) or a partition
                       launch does.

The keys per lane (E = 64, one line of the 64 x 64 wave tile) are fixed by the
conflict-free layout: the register index of a key is a compile-time constant,
so E is a property of the compiled kernels, not a run-time knob.
"""

from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bcf_sort", "autotune.json")

SORT_SPACE = {"block_sort": [3, 1], "merge_fan_in": [0, 4, 2], "merge_variant": [3, 1, 2, 0], "nontemporal": [1, 0],
              "fused_partition": [1, 0]}
SEGMENTED_SPACE = {"merge_fan_in": [4, 2], "merge_variant": [3, 1, 2], "nontemporal": [1, 0],
                   "group_min_keys": [4097, 16384, 65536, 1 << 40]}


def signature(kind: str, n: int, pairs: bool = False, extra: str = "") -> str:
    bucket = int(math.log2(max(1, n)))
    return f"{kind}:{'pairs' if pairs else 'keys'}:2^{bucket}{':' + extra if extra else ''}"


def time_ms(fn, reps: int = 3, warmup: int = 1, stream=None) -> float:
    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return sorted(times)[len(times) // 2]


def tune(fn, space: dict, reps: int = 3, warmup: int = 1):
    """Time ``fn`` under every combination in ``space``; returns (best, table)."""
    names = list(space)
    table = []
    for combo in itertools.product(*(space[k] for k in names)):
        knobs = dict(zip(names, combo))
        with api.tuning(**knobs):
            ms = time_ms(fn, reps=reps, warmup=warmup)
        table.append({**knobs, "ms": round(ms, 4)})
    best = min(table, key=lambda r: r["ms"])
    return {k: best[k] for k in names}, table


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(sig: str, knobs: dict, path: str = DEFAULT_CACHE):
    cache = load_cache(path)
    cache[sig] = knobs
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(sig: str, fn, space: dict, path: str | None = DEFAULT_CACHE, reps: int = 3):
    """Cached knobs for ``sig``, tuning (and caching) them on a miss.

    Returns (knobs, table or None when the cache answered).
    """
    if path:
        hit = load_cache(path).get(sig)
        if hit:
            return hit, None
    knobs, table = tune(fn, space, reps=reps)
    if path:
        store_cache(sig, knobs, path)
    return knobs, table
