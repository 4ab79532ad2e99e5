"""Continuous-batching sort service on one GPU, and its one-call-per-request baseline.

:class:`SortServer` accepts sort requests (u32 keys, or u32/u32 pairs sorted
stably by key) from any thread.  A launch thread

* admits waiting requests in arrival order while their device bytes fit the
  HBM budget (a request larger than the whole budget is rejected) and the
  batch stays under ``max_batch_keys``;
* packs the admitted requests into one batch: requests of at least
  ``solo_keys`` keys, and a request alone in its batch, are sorted on their
  own (``bcf_sort_u32`` / ``bcf_sort_pairs_u32``, no launch plan to build),
  the smaller ones of each kind share one segmented sort
  (``bcf_segmented_sort`` / ``bcf_segmented_sort_pairs``) in which each
  request is a segment;
* runs each batch (host-to-device copy, sorts, device-to-host copy) on the
  stream of one of ``slots`` buffer slots, so up to that many batches are in
  flight and one batch's copies overlap another's kernels; requests that
  arrive meanwhile join the next batch;
* keeps its device buffers and pinned host staging resident between batches
  (they grow on demand and are reused, never freed per request).

A completion thread waits for each batch's device-to-host copy, hands every
request its result, records its latency from arrival to completion and
returns the batch's buffers and HBM budget share.

:func:`serve_serial` is the baseline: one request at a time, in arrival order,
each with its own copy in, ``bcf_sort_u32`` / ``bcf_sort_pairs_u32`` call and
copy out, synchronised.
"""

from __future__ import annotations

import collections
import contextlib
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

__all__ = ["SortServer", "SortFuture", "serve_serial", "serve_batched", "latency_stats", "make_requests", "run_serving_benchmark"]


class SortFuture(Future):
    """Future of one request; ``timing`` holds the request's timestamps
    (time.perf_counter(): submitted, admitted, launched, done, finished)
    once it has completed."""

    timing = None


@dataclass
class _Request:
    keys: object            # numpy array (host request) or CUDA tensor (device request)
    vals: object | None
    arrival: float
    ready: object = None    # device request: event recorded on the submitting stream
    future: SortFuture = field(default_factory=SortFuture)
    submitted: float = 0.0  # perf_counter() when submit() queued it
    admitted: float = 0.0   # ... when the launch thread took it into a batch
    launched: float = 0.0   # ... when its batch's copies and kernels were enqueued
    done: float = 0.0       # ... when its batch's device-to-host copy had finished
    finished: float = 0.0   # ... when its result was handed out

    @property
    def n(self) -> int:
        return int(self.keys.numel()) if self.on_device else int(self.keys.size)

    @property
    def on_device(self) -> bool:
        return self.ready is not None

    @property
    def pairs(self) -> bool:
        return self.vals is not None

    def device_bytes(self) -> int:
        words = 2 if self.pairs else 1
        # input + output arrays, plus merge scratch of the same size and a margin for descriptors
        return self.n * 4 * words * 3 + 64 * 1024


class _Grow:
    """A tensor that grows on demand (to the next power of two) and is reused,
    on the device or in pinned host memory."""

    def __init__(self, device=None, pinned=False):
        self.device, self.pinned, self.t = device, pinned, None

    def get(self, n: int):
        if self.t is None or self.t.numel() < n:
            cap = 1 << max(16, (max(n, 1) - 1).bit_length())
            self.t = None  # release the old buffer before taking the new one
            if self.pinned:
                self.t = torch.empty(cap, dtype=torch.uint32, pin_memory=True)
            else:
                self.t = torch.empty(cap, dtype=torch.uint32, device=self.device)
        return self.t[:n]


class _Slot:
    """Resident buffers of one in-flight batch."""

    def __init__(self, device, reserve_keys: int = 0):
        self.hk, self.hv = _Grow(pinned=True), _Grow(pinned=True)      # host in
        self.ok, self.ov = _Grow(pinned=True), _Grow(pinned=True)      # host out
        self.dk, self.dv = _Grow(device), _Grow(device)                # device in
        for g in (self.hk, self.hv, self.ok, self.ov, self.dk, self.dv):
            g.get(reserve_keys)
        self.out = None     # the batch's device outputs (keys, values)
        self.ws = api.Workspace(device)
        self.stream = torch.cuda.Stream(device)
        self.done = None
        self.reqs = []
        self.loc = []       # per request: (key lo, key hi, value lo) in the batch buffers


class SortServer:
    """Continuous-batching sort server (see module docstring)."""

    def __init__(self, device="cuda:0", hbm_budget: int = 16 << 30, max_batch_keys: int = 1 << 24,
                 slots: int = 3, reserve_keys: int = 0, solo_keys: int = 1 << 20):
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_batch_keys = int(max_batch_keys)
        self.solo_keys = int(solo_keys)
        self.slots = [_Slot(self.device, reserve_keys) for _ in range(slots)]
        self.free_slots = collections.deque(self.slots)
        self.busy = collections.deque()
        self.pending = collections.deque()
        self.used = 0
        self.peak_used = 0
        self.batches = 0
        self.batch_sizes = []
        self.cv = threading.Condition()
        self.stop = False
        self.launcher_done = False
        self.holds = 0
        self.error = None
        self.launcher = threading.Thread(target=self._guard, args=(self._launch_loop,), name="bcf-sort-launch",
                                         daemon=True)
        self.completer = threading.Thread(target=self._guard, args=(self._complete_loop,),
                                          name="bcf-sort-complete", daemon=True)
        self.launcher.start()
        self.completer.start()

    # ---------------------------------------------------------------- client side

    def submit(self, keys, vals=None, arrival: float | None = None) -> Future:
        """Queue one sort request; the future's result is the sorted keys, or
        (keys, values) for a key/value request.

        Host requests (array-likes) get numpy results.  Device requests (uint32
        CUDA tensors on the server's device) are read on the device after the
        work already enqueued on the submitting thread's current stream, and
        get CUDA tensors back: views of the batch's output buffers, complete
        when the future resolves (a consumer on another stream should call
        ``record_stream`` on them).
        """
        ready = None
        if isinstance(keys, torch.Tensor) and keys.is_cuda:
            if keys.dtype != torch.uint32 or keys.device != self.device or not keys.is_contiguous():
                raise ValueError("device keys must be a contiguous uint32 tensor on the server's device")
            if vals is not None and (not isinstance(vals, torch.Tensor) or vals.dtype != torch.uint32
                                     or vals.device != self.device or vals.shape != keys.shape
                                     or not vals.is_contiguous()):
                raise ValueError("device values must be a contiguous uint32 tensor shaped like the keys")
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(self.device))
        else:
            keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint32))
            if vals is not None:
                vals = np.ascontiguousarray(np.asarray(vals, dtype=np.uint32))
                if vals.shape != keys.shape:
                    raise ValueError("keys and vals must have the same length")
        r = _Request(keys, vals, time.perf_counter() if arrival is None else arrival, ready)
        if r.device_bytes() > self.budget:
            r.future.set_exception(MemoryError(f"request of {r.n} keys exceeds the HBM budget"))
            return r.future
        r.submitted = time.perf_counter()
        with self.cv:
            if self.stop:
                raise RuntimeError("server is closed")
            self.pending.append(r)
            self.cv.notify_all()
        return r.future

    @contextlib.contextmanager
    def held(self):
        """Admit nothing new while inside the block (requests still queue up);
        on exit everything that queued meanwhile is admitted together."""
        with self.cv:
            self.holds += 1
        try:
            yield self
        finally:
            with self.cv:
                self.holds -= 1
                self.cv.notify_all()

    def reset_stats(self):
        """Zero the batch counters and the peak of admitted device bytes."""
        with self.cv:
            self.batches, self.batch_sizes, self.peak_used = 0, [], self.used

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        self.launcher.join()
        self.completer.join()
        if self.error:
            raise self.error

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- scheduler

    def _guard(self, loop):
        try:
            torch.cuda.set_device(self.device)
            loop()
        except BaseException as e:  # surface in close(); fail everything still queued
            with self.cv:
                self.error = self.error or e
                self.stop = True
                self.launcher_done = True
                for r in list(self.pending) + [r for s in self.busy for r in s.reqs]:
                    if not r.future.done():
                        r.future.set_exception(e)
                self.pending.clear()
                self.cv.notify_all()

    def _take_batch(self):
        """Admit requests in arrival order while they fit the batch and the HBM
        budget (called with the lock held)."""
        batch, keys = [], 0
        while self.pending:
            r = self.pending[0]
            if batch and keys + r.n > self.max_batch_keys:
                break
            if self.used + r.device_bytes() > self.budget:
                break  # admission by free-HBM budget: wait for completions
            self.pending.popleft()
            batch.append(r)
            keys += r.n
            self.used += r.device_bytes()
        return batch

    def _launch_loop(self):
        while True:
            with self.cv:
                while True:
                    if self.stop and not self.pending:
                        self.launcher_done = True
                        self.cv.notify_all()
                        return
                    batch = []
                    if self.pending and self.free_slots and (not self.holds or self.stop):
                        batch = self._take_batch()
                    if batch:
                        break
                    self.cv.wait()
                slot = self.free_slots.popleft()
                self.peak_used = max(self.peak_used, self.used)
                self.batches += 1
                self.batch_sizes.append(len(batch))
            now = time.perf_counter()
            for r in batch:
                r.admitted = now
            self._launch(slot, batch)
            now = time.perf_counter()
            for r in batch:
                r.launched = now
            with self.cv:
                self.busy.append(slot)
                self.cv.notify_all()

    def _complete_loop(self):
        while True:
            with self.cv:
                while not self.busy:
                    if self.launcher_done:
                        return
                    self.cv.wait()
                slot = self.busy[0]
            slot.done.synchronize()  # releases the GIL while the device finishes the batch
            done = time.perf_counter()
            ok, ov = slot.ok.t, slot.ov.t
            rk, rv = slot.out
            for r, (lo, hi, vlo) in zip(slot.reqs, slot.loc):
                if r.on_device:
                    k = rk[lo:hi]
                    v = rv[vlo:vlo + (hi - lo)] if r.pairs else None
                else:
                    k = ok[lo:hi].clone().numpy()
                    v = ov[vlo:vlo + (hi - lo)].clone().numpy() if r.pairs else None
                r.done = done
                r.finished = time.perf_counter()
                r.future.timing = {"submitted": r.submitted, "admitted": r.admitted, "launched": r.launched,
                                   "done": r.done, "finished": r.finished}
                r.future.set_result((k, v) if r.pairs else k)
            with self.cv:
                self.busy.popleft()
                self.used -= sum(r.device_bytes() for r in slot.reqs)
                slot.reqs, slot.loc, slot.out = [], [], None
                self.free_slots.append(slot)
                self.cv.notify_all()

    def _launch(self, slot: _Slot, batch):
        # order in the batch buffers: host requests before device requests, within
        # each keys-only before key/value, small before large, so that the host
        # part is one span (one copy each way) and the small requests of each
        # (residence, kind) group are contiguous; values exist for key/value
        # requests only and follow the same order
        solo = lambda r: r.n >= self.solo_keys
        slot.reqs = sorted(batch, key=lambda r: (r.on_device, r.pairs, solo(r)))
        slot.loc = []
        pos, vpos, nh, nvh = 0, 0, 0, 0
        for r in slot.reqs:
            slot.loc.append((pos, pos + r.n, vpos))
            pos += r.n
            vpos += r.n if r.pairs else 0
            if not r.on_device:
                nh, nvh = pos, vpos
        n, npairs = pos, vpos
        # pack host requests into the slot's pinned buffers (torch copies:
        # multi-threaded, GIL released)
        hk, hv = slot.hk.get(nh), slot.hv.get(nvh)
        for r, (lo, hi, vlo) in zip(slot.reqs, slot.loc):
            if not r.on_device:
                hk[lo:hi].copy_(torch.from_numpy(r.keys))
                if r.pairs:
                    hv[vlo:vlo + (hi - lo)].copy_(torch.from_numpy(r.vals))
        dk, dv = slot.dk.get(n), slot.dv.get(npairs)
        # copy in, sort, copy out, all on the slot's own stream: batches in
        # different slots overlap (one batch's copies with another's kernels)
        st = slot.stream
        with torch.cuda.stream(st):
            if nh:
                dk[:nh].copy_(hk, non_blocking=True)
            if nvh:
                dv[:nvh].copy_(hv, non_blocking=True)
            alone = len(slot.reqs) == 1
            for r, (lo, hi, vlo) in zip(slot.reqs, slot.loc):
                if r.on_device:
                    st.wait_event(r.ready)
                    if not (alone or solo(r)):  # sorted from its own buffer otherwise
                        dk[lo:hi].copy_(r.keys, non_blocking=True)
                        if r.pairs:
                            dv[vlo:vlo + r.n].copy_(r.vals, non_blocking=True)
            rk = torch.empty(n, dtype=torch.uint32, device=self.device)
            rv = torch.empty(npairs, dtype=torch.uint32, device=self.device)
            slot.out = (rk, rv)
            # large requests, and a request alone in its batch, sort on their own
            # (no launch plan to build); the small ones of each group share one
            # segmented sort
            groups = {}
            for r, (lo, hi, vlo) in zip(slot.reqs, slot.loc):
                if alone or solo(r):
                    ki = r.keys if r.on_device else dk[lo:hi]
                    if r.pairs:
                        vi = r.vals if r.on_device else dv[vlo:vlo + r.n]
                        api.sort_pairs_u32(ki, vi, rk[lo:hi], rv[vlo:vlo + r.n], stream=st, workspace=slot.ws)
                    else:
                        api.sort_u32(ki, out=rk[lo:hi], stream=st, workspace=slot.ws)
                else:
                    groups.setdefault((r.on_device, r.pairs), []).append((lo, hi, vlo))
            for (_, pairs), segs in groups.items():
                lo0, hi1, v0 = segs[0][0], segs[-1][1], segs[0][2]
                offs = np.asarray([0] + [hi - lo0 for _, hi, _ in segs], dtype=np.uint64)
                if pairs:
                    v1 = v0 + (hi1 - lo0)
                    api.segmented_sort(dk[lo0:hi1], offs, vals=dv[v0:v1], keys_out=rk[lo0:hi1],
                                       vals_out=rv[v0:v1], stream=st, workspace=slot.ws)
                else:
                    api.segmented_sort(dk[lo0:hi1], offs, keys_out=rk[lo0:hi1], stream=st, workspace=slot.ws)
            if nh:
                slot.ok.get(nh).copy_(rk[:nh], non_blocking=True)
            if nvh:
                slot.ov.get(nvh).copy_(rv[:nvh], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        slot.done = ev


def serve_serial(requests, device="cuda:0", realtime: bool = True, keep_results: bool = True):
    """Baseline: each request alone (copy in, sort, copy out, synchronise), FIFO.

    ``requests`` is a list of ``(arrival_offset_s, keys, vals_or_None)``, keys
    and values host arrays or CUDA tensors (no copies then); with ``realtime``
    a request is not started before its arrival time.  Host staging is pinned
    and resident, as in :class:`SortServer`.  Returns ``(results,
    latencies_s, wall_s)``; without ``keep_results`` each result is dropped
    once complete (a client that consumes its results; memory stays flat).
    """
    dev = torch.device(device)
    ws = api.Workspace(dev)
    hk, hv, ok, ov = (_Grow(pinned=True) for _ in range(4))
    dk, dv, rk, rv = (_Grow(dev) for _ in range(4))
    out, lat = [], []
    t0 = time.perf_counter()
    for arr, keys, vals in requests:
        if realtime:
            _wait_until(t0 + arr)
        arrival = t0 + arr if realtime else time.perf_counter()
        if isinstance(keys, torch.Tensor):  # device request: sort into fresh device outputs
            ko = torch.empty_like(keys)
            if vals is not None:
                vo = torch.empty_like(vals)
                api.sort_pairs_u32(keys, vals, ko, vo, workspace=ws)
                res = (ko, vo)
            else:
                res = api.sort_u32(keys, out=ko, workspace=ws)
            torch.cuda.synchronize(dev)
            lat.append(time.perf_counter() - arrival)
            out.append(res if keep_results else None)
            continue
        n = keys.size
        hkk, dkk, rkk, okk = hk.get(n), dk.get(n), rk.get(n), ok.get(n)
        hkk.copy_(torch.from_numpy(keys))
        dkk.copy_(hkk, non_blocking=True)
        if vals is not None:
            hvv, dvv, rvv, ovv = hv.get(n), dv.get(n), rv.get(n), ov.get(n)
            hvv.copy_(torch.from_numpy(vals))
            dvv.copy_(hvv, non_blocking=True)
            api.sort_pairs_u32(dkk, dvv, rkk, rvv, workspace=ws)
            okk.copy_(rkk, non_blocking=True)
            ovv.copy_(rvv, non_blocking=True)
        else:
            api.sort_u32(dkk, out=rkk, workspace=ws)
            okk.copy_(rkk, non_blocking=True)
        torch.cuda.synchronize(dev)
        res = (okk.clone().numpy(), ovv.clone().numpy()) if vals is not None else okk.clone().numpy()
        lat.append(time.perf_counter() - arrival)
        out.append(res if keep_results else None)
    return out, lat, time.perf_counter() - t0


def _wait_until(at: float):
    """Wait until perf_counter() reaches `at` without holding the GIL: sleep
    most of the way, then poll with zero-length sleeps (each one lets the
    server's threads take the GIL; a plain spin would hold it for a whole
    switch interval, 5 ms by default, and stall them)."""
    while True:
        left = at - time.perf_counter()
        if left <= 0:
            return
        time.sleep(left - 1e-4 if left > 2e-4 else 0)


def latency_stats(lat_s):
    a = np.asarray(lat_s, dtype=np.float64) * 1e3
    return {"p50_ms": round(float(np.percentile(a, 50)), 3), "p99_ms": round(float(np.percentile(a, 99)), 3),
            "mean_ms": round(float(a.mean()), 3), "max_ms": round(float(a.max()), 3)}


def make_requests(count: int, lo: int = 1 << 10, hi: int = 1 << 24, seed: int = 1, pool_keys: int = 1 << 25,
                  device=None):
    """Seeded serving workload: (arrival_at_qps_1, keys, vals_or_None) per request.

    Sizes are log-uniform in [lo, hi]; half the requests are key/value pairs
    (value = position in the request); keys are slices of one seeded uniform
    pool so that the request set is cheap to build.  With ``device`` the keys
    and values are CUDA tensors there (requests already resident in HBM),
    else numpy arrays.
    """
    import workloads

    if device is None:
        pool = workloads.keys_u32("uniform", pool_keys, seed=seed)
    else:
        pool = workloads.keys_u32_torch("uniform", pool_keys, torch.device(device), seed=seed)
    spec = workloads.request_stream(count, qps=1.0, lo=lo, hi=hi, seed=seed)
    offs = workloads.draws_u64(seed ^ 0x0FF, count) % np.uint64(max(1, pool_keys - hi))
    reqs = []
    for i, (t, size, pairs, _) in enumerate(spec):
        size = min(size, pool_keys)
        o = int(offs[i])
        keys = pool[o:o + size]
        if device is None:
            vals = np.arange(size, dtype=np.uint32) if pairs else None
        else:
            vals = torch.arange(size, dtype=torch.int32, device=device).view(torch.uint32) if pairs else None
        reqs.append((t, keys, vals))
    return reqs


def serve_batched(requests, qps: float, device="cuda:0", hbm_budget: int = 16 << 30, server=None,
                  keep_results: bool = True):
    """Submit ``requests`` at their arrival times (scaled to ``qps``) to a
    :class:`SortServer` (``server``, else a new one); returns
    (results, latencies_s, wall_s, server stats).  Without ``keep_results``
    every result is dropped as soon as it is complete (results are None)."""
    own = server is None
    if own:
        server = SortServer(device, hbm_budget=hbm_budget)
    server.reset_stats()
    arrivals, timings = [], [None] * len(requests)
    results = [None] * len(requests)
    remaining = [len(requests)]
    all_done = threading.Event()
    lock = threading.Lock()

    def on_done(i, f):
        # runs on the server's completion thread: keep the timestamps (and the
        # result only if asked: a consumer that drops results keeps memory flat)
        try:
            if f.exception() is None:
                timings[i] = f.timing
                if keep_results:
                    results[i] = f.result()
        finally:
            with lock:
                remaining[0] -= 1
                if remaining[0] == 0:
                    all_done.set()

    t0 = time.perf_counter()
    if not requests:
        all_done.set()
    for i, (t, keys, vals) in enumerate(requests):
        at = t0 + t / qps
        _wait_until(at)
        arrivals.append(at)
        server.submit(keys, vals, arrival=at).add_done_callback(lambda f, i=i: on_done(i, f))
    all_done.wait()
    wall = time.perf_counter() - t0
    stats = {"batches": server.batches, "mean_batch": round(float(np.mean(server.batch_sizes)), 2),
             "peak_hbm_bytes": server.peak_used, "hbm_budget": server.budget,
             "max_batch_keys": server.max_batch_keys}
    if own:
        server.close()
    if any(tm is None for tm in timings):  # a request failed: its future holds the error
        raise RuntimeError("a request of the serving run failed")
    lat = [tm["finished"] - a for tm, a in zip(timings, arrivals)]
    stats["stage_p50_ms"] = {
        "queued": _p50([tm["admitted"] - tm["submitted"] for tm in timings]),
        "pack_and_enqueue": _p50([tm["launched"] - tm["admitted"] for tm in timings]),
        "device": _p50([tm["done"] - tm["launched"] for tm in timings]),
        "unpack": _p50([tm["finished"] - tm["done"] for tm in timings]),
    }
    return results, lat, wall, stats


def _p50(xs):
    return round(float(np.median(xs)) * 1e3, 3) if xs else 0.0


def run_serving_benchmark(count: int = 400, fracs=(0.5, 0.8, 0.95, 1.5), seed: int = 1, device="cuda:0",
                          hbm_budget: int = 16 << 30, lo: int = 1 << 10, hi: int = 1 << 24,
                          max_batch_keys: int = 1 << 24, resident: str = "host"):
    """p50/p99 latency and Gkeys/s of the batched server and of the serial
    baseline at fractions of the baseline's saturation request rate (above 1:
    more requests per second than one-at-a-time serving can complete), and
    both paths' saturation rates (all requests submitted at once).

    ``resident="host"``: requests and results are host arrays (every request
    crosses PCIe twice); ``"device"``: they are CUDA tensors already in HBM.
    """
    reqs = make_requests(count, lo=lo, hi=hi, seed=seed, device=device if resident == "device" else None)
    total_keys = sum(int(k.numel()) if isinstance(k, torch.Tensor) else k.size for _, k, _ in reqs)
    out = {"requests": count, "resident": resident, "total_keys": int(total_keys), "sizes": [lo, hi],
           "pairs_fraction": 0.5, "hbm_budget_bytes": hbm_budget, "runs": []}
    reserve = 0 if resident == "device" else min(max(hi, max_batch_keys), total_keys)
    with SortServer(device, hbm_budget=hbm_budget, max_batch_keys=max_batch_keys, reserve_keys=reserve) as server:
        # warm up both paths over the whole request set (library load, buffer growth)
        serve_serial(reqs, device, realtime=False, keep_results=False)
        serve_batched(reqs, qps=1e9, server=server, keep_results=False)
        _, _, sat_wall = serve_serial(reqs, device, realtime=False, keep_results=False)
        sat_qps = count / sat_wall
        _, _, bsat_wall, _ = serve_batched(reqs, qps=1e9, server=server, keep_results=False)
        out["serial_saturation_qps"] = round(sat_qps, 2)
        out["batched_saturation_qps"] = round(count / bsat_wall, 2)
        for frac in fracs:
            qps = frac * sat_qps
            timed = [(t / qps, k, v) for t, k, v in reqs]
            _, slat, swall = serve_serial(timed, device, realtime=True, keep_results=False)
            _, blat, bwall, bst = serve_batched(reqs, qps=qps, server=server, keep_results=False)
            out["runs"].append({
                "qps": round(qps, 2), "frac_of_serial_saturation": frac,
                "serial": {**latency_stats(slat), "gkeys_per_s": round(total_keys / swall / 1e9, 4)},
                "batched": {**latency_stats(blat), "gkeys_per_s": round(total_keys / bwall / 1e9, 4), **bst},
            })
    return out
