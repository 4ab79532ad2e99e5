"""Continuous-batching sort service on one GPU, and its one-call-per-request baseline.

:class:`SortServer` accepts sort requests (u32 keys, or u32/u32 pairs sorted
stably by key) and merge requests (k sorted runs of keys or pairs, merged
stably by run) from any thread.  A launch thread

* admits waiting requests in arrival order while their device bytes fit both
  the HBM budget and the HBM that is actually free on the device
  (``torch.cuda.mem_get_info`` plus what torch's caching allocator holds
  unused), and the batch stays under ``max_batch_keys``; a request larger
  than the whole budget, or larger than the free HBM while nothing else is
  in flight, is rejected with ``MemoryError``;
* packs the admitted requests into one batch: merge requests, requests of at
  least ``solo_keys`` keys, and a request alone in its batch, run on their
  own (``bcf_merge_runs``, ``bcf_sort_u32`` / ``bcf_sort_pairs_u32``), the
  smaller sorts of each kind share one segmented sort
  (``bcf_segmented_sort`` / ``bcf_segmented_sort_pairs``) in which each
  request is a segment;
* runs each batch (host-to-device copy, sorts, device-to-host copy) on the
  stream of one of ``slots`` buffer slots, so up to that many batches are in
  flight and one batch's copies overlap another's kernels; requests that
  arrive meanwhile join the next batch;
* keeps its device buffers and pinned host staging resident between batches
  (they grow on demand and are reused, never freed per request).

A request that arrives while nothing is queued before it, no launch is under
way and a slot is free is launched on the submitting thread itself, so a
request at light load does not wait for the launch thread to wake up (a
device request then runs on the submitting stream, after the work already
there, and needs no event); requests that arrive during a launch, or while
every slot is in flight, queue and are batched by the launch thread.

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
    src: object = None      # device request: the submitting thread's current stream
    ready: object = None    # device request: event recorded on `src` at submission (none when
                            # launched inline: then its work is enqueued on `src` itself)
    runs: object = None     # merge request: its k+1 run offsets (numpy uint64)
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
        return self.src is not None

    @property
    def pairs(self) -> bool:
        return self.vals is not None

    @property
    def merge(self) -> bool:
        return self.runs is not None

    def device_bytes(self) -> int:
        words = 2 if self.pairs else 1
        # input + output arrays, plus merge scratch of the same size and a margin for descriptors
        # (a merge's tables grow with its run count)
        runs = 32 * (len(self.runs) if self.merge else 0)
        return self.n * 4 * words * 3 + 64 * 1024 + runs


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
        self.event = torch.cuda.Event()  # recorded again only once the slot's last batch is complete
        self.done = None
        self.reqs = []
        self.loc = []       # per request: (key lo, key hi, value lo) in the batch buffers


class SortServer:
    """Continuous-batching sort server (see module docstring)."""

    def __init__(self, device="cuda:0", hbm_budget: int = 16 << 30, max_batch_keys: int = 1 << 24,
                 slots: int = 3, reserve_keys: int = 0, solo_keys: int = 1 << 20, hbm_headroom: int = 256 << 20,
                 inline: bool = True):
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_batch_keys = int(max_batch_keys)
        self.solo_keys = int(solo_keys)
        self.headroom = int(hbm_headroom)  # free HBM left untouched by admission
        self.inline = bool(inline)
        self.launching = 0                 # launches under way (launch thread or an inline submit)
        self.min_free_hbm = None           # least device-free HBM seen at an admission
        self._free_at = None               # (free HBM, admitted bytes) at the last query
        self._free_time = 0.0
        self.slots = [_Slot(self.device, reserve_keys) for _ in range(slots)]
        self.free_slots = collections.deque(self.slots)
        self.busy = collections.deque()
        self.pending = collections.deque()
        self.used = 0
        self.peak_used = 0
        self.batches = 0
        self.batch_sizes = []
        # one lock, two conditions: the launch thread waits on `cv` (new
        # requests, freed slots, released holds), the completion thread on
        # `cv_done` (batches in flight), so that neither wakes for the other's
        # events
        self.lock = threading.RLock()
        self.cv = threading.Condition(self.lock)
        self.cv_done = threading.Condition(self.lock)
        self._no_values = torch.empty(0, dtype=torch.uint32, device=self.device)
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
        keys, vals, src = self._inputs(keys, vals)
        return self._enqueue(_Request(keys, vals, time.perf_counter() if arrival is None else arrival, src=src))

    def submit_merge(self, keys, run_offsets, vals=None, arrival: float | None = None) -> Future:
        """Queue one merge request: ``keys`` holds k sorted runs, run r at
        [run_offsets[r], run_offsets[r+1]); the result is their stable merge
        (equal keys: lower run first), keys or (keys, values), host or device
        as for :meth:`submit`.  ``run_offsets`` is a host sequence of k+1
        offsets (a CUDA tensor is read back here, on the submitting thread);
        it must rise from 0 to the number of keys."""
        keys, vals, src = self._inputs(keys, vals)
        if isinstance(run_offsets, torch.Tensor):
            run_offsets = run_offsets.cpu().numpy()
        offs = np.ascontiguousarray(np.asarray(run_offsets, dtype=np.uint64))
        n = int(keys.numel()) if src is not None else int(keys.size)
        if offs.ndim != 1 or offs.size < 1 or int(offs[0]) != 0 or int(offs[-1]) != n or np.any(offs[1:] < offs[:-1]):
            raise ValueError("run_offsets must rise from 0 to the number of keys")
        r = _Request(keys, vals, time.perf_counter() if arrival is None else arrival, src=src, runs=offs)
        return self._enqueue(r)

    def _inputs(self, keys, vals):
        src = None
        if isinstance(keys, torch.Tensor) and keys.is_cuda:
            if keys.dtype != torch.uint32 or keys.device != self.device or not keys.is_contiguous():
                raise ValueError("device keys must be a contiguous uint32 tensor on the server's device")
            if vals is not None and (not isinstance(vals, torch.Tensor) or vals.dtype != torch.uint32
                                     or vals.device != self.device or vals.shape != keys.shape
                                     or not vals.is_contiguous()):
                raise ValueError("device values must be a contiguous uint32 tensor shaped like the keys")
            src = torch.cuda.current_stream(self.device)
        else:
            keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint32))
            if vals is not None:
                vals = np.ascontiguousarray(np.asarray(vals, dtype=np.uint32))
                if vals.shape != keys.shape:
                    raise ValueError("keys and vals must have the same length")
        return keys, vals, src

    def _enqueue(self, r: _Request) -> Future:
        if r.device_bytes() > self.budget:
            r.future.set_exception(MemoryError(f"request of {r.n} keys exceeds the HBM budget"))
            return r.future
        r.submitted = time.perf_counter()
        with self.cv:
            if self.stop:
                raise RuntimeError("server is closed")
            self.pending.append(r)
            # an idle server launches the request on this thread (no hand-off
            # to the launch thread); otherwise the launch thread admits it
            inline = (self.inline and len(self.pending) == 1 and not self.launching and not self.holds
                      and bool(self.free_slots))
            if inline:
                batch = self._take_batch()
                inline = bool(batch)
                if inline:
                    slot = self._begin_launch(batch)
            if not inline:
                if r.on_device:
                    # the server reads the keys after the work the submitter has
                    # enqueued so far (recorded before the launch thread can see r)
                    r.ready = torch.cuda.Event()
                    r.ready.record(r.src)
                self.cv.notify_all()
                return r.future
        try:
            self._run_launch(slot, batch)
        except Exception:
            pass  # the batch's futures hold the error
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
            self.cv_done.notify_all()
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
                self.cv_done.notify_all()

    def _free_hbm(self) -> int:
        """HBM a new allocation can take now: what the device reports free plus
        what torch's caching allocator holds without using it."""
        free, _ = torch.cuda.mem_get_info(self.device)
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        return int(free) + int(cached)

    def _free_estimate(self, need: int, refresh_s: float = 0.05) -> int:
        """Free HBM for admission: the last device query less what was admitted
        since (completions give it back), queried again when that estimate
        does not cover ``need`` or is older than ``refresh_s``."""
        now = time.perf_counter()
        if self._free_at is not None and now - self._free_time < refresh_s:
            free, used = self._free_at
            est = free - (self.used - used)
            if est - self.headroom >= need:
                return est
        free = self._free_hbm()
        self._free_at, self._free_time = (free, self.used), now
        self.min_free_hbm = free if self.min_free_hbm is None else min(self.min_free_hbm, free)
        return free

    def _take_batch(self):
        """Admit requests in arrival order while they fit the batch, the HBM
        budget and the HBM free on the device (called with the lock held).
        Requests already in flight hold their memory, so the free figure
        already excludes them."""
        batch, keys = [], 0
        avail = None
        while self.pending:
            r = self.pending[0]
            if batch and keys + r.n > self.max_batch_keys:
                break
            need = r.device_bytes()
            if self.used + need > self.budget:
                break  # over the budget: wait for completions
            if avail is None:
                avail = self._free_estimate(need) - self.headroom
            if need > avail:
                if not batch and not self.busy and not self.launching:
                    # nothing in flight holds memory that could come back
                    self.pending.popleft()
                    r.future.set_exception(MemoryError(
                        f"request of {r.n} keys needs {need} bytes, {max(avail, 0)} bytes of HBM are free"))
                    continue
                break  # wait for completions to free device memory
            self.pending.popleft()
            batch.append(r)
            keys += r.n
            avail -= need
            self.used += need
        return batch

    def _begin_launch(self, batch):
        """Take a slot for an admitted batch (lock held)."""
        slot = self.free_slots.popleft()
        self.launching += 1
        self.peak_used = max(self.peak_used, self.used)
        self.batches += 1
        self.batch_sizes.append(len(batch))
        return slot

    def _run_launch(self, slot, batch):
        """Enqueue a batch (lock not held) and hand it to the completion thread."""
        now = time.perf_counter()
        for r in batch:
            r.admitted = now
        try:
            self._launch(slot, batch)
        except BaseException as e:
            # nothing of this batch reaches the completion thread: fail its
            # requests and give back the slot and the budget share
            with self.cv:
                self.launching -= 1
                self.used -= sum(r.device_bytes() for r in batch)
                slot.reqs, slot.loc, slot.out, slot.done = [], [], None, None
                self.free_slots.append(slot)
                self.cv.notify_all()
            for r in batch:
                if not r.future.done():
                    r.future.set_exception(e)
            raise
        now = time.perf_counter()
        for r in batch:
            r.launched = now
        with self.cv:
            self.launching -= 1
            self.busy.append(slot)
            self.cv_done.notify()
            if self.pending or self.stop:  # requests that queued meanwhile, or a closing launch thread
                self.cv.notify_all()

    def _launch_loop(self):
        while True:
            with self.cv:
                while True:
                    if self.stop and not self.pending and not self.launching:
                        self.launcher_done = True
                        self.cv_done.notify_all()
                        return
                    batch = []
                    # one launch at a time: the library's host-planned calls share staging
                    if self.pending and self.free_slots and not self.launching and (not self.holds or self.stop):
                        batch = self._take_batch()
                    if batch:
                        break
                    self.cv.wait()
                slot = self._begin_launch(batch)
            self._run_launch(slot, batch)

    def _complete_loop(self):
        while True:
            with self.cv:
                while not self.busy:
                    if self.launcher_done:
                        return
                    self.cv_done.wait()
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
                if self.pending:  # requests waiting for a slot or budget
                    self.cv.notify_all()

    def _launch(self, slot: _Slot, batch):
        if len(batch) == 1 and batch[0].on_device:
            self._launch_alone(slot, batch[0])
            return
        # order in the batch buffers: host requests before device requests, within
        # each keys-only before key/value, small before large, so that the host
        # part is one span (one copy each way) and the small requests of each
        # (residence, kind) group are contiguous; values exist for key/value
        # requests only and follow the same order
        solo = lambda r: r.merge or r.n >= self.solo_keys
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
                    if r.ready is None:
                        raise RuntimeError("a device request launched inline must be alone in its batch")
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
                if r.merge:
                    ki = r.keys if r.on_device else dk[lo:hi]
                    if r.pairs:
                        vi = r.vals if r.on_device else dv[vlo:vlo + r.n]
                        api.merge_runs(ki, r.runs, vals=vi, keys_out=rk[lo:hi], vals_out=rv[vlo:vlo + r.n], stream=st,
                                       workspace=slot.ws)
                    else:
                        api.merge_runs(ki, r.runs, keys_out=rk[lo:hi], stream=st, workspace=slot.ws)
                elif alone or solo(r):
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
            slot.event.record(st)
        slot.done = slot.event

    def _launch_alone(self, slot: _Slot, r: _Request):
        """A device request alone in its batch: sorted or merged from its own
        buffer into fresh outputs, with none of the batch buffers (the common
        case at light load).  Launched inline it runs on the submitting
        stream itself, after the work already there; from the launch thread
        on the slot's stream, after the request's ready event.  The slot's
        workspace is reused only after the batch's done event has completed,
        whichever stream it ran on."""
        slot.reqs, slot.loc = [r], [(0, r.n, 0)]
        queued = r.ready is not None
        st = slot.stream if queued else r.src
        # inline, the submitting stream is already the current one
        with torch.cuda.stream(st) if queued else contextlib.nullcontext():
            if queued:
                st.wait_event(r.ready)
            rk = torch.empty(r.n, dtype=torch.uint32, device=self.device)
            rv = torch.empty(r.n, dtype=torch.uint32, device=self.device) if r.pairs else self._no_values
            if r.merge:
                if r.pairs:
                    api.merge_runs(r.keys, r.runs, vals=r.vals, keys_out=rk, vals_out=rv, stream=st, workspace=slot.ws)
                else:
                    api.merge_runs(r.keys, r.runs, keys_out=rk, stream=st, workspace=slot.ws)
            elif r.pairs:
                api.sort_pairs_u32(r.keys, r.vals, rk, rv, stream=st, workspace=slot.ws)
            else:
                api.sort_u32(r.keys, out=rk, stream=st, workspace=slot.ws)
            slot.event.record(st)
        slot.out = (rk, rv)
        slot.done = slot.event


def serve_serial(requests, device="cuda:0", realtime: bool = True, keep_results: bool = True):
    """Baseline: each request alone (copy in, sort, copy out, synchronise), FIFO.

    ``requests`` is a list of ``(arrival_offset_s, keys, vals_or_None)``, keys
    and values host arrays or CUDA tensors (no copies then), or of
    ``(arrival_offset_s, keys, vals_or_None, run_offsets)`` for a merge of the
    sorted runs ``run_offsets`` delimits (``bcf_merge_runs``); with
    ``realtime`` a request is not started before its arrival time.  Host staging is pinned
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
    for arr, keys, vals, *runs in requests:
        runs = runs[0] if runs else None
        if realtime:
            _wait_until(t0 + arr)
        arrival = t0 + arr if realtime else time.perf_counter()
        if isinstance(keys, torch.Tensor):  # device request: sort into fresh device outputs
            ko = torch.empty_like(keys)
            if vals is not None:
                vo = torch.empty_like(vals)
                if runs is not None:
                    api.merge_runs(keys, runs, vals=vals, keys_out=ko, vals_out=vo, workspace=ws)
                else:
                    api.sort_pairs_u32(keys, vals, ko, vo, workspace=ws)
                res = (ko, vo)
            elif runs is not None:
                res = api.merge_runs(keys, runs, keys_out=ko, workspace=ws)
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
            if runs is not None:
                api.merge_runs(dkk, runs, vals=dvv, keys_out=rkk, vals_out=rvv, workspace=ws)
            else:
                api.sort_pairs_u32(dkk, dvv, rkk, rvv, workspace=ws)
            okk.copy_(rkk, non_blocking=True)
            ovv.copy_(rvv, non_blocking=True)
        else:
            if runs is not None:
                api.merge_runs(dkk, runs, keys_out=rkk, workspace=ws)
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
                  device=None, merge_fraction: float = 0.0, max_runs: int = 16):
    """Seeded serving workload: (arrival_at_qps_1, keys, vals_or_None) per sort
    request, (arrival_at_qps_1, keys, vals_or_None, run_offsets) per merge
    request.

    Sizes are log-uniform in [lo, hi]; half the requests are key/value pairs
    (value = position in the request); keys are slices of one seeded uniform
    pool so that the request set is cheap to build.  A ``merge_fraction`` of
    the requests (chosen by a seeded draw) are merges of 2..``max_runs``
    sorted runs of uneven lengths, each run a slice of the sorted pool.  With
    ``device`` the keys and values are CUDA tensors there (requests already
    resident in HBM), else numpy arrays.
    """
    import workloads

    host_pool = workloads.keys_u32("uniform", pool_keys, seed=seed)
    if device is None:
        pool = host_pool
    else:
        pool = workloads.keys_u32_torch("uniform", pool_keys, torch.device(device), seed=seed)
    spec = workloads.request_stream(count, qps=1.0, lo=lo, hi=hi, seed=seed)
    offs = workloads.draws_u64(seed ^ 0x0FF, count) % np.uint64(max(1, pool_keys - hi))
    mdraw = workloads.draws_u64(seed ^ 0x3E6, count)
    is_merge = (mdraw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) < merge_fraction
    sorted_pool = None
    if is_merge.any():
        sorted_pool = np.sort(host_pool)  # input preparation: runs are slices of a sorted pool
        if device is not None:
            sorted_pool = torch.from_numpy(sorted_pool).to(device)
    reqs = []
    for i, (t, size, pairs, _) in enumerate(spec):
        size = min(size, pool_keys)
        o = int(offs[i])
        if device is None:
            vals = np.arange(size, dtype=np.uint32) if pairs else None
        else:
            vals = torch.arange(size, dtype=torch.int32, device=device).view(torch.uint32) if pairs else None
        if not is_merge[i]:
            reqs.append((t, pool[o:o + size], vals))
            continue
        k = 2 + int(mdraw[i] % np.uint64(max_runs - 1))
        d = workloads.draws_u64(seed * 7919 + i, 2 * k)
        cuts = np.sort(d[:k - 1] % np.uint64(size + 1)).astype(np.int64)
        run_off = np.concatenate([[0], cuts, [size]]).astype(np.uint64)
        starts = (d[k:] % np.uint64(max(1, pool_keys - size))).astype(np.int64)
        pieces = [sorted_pool[int(starts[j]):int(starts[j]) + int(run_off[j + 1] - run_off[j])] for j in range(k)]
        keys = np.concatenate(pieces) if device is None else torch.cat(pieces)
        reqs.append((t, keys, vals, run_off))
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
    for i, (t, keys, vals, *runs) in enumerate(requests):
        at = t0 + t / qps
        _wait_until(at)
        arrivals.append(at)
        if runs:
            fut = server.submit_merge(keys, runs[0], vals, arrival=at)
        else:
            fut = server.submit(keys, vals, arrival=at)
        fut.add_done_callback(lambda f, i=i: on_done(i, f))
    all_done.wait()
    wall = time.perf_counter() - t0
    stats = {"batches": server.batches, "mean_batch": round(float(np.mean(server.batch_sizes)), 2),
             "peak_hbm_bytes": server.peak_used, "hbm_budget": server.budget,
             "min_free_hbm_bytes": server.min_free_hbm, "max_batch_keys": server.max_batch_keys}
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
                          max_batch_keys: int = 1 << 24, resident: str = "host", merge_fraction: float = 0.0):
    """p50/p99 latency and Gkeys/s of the batched server and of the serial
    baseline at fractions of the baseline's saturation request rate (above 1:
    more requests per second than one-at-a-time serving can complete), and
    both paths' saturation rates (all requests submitted at once).

    ``resident="host"``: requests and results are host arrays (every request
    crosses PCIe twice); ``"device"``: they are CUDA tensors already in HBM.
    ``merge_fraction`` of the requests are merges of sorted runs.
    """
    reqs = make_requests(count, lo=lo, hi=hi, seed=seed, device=device if resident == "device" else None,
                         merge_fraction=merge_fraction)
    total_keys = sum(int(k.numel()) if isinstance(k, torch.Tensor) else k.size for _, k, *_ in reqs)
    out = {"requests": count, "resident": resident, "total_keys": int(total_keys), "sizes": [lo, hi],
           "pairs_fraction": 0.5, "merge_fraction": merge_fraction, "hbm_budget_bytes": hbm_budget, "runs": []}
    reserve = 0 if resident == "device" else min(max(hi, max_batch_keys), total_keys)
    with SortServer(device, hbm_budget=hbm_budget, max_batch_keys=max_batch_keys, reserve_keys=reserve) as server:
        # warm up both paths over the whole request set (library load, buffer
        # growth: all at once, then paced so that every slot also sees the
        # large requests alone)
        serve_serial(reqs, device, realtime=False, keep_results=False)
        serve_batched(reqs, qps=1e9, server=server, keep_results=False)
        _, _, sat_wall = serve_serial(reqs, device, realtime=False, keep_results=False)
        sat_qps = count / sat_wall
        serve_batched(reqs, qps=0.5 * sat_qps, server=server, keep_results=False)
        _, _, bsat_wall, _ = serve_batched(reqs, qps=1e9, server=server, keep_results=False)
        out["serial_saturation_qps"] = round(sat_qps, 2)
        out["batched_saturation_qps"] = round(count / bsat_wall, 2)
        for frac in fracs:
            qps = frac * sat_qps
            timed = [(t / qps, *rest) for t, *rest in reqs]
            _, slat, swall = serve_serial(timed, device, realtime=True, keep_results=False)
            _, blat, bwall, bst = serve_batched(reqs, qps=qps, server=server, keep_results=False)
            out["runs"].append({
                "qps": round(qps, 2), "frac_of_serial_saturation": frac,
                "serial": {**latency_stats(slat), "gkeys_per_s": round(total_keys / swall / 1e9, 4)},
                "batched": {**latency_stats(blat), "gkeys_per_s": round(total_keys / bwall / 1e9, 4), **bst},
            })
    return out
