"""Torch-tensor front end of the C ABI (include/bcf.h).

Tensors must be contiguous uint32 (or int32, reinterpreted bit-for-bit) CUDA
tensors on the same device.  Work is enqueued on ``stream`` (default: torch's
current stream); the calls return without synchronising.  Temporary storage
comes from torch's caching allocator through :class:`Workspace`.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

import contextlib

from ._native import KernelStat, Tuning, check, load

__all__ = [
    "Workspace",
    "sort_u32",
    "sort_pairs_u32",
    "sort_i32",
    "sort_f32",
    "sort_pairs_i32",
    "sort_pairs_f32",
    "colored_prefix_sums",
    "sort_u64",
    "merge_runs",
    "distribute_runs",
    "merge_run_groups",
    "sort_u32_pb",
    "segmented_sort",
    "SegmentedPlan",
    "tile_keys",
    "run_keys",
    "sort_passes",
    "profile_enable",
    "profile_collect",
    "get_tuning",
    "set_tuning",
    "tuning",
]

_U32 = (torch.uint32, torch.int32)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _stream(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream, ctypes.c_void_p(stream.cuda_stream)


def _check_tensor(t, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype not in _U32:
        raise TypeError(f"{name} must be uint32 or int32, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def _device_offsets(off, device):
    """Offsets given as a device tensor (int64 or uint64, contiguous): the
    device-planned entry points take them as they are."""
    if not isinstance(off, torch.Tensor) or not off.is_cuda:
        return None
    if off.dtype not in (torch.int64, torch.uint64) or off.dim() != 1 or not off.is_contiguous():
        raise TypeError("device offsets must be a contiguous 1-D int64 / uint64 CUDA tensor")
    if off.device != device:
        raise ValueError(f"offsets are on {off.device}, expected {device}")
    if off.numel() < 1:
        raise ValueError("offsets must have at least one entry")
    return off


def _offsets(off, total=None):
    a = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    if a.ndim != 1 or a.size < 1:
        raise ValueError("offsets must be a 1-D sequence with at least one entry")
    if total is not None and int(a[-1]) != total:
        raise ValueError(f"last offset {int(a[-1])} != number of keys {total}")
    return a


class Workspace:
    """A reusable device scratch buffer (grows on demand, never shrinks)."""

    def __init__(self, device=None):
        self.device = torch.device(device) if device is not None else None
        self.buf = None

    def get(self, nbytes: int, device, stream=None):
        if nbytes == 0:
            return None
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        if stream is not None and stream != torch.cuda.current_stream(device):
            self.buf.record_stream(stream)
        return self.buf


def _temp(ws, nbytes, device, stream):
    if nbytes == 0:
        return None, ctypes.c_uint64(0)
    if ws is None:
        buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        if stream != torch.cuda.current_stream(device):
            buf.record_stream(stream)
    else:
        buf = ws.get(nbytes, device, stream)
    return buf, ctypes.c_uint64(buf.numel())


def tile_keys() -> int:
    """Keys per wave tile (block sort and merge work item): 4096."""
    return int(load().bcf_tile_keys())


def run_keys(pairs: bool = False) -> int:
    """Length of the sorted runs the block sort hands to the merge passes."""
    return int(load().bcf_run_keys(1 if pairs else 0))


def sort_passes(n: int, pairs: bool = False) -> int:
    """Passes over HBM (block sort + merge passes) of a sort of n keys."""
    return int(load().bcf_sort_passes(n, 1 if pairs else 0))


def sort_u32(keys, out=None, stream=None, workspace=None):
    """Ascending sort of u32 keys; returns ``out``."""
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    _check_tensor(out, "out", keys.device)
    if out.numel() != n:
        raise ValueError("out must have as many elements as keys")
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    check("bcf_sort_u32", lib.bcf_sort_u32(None, None, n, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check(
            "bcf_sort_u32",
            lib.bcf_sort_u32(_ptr(keys), _ptr(out), n, _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh),
        )
    return out


def sort_pairs_u32(keys, vals, keys_out=None, vals_out=None, stream=None, workspace=None):
    """Stable sort of (key, value) pairs by key; returns (keys_out, vals_out)."""
    lib = load()
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals", keys.device)
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and vals must have the same length")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    _check_tensor(keys_out, "keys_out", keys.device)
    _check_tensor(vals_out, "vals_out", keys.device)
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    check("bcf_sort_pairs_u32", lib.bcf_sort_pairs_u32(None, None, None, None, n, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check(
            "bcf_sort_pairs_u32",
            lib.bcf_sort_pairs_u32(
                _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), n,
                _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh,
            ),
        )
    return keys_out, vals_out


def _sort_typed(kind, keys, vals, keys_out, vals_out, stream, workspace):
    """int32 (kind "i32") or float32 ("f32") keys, optionally with u32 values."""
    lib = load()
    dtype = torch.int32 if kind == "i32" else torch.float32
    for name, t in (("keys", keys), ("keys_out", keys_out)):
        if t is not None and (not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda
                              or not t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    n = keys.numel()
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if keys_out.numel() != n or keys_out.device != keys.device:
        raise ValueError("keys_out must match keys")
    pairs = vals is not None
    if pairs:
        _check_tensor(vals, "vals", keys.device)
        if vals.numel() != n:
            raise ValueError("keys and vals must have the same length")
        vals_out = torch.empty_like(vals) if vals_out is None else vals_out
        _check_tensor(vals_out, "vals_out", keys.device)
    fname = f"bcf_sort_{'pairs_' if pairs else ''}{kind}"
    fn = getattr(lib, fname)
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    if pairs:
        check(fname, fn(None, None, None, None, n, None, ctypes.byref(need), None))
    else:
        check(fname, fn(None, None, n, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        tp = _ptr(temp) or ctypes.c_void_p(1)
        if pairs:
            check(fname, fn(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), n, tp, ctypes.byref(tb), sh))
        else:
            check(fname, fn(_ptr(keys), _ptr(keys_out), n, tp, ctypes.byref(tb), sh))
    return (keys_out, vals_out) if pairs else keys_out


def sort_i32(keys, out=None, stream=None, workspace=None):
    """Ascending sort of int32 keys (signed order); returns ``out``."""
    return _sort_typed("i32", keys, None, out, None, stream, workspace)


def sort_f32(keys, out=None, stream=None, workspace=None):
    """Ascending sort of float32 keys in IEEE 754 totalOrder (-0.0 before +0.0,
    NaNs at the ends by sign); returns ``out``."""
    return _sort_typed("f32", keys, None, out, None, stream, workspace)


def sort_pairs_i32(keys, vals, keys_out=None, vals_out=None, stream=None, workspace=None):
    """Stable sort of (int32 key, u32 value) pairs by key."""
    return _sort_typed("i32", keys, vals, keys_out, vals_out, stream, workspace)


def sort_pairs_f32(keys, vals, keys_out=None, vals_out=None, stream=None, workspace=None):
    """Stable sort of (float32 key, u32 value) pairs by key (totalOrder)."""
    return _sort_typed("f32", keys, vals, keys_out, vals_out, stream, workspace)


def sort_u64(keys, out=None, stream=None, workspace=None):
    """Ascending sort of a contiguous torch.uint64 CUDA tensor (``bcf_sort_u64``:
    keys in register pairs, block sort and binary merge passes).  Returns
    ``out``."""
    lib = load()
    for name, t in (("keys", keys), ("out", out)):
        if t is not None and (not isinstance(t, torch.Tensor) or t.dtype != torch.uint64 or not t.is_cuda
                              or not t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous torch.uint64 CUDA tensor")
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else out
    if out.numel() != n or out.device != keys.device:
        raise ValueError("out must match keys")
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    check("bcf_sort_u64", lib.bcf_sort_u64(None, None, n, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check("bcf_sort_u64", lib.bcf_sort_u64(_ptr(keys), _ptr(out), n, _ptr(temp) or ctypes.c_void_p(1),
                                               ctypes.byref(tb), sh))
    return out


def colored_prefix_sums(values, colors, d, conflict_free=True, out=None, stream=None, workspace=None):
    """Per-color inclusive prefix sums of u32 ``values`` (uint8 ``colors`` < d,
    d <= 32); ``conflict_free`` picks the LDS counter layout.  Returns ``out``."""
    lib = load()
    _check_tensor(values, "values")
    if not isinstance(colors, torch.Tensor) or colors.dtype != torch.uint8 or not colors.is_cuda \
            or not colors.is_contiguous() or colors.device != values.device:
        raise TypeError("colors must be a contiguous uint8 tensor on the values' device")
    n = values.numel()
    if colors.numel() != n:
        raise ValueError("values and colors must have the same length")
    out = torch.empty_like(values) if out is None else out
    _check_tensor(out, "out", values.device)
    stream, sh = _stream(stream, values.device)
    need = ctypes.c_uint64(0)
    check("bcf_colored_prefix_sums", lib.bcf_colored_prefix_sums(None, None, None, n, d, 1, None,
                                                                 ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, values.device, stream)
    if n:
        check("bcf_colored_prefix_sums",
              lib.bcf_colored_prefix_sums(_ptr(values), _ptr(colors), _ptr(out), n, d, 1 if conflict_free else 0,
                                          _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh))
    return out


def merge_runs(keys, run_offsets, vals=None, keys_out=None, vals_out=None, stream=None, workspace=None):
    """Stable merge of the sorted runs [off[r], off[r+1]) of ``keys``.

    ``run_offsets`` holds k+1 offsets: a CUDA tensor (int64 / uint64) takes the
    device-planned ``bcf_merge_runs`` (nothing read back while merging), a host
    sequence ``bcf_merge_runs_host``.  Returns ``keys_out``, or
    ``(keys_out, vals_out)`` when ``vals`` is given.
    """
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    doff = _device_offsets(run_offsets, keys.device)
    if doff is not None:
        return _planned(lib.bcf_merge_runs, "bcf_merge_runs", keys, doff, vals, keys_out, vals_out, stream, workspace,
                        merge=True)
    off = _offsets(run_offsets, n)
    k = off.size - 1
    if vals is not None:
        _check_tensor(vals, "vals", keys.device)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    stream, sh = _stream(stream, keys.device)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    need = ctypes.c_uint64(0)
    vdummy = ctypes.c_void_p(1) if vals is not None else None
    check("bcf_merge_runs_host", lib.bcf_merge_runs_host(None, vdummy, offp, k, None, None, None, ctypes.byref(need),
                                                         None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check(
            "bcf_merge_runs_host",
            lib.bcf_merge_runs_host(
                _ptr(keys), _ptr(vals), offp, k, _ptr(keys_out), _ptr(vals_out),
                _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh,
            ),
        )
    return (keys_out, vals_out) if vals is not None else keys_out


def _planned(fn, fname, keys, off, vals, keys_out, vals_out, stream, workspace, merge):
    """A call of a device-planned entry point (offsets in device memory)."""
    k = off.numel() - 1
    if vals is not None:
        _check_tensor(vals, "vals", keys.device)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_tensor(keys_out, "keys_out", keys.device)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    vdummy = ctypes.c_void_p(1) if vals is not None else None
    if merge:
        check(fname, fn(None, vdummy, _ptr(off), k, None, None, None, ctypes.byref(need), sh))
    elif vals is None:
        check(fname, fn(None, None, _ptr(off), k, None, ctypes.byref(need), sh))
    else:
        check(fname, fn(None, None, None, None, _ptr(off), k, None, ctypes.byref(need), sh))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if keys.numel() and k:
        tp = _ptr(temp) or ctypes.c_void_p(1)
        if merge:
            check(fname, fn(_ptr(keys), _ptr(vals), _ptr(off), k, _ptr(keys_out), _ptr(vals_out), tp, ctypes.byref(tb),
                            sh))
        elif vals is None:
            check(fname, fn(_ptr(keys), _ptr(keys_out), _ptr(off), k, tp, ctypes.byref(tb), sh))
        else:
            check(fname, fn(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), _ptr(off), k, tp,
                            ctypes.byref(tb), sh))
    return (keys_out, vals_out) if vals is not None else keys_out


def distribute_runs(keys, run_offsets, P, t, pivot_buckets=False, keys_out=None, stream=None, workspace=None):
    """Distribute the sorted runs [off[r], off[r+1]) of ``keys`` into buckets
    by P-1 sampled splitters (t candidates per run), with 2P-1 pivot buckets
    when ``pivot_buckets``.

    ``run_offsets`` is a host sequence of s+1 offsets.  Returns
    ``(keys_out, piece_offsets, splitters)``: the keys by (bucket, run), the
    nb*s + 1 piece offsets (int64 on the device; piece (b, r) at b*s + r) and
    the P-1 splitters (uint32 on the device).
    """
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    off = _offsets(run_offsets, n)
    s = off.size - 1
    nb = 2 * P - 1 if pivot_buckets else P
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    pieces = torch.empty(nb * s + 1, dtype=torch.int64, device=keys.device)
    spl = torch.empty(max(P - 1, 1), dtype=torch.uint32, device=keys.device)
    stream, sh = _stream(stream, keys.device)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    need = ctypes.c_uint64(0)
    check("bcf_distribute_runs", lib.bcf_distribute_runs(None, offp, s, P, t, int(bool(pivot_buckets)), None, None,
                                                         None, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if s:
        check(
            "bcf_distribute_runs",
            lib.bcf_distribute_runs(
                _ptr(keys) or ctypes.c_void_p(1), offp, s, P, t, int(bool(pivot_buckets)),
                _ptr(keys_out) or ctypes.c_void_p(1), _ptr(pieces), _ptr(spl) if P > 1 else None,
                _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh,
            ),
        )
    return keys_out, pieces, spl[: P - 1]


def merge_run_groups(keys, run_offsets, group_starts, keys_out=None, stream=None, workspace=None):
    """Stable merge of every group of consecutive sorted runs on its own: group
    g is runs [group_starts[g], group_starts[g+1]) (host sequences)."""
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    off = _offsets(run_offsets, n)
    k = off.size - 1
    gs = np.ascontiguousarray(np.asarray(group_starts, dtype=np.uint32))
    ng = gs.size - 1
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    stream, sh = _stream(stream, keys.device)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    gsp = gs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    need = ctypes.c_uint64(0)
    check("bcf_merge_run_groups", lib.bcf_merge_run_groups(None, None, offp, k, gsp, ng, None, None, None,
                                                           ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check("bcf_merge_run_groups", lib.bcf_merge_run_groups(
            _ptr(keys), None, offp, k, gsp, ng, _ptr(keys_out), None, _ptr(temp) or ctypes.c_void_p(1),
            ctypes.byref(tb), sh))
    return keys_out


def bucket_groups(piece_offsets, s, P, pivot_buckets):
    """Run offsets and group starts for the merge of every bucket's pieces
    after a distribution of s runs into P (2P-1 with pivot buckets) buckets:
    group b holds the s pieces of bucket b, except that a pivot bucket, whose
    keys are all equal, is one run (its pieces are already in merged order)."""
    po = np.asarray(piece_offsets, dtype=np.uint64)
    nb = 2 * P - 1 if pivot_buckets else P
    b = np.arange(nb)
    one = (b % 2 == 1) if pivot_buckets else np.zeros(nb, dtype=bool)
    per = np.where(one, 1, s)
    ends = np.where(one[:, None], (b[:, None] + 1) * s, b[:, None] * s + 1 + np.arange(s)[None, :])
    keep = np.arange(s)[None, :] < per[:, None]
    offs = np.concatenate([[0], po[ends[keep]]]).astype(np.uint64)
    starts = np.concatenate([[0], np.cumsum(per)]).astype(np.uint32)
    return offs, starts


def sort_u32_pb(keys, P=256, run_keys=1 << 18, pivot_buckets=True, out=None, stream=None, workspace=None):
    """Sort by distribution (``bcf_sort_u32_pb``: BCFMergesort with the
    distribution step of Sec. 3.2 and, with ``pivot_buckets``, the pivot
    buckets of Sec. 3.3): sort runs of ``run_keys`` keys, distribute them into
    buckets by P-1 sampled splitters (P candidates per run), then merge every
    bucket's pieces, all buckets in one batched merge planned on the device (no
    read-back).  Returns ``out``."""
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else out
    _check_tensor(out, "out", keys.device)
    if out.data_ptr() == keys.data_ptr() and n:
        raise ValueError("sort_u32_pb does not sort in place")
    stream, sh = _stream(stream, keys.device)
    need = ctypes.c_uint64(0)
    piv = int(bool(pivot_buckets))
    check("bcf_sort_u32_pb", lib.bcf_sort_u32_pb(None, None, n, P, run_keys, piv, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        check("bcf_sort_u32_pb", lib.bcf_sort_u32_pb(_ptr(keys), _ptr(out), n, P, run_keys, piv,
                                                     _ptr(temp) or ctypes.c_void_p(1), ctypes.byref(tb), sh))
    return out


def segmented_sort(keys, seg_offsets, vals=None, keys_out=None, vals_out=None, stream=None, workspace=None,
                   out=None):
    """Sort every segment [off[s], off[s+1]) of ``keys`` independently.

    With ``vals`` the sort is a stable key/value sort per segment and
    ``(keys_out, vals_out)`` is returned; otherwise ``keys_out``.
    """
    lib = load()
    _check_tensor(keys, "keys")
    n = keys.numel()
    keys_out = out if keys_out is None else keys_out
    doff = _device_offsets(seg_offsets, keys.device)
    if doff is not None:
        if vals is None:
            return _planned(lib.bcf_segmented_sort, "bcf_segmented_sort", keys, doff, None, keys_out, None, stream,
                            workspace, merge=False)
        return _planned(lib.bcf_segmented_sort_pairs, "bcf_segmented_sort_pairs", keys, doff, vals, keys_out,
                        vals_out, stream, workspace, merge=False)
    off = _offsets(seg_offsets, n)
    nseg = off.size - 1
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if vals is not None:
        _check_tensor(vals, "vals", keys.device)
        vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    stream, sh = _stream(stream, keys.device)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    need = ctypes.c_uint64(0)
    if vals is None:
        check("bcf_segmented_sort_host", lib.bcf_segmented_sort_host(None, None, offp, nseg, None, ctypes.byref(need),
                                                                     None))
    else:
        check("bcf_segmented_sort_pairs_host", lib.bcf_segmented_sort_pairs_host(
            None, None, None, None, offp, nseg, None, ctypes.byref(need), None))
    temp, tb = _temp(workspace, need.value, keys.device, stream)
    if n:
        tp = _ptr(temp) or ctypes.c_void_p(1)
        if vals is None:
            check("bcf_segmented_sort_host", lib.bcf_segmented_sort_host(
                _ptr(keys), _ptr(keys_out), offp, nseg, tp, ctypes.byref(tb), sh))
        else:
            check("bcf_segmented_sort_pairs_host", lib.bcf_segmented_sort_pairs_host(
                _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), offp, nseg, tp, ctypes.byref(tb), sh))
    return (keys_out, vals_out) if vals is not None else keys_out


class SegmentedPlan:
    """A segmented sort planned once for fixed segment offsets.

    The constructor uploads the launch plan into a device buffer owned by the
    plan; :meth:`run` then enqueues kernels only (no copy, no allocation), so
    it can be captured in a graph (:meth:`capture`) and replayed.
    """

    def __init__(self, seg_offsets, device, pairs: bool = False, stream=None):
        lib = load()
        self.device = torch.device(device)
        self.off = _offsets(seg_offsets)
        self.nseg = self.off.size - 1
        self.n = int(self.off[-1]) if self.off.size else 0
        self.pairs = bool(pairs)
        self._offp = self.off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        need = ctypes.c_uint64(0)
        check("bcf_segmented_upload", lib.bcf_segmented_upload(
            self._offp, self.nseg, int(self.pairs), None, ctypes.byref(need), None))
        self.temp = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=self.device)
        self._tb = ctypes.c_uint64(self.temp.numel())
        stream, sh = _stream(stream, self.device)
        if self.n:
            check("bcf_segmented_upload", lib.bcf_segmented_upload(
                self._offp, self.nseg, int(self.pairs), _ptr(self.temp), ctypes.byref(self._tb), sh))

    def run(self, keys, keys_out, vals=None, vals_out=None, stream=None):
        lib = load()
        _check_tensor(keys, "keys", self.device)
        _check_tensor(keys_out, "keys_out", self.device)
        if keys.numel() != self.n or keys_out.numel() != self.n:
            raise ValueError("keys do not match the planned segments")
        if (vals is not None) != self.pairs:
            raise ValueError("values must be given exactly when the plan is for pairs")
        stream, sh = _stream(stream, self.device)
        if self.n:
            check("bcf_segmented_execute", lib.bcf_segmented_execute(
                _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), self._offp, self.nseg,
                _ptr(self.temp), ctypes.byref(self._tb), sh))
        return (keys_out, vals_out) if self.pairs else keys_out

    def capture(self, keys, keys_out, vals=None, vals_out=None):
        """Capture :meth:`run` on fixed buffers into a torch CUDA (HIP) graph."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):  # warm-up outside capture
            self.run(keys, keys_out, vals, vals_out, stream=s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(keys, keys_out, vals, vals_out)
        return g


def profile_enable(on: bool = True):
    """Bracket every library launch with HIP events (see bcf_profile_collect)."""
    load().bcf_profile_enable(1 if on else 0)


def profile_collect():
    """Per-kernel {name: {launches, total_ms, bytes}} since the last collect."""
    buf = (KernelStat * 32)()
    n = load().bcf_profile_collect(buf, 32)
    if n < 0:
        raise RuntimeError("bcf_profile_collect failed")
    return {
        buf[i].name.decode(): {"launches": int(buf[i].launches), "total_ms": buf[i].total_ms, "bytes": buf[i].bytes}
        for i in range(n)
    }


_TUNING_FIELDS = [f[0] for f in Tuning._fields_]


def get_tuning() -> dict:
    """The library's process-wide tuning knobs (see bcf_tuning in include/bcf.h)."""
    t = Tuning()
    load().bcf_get_tuning(ctypes.byref(t))
    return {f: int(getattr(t, f)) for f in _TUNING_FIELDS}


def set_tuning(**knobs) -> dict:
    """Change some knobs; returns the previous setting."""
    prev = get_tuning()
    unknown = set(knobs) - set(_TUNING_FIELDS)
    if unknown:
        raise KeyError(f"unknown tuning knobs {sorted(unknown)}")
    t = Tuning(**{**prev, **knobs})
    check("bcf_set_tuning", load().bcf_set_tuning(ctypes.byref(t)))
    return prev


@contextlib.contextmanager
def tuning(**knobs):
    """Temporarily change tuning knobs."""
    prev = set_tuning(**knobs)
    try:
        yield
    finally:
        set_tuning(**prev)
