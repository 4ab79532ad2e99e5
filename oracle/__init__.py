"""CPU oracle for the sort library -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``liboracle.so`` (built from ``bcf_oracle.c`` by
``oracle/build.py``).  It is imported only by the tests, by the smoke check and
by the benchmark's CPU-baseline leg; the GPU path neither imports nor links it.

Each function follows the problem statement it names (Sitchinava & Weichert,
Sec. 3: sort n keys ascending; Sec. 3.2: merge sorted sequences); see the C file
for the algorithm.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"oracle library not built: {LIB_PATH} (run oracle/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_sort_u32.argtypes = [u32p, u32p, ctypes.c_uint64]
    lib.oracle_sort_u32.restype = ctypes.c_int
    lib.oracle_sort_pairs_u32.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_uint64]
    lib.oracle_sort_pairs_u32.restype = ctypes.c_int
    lib.oracle_merge_runs.argtypes = [u32p, u32p, u64p, ctypes.c_uint32, u32p, u32p]
    lib.oracle_merge_runs.restype = ctypes.c_int
    lib.oracle_segmented_sort.argtypes = [u32p, u32p, u64p, ctypes.c_uint32]
    lib.oracle_segmented_sort.restype = ctypes.c_int
    lib.oracle_multiset_hash.argtypes = [u32p, u32p, ctypes.c_uint64, u64p, u64p]
    lib.oracle_multiset_hash.restype = None
    lib.oracle_is_sorted_u32.argtypes = [u32p, ctypes.c_uint64]
    lib.oracle_is_sorted_u32.restype = ctypes.c_int
    lib.oracle_sort_typed.argtypes = [ctypes.c_int, u32p, u32p, u32p, u32p, ctypes.c_uint64]
    lib.oracle_sort_typed.restype = ctypes.c_int
    lib.oracle_colored_prefix_sums.argtypes = [u32p, ctypes.POINTER(ctypes.c_uint8), u32p, ctypes.c_uint64,
                                               ctypes.c_uint32]
    lib.oracle_colored_prefix_sums.restype = ctypes.c_int
    lib.oracle_sort_u64.argtypes = [u64p, u64p, ctypes.c_uint64]
    lib.oracle_sort_u64.restype = ctypes.c_int
    lib.oracle_distribute_runs.argtypes = [u32p, u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_int, u32p, u64p, u32p]
    lib.oracle_distribute_runs.restype = ctypes.c_int
    _lib = lib
    return lib


def _p32(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def sort_u32(keys) -> np.ndarray:
    """Ascending sort of u32 keys (top-down merge sort)."""
    k = _u32(keys)
    out = np.empty_like(k)
    if k.size and _load().oracle_sort_u32(_p32(k), _p32(out), k.size) != 0:
        raise MemoryError("oracle_sort_u32")
    return out


def sort_pairs_u32(keys, vals):
    """Stable sort of (key, value) pairs by key."""
    k, v = _u32(keys), _u32(vals)
    assert k.shape == v.shape
    ko, vo = np.empty_like(k), np.empty_like(v)
    if k.size and _load().oracle_sort_pairs_u32(_p32(k), _p32(v), _p32(ko), _p32(vo), k.size) != 0:
        raise MemoryError("oracle_sort_pairs_u32")
    return ko, vo


def merge_runs(keys, offsets, vals=None):
    """Stable k-way merge of the sorted runs [off[r], off[r+1])."""
    k = _u32(keys)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    nr = off.size - 1
    ko = np.empty_like(k)
    v = _u32(vals) if vals is not None else None
    vo = np.empty_like(v) if v is not None else None
    if nr > 0 and _load().oracle_merge_runs(_p32(k), _p32(v), _p64(off), nr, _p32(ko), _p32(vo)) != 0:
        raise ValueError("oracle_merge_runs: bad offsets")
    return (ko, vo) if v is not None else ko


def segmented_sort(keys, offsets) -> np.ndarray:
    """Sort every segment [off[s], off[s+1]) independently."""
    k = _u32(keys)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    ko = np.empty_like(k)
    ns = off.size - 1
    if ns > 0 and _load().oracle_segmented_sort(_p32(k), _p32(ko), _p64(off), ns) != 0:
        raise ValueError("oracle_segmented_sort: bad offsets")
    return ko


def multiset_hash(keys, vals=None):
    """(sum, xor) order-independent hash of the (key, value) multiset."""
    k = _u32(keys)
    v = _u32(vals) if vals is not None else None
    s, x = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _load().oracle_multiset_hash(_p32(k), _p32(v), k.size, ctypes.byref(s), ctypes.byref(x))
    return int(s.value), int(x.value)


def is_sorted_u32(keys) -> bool:
    """True when the keys are nondecreasing."""
    k = _u32(keys)
    return bool(_load().oracle_is_sorted_u32(_p32(k), k.size))


# ---------------------------------------------------------- chunked (all cores)
#
# The same results on several host cores: the input is cut into `threads`
# equal chunks, every chunk is sorted by the plain merge sort above in its own
# thread (ctypes releases the GIL during the C call), then a pairwise merge
# tree joins the sorted chunks, the merges of one level running in parallel.
# Each merge is the stable k-cursor merge of two adjacent runs, so the result
# is the stable sort of the whole input: equal to sort_u32 / sort_pairs_u32.


def _chunk_bounds(n, threads):
    threads = max(1, min(int(threads), n if n else 1))
    return [n * c // threads for c in range(threads + 1)]


def _merge_tree(ks, vs, bounds, pool):
    """Merge the adjacent sorted runs [bounds[i], bounds[i+1]) pairwise, level
    by level; ks/vs are swapped with same-size scratch arrays between levels."""
    src_k, src_v = ks, vs
    dst_k = np.empty_like(ks)
    dst_v = np.empty_like(vs) if vs is not None else None
    while len(bounds) > 2:
        jobs, nb = [], [bounds[0]]
        for i in range(0, len(bounds) - 1, 2):
            lo = bounds[i]
            mid = bounds[i + 1]
            hi = bounds[i + 2] if i + 2 < len(bounds) else mid
            jobs.append((lo, mid, hi))
            nb.append(hi)

        def merge_one(job, sk=src_k, sv=src_v, dk=dst_k, dv=dst_v):
            lo, mid, hi = job
            off = np.array([0, mid - lo, hi - lo], dtype=np.uint64)
            vin = sv[lo:hi] if sv is not None else None
            r = merge_runs(sk[lo:hi], off, vin)
            if sv is not None:
                dk[lo:hi], dv[lo:hi] = r
            else:
                dk[lo:hi] = r

        list(pool.map(merge_one, jobs))
        src_k, dst_k = dst_k, src_k
        if vs is not None:
            src_v, dst_v = dst_v, src_v
        bounds = nb
    return src_k, src_v


def sort_u32_chunked(keys, threads: int) -> np.ndarray:
    """sort_u32 on `threads` host threads (chunk sorts + pairwise merge tree)."""
    from concurrent.futures import ThreadPoolExecutor

    k = _u32(keys)
    bounds = _chunk_bounds(k.size, threads)
    out = np.empty_like(k)
    with ThreadPoolExecutor(max_workers=len(bounds) - 1) as pool:
        def sort_one(c):
            out[bounds[c]:bounds[c + 1]] = sort_u32(k[bounds[c]:bounds[c + 1]])

        list(pool.map(sort_one, range(len(bounds) - 1)))
        res, _ = _merge_tree(out, None, bounds, pool)
    return res


def sort_pairs_u32_chunked(keys, vals, threads: int):
    """sort_pairs_u32 (stable) on `threads` host threads."""
    from concurrent.futures import ThreadPoolExecutor

    k, v = _u32(keys), _u32(vals)
    assert k.shape == v.shape
    bounds = _chunk_bounds(k.size, threads)
    ko, vo = np.empty_like(k), np.empty_like(v)
    with ThreadPoolExecutor(max_workers=len(bounds) - 1) as pool:
        def sort_one(c):
            lo, hi = bounds[c], bounds[c + 1]
            ko[lo:hi], vo[lo:hi] = sort_pairs_u32(k[lo:hi], v[lo:hi])

        list(pool.map(sort_one, range(len(bounds) - 1)))
        return _merge_tree(ko, vo, bounds, pool)


def segmented_sort_threads(keys, offsets, threads: int, vals=None):
    """segmented_sort (or, with vals, the stable pair sort of every segment),
    segments spread over `threads` host threads."""
    from concurrent.futures import ThreadPoolExecutor

    k = _u32(keys)
    off = np.asarray(offsets, dtype=np.uint64)
    ko = np.empty_like(k)
    v = _u32(vals) if vals is not None else None
    vo = np.empty_like(v) if v is not None else None
    nseg = off.size - 1
    # contiguous slices of segments with about equal key counts
    cuts = np.searchsorted(off, np.linspace(0, int(off[-1]), max(1, threads) * 4 + 1), side="left")
    cuts = sorted(set(int(c) for c in np.clip(cuts, 0, nseg)) | {0, nseg})

    def one(i):
        s0, s1 = cuts[i], cuts[i + 1]
        lo, hi = int(off[s0]), int(off[s1])
        sub = off[s0:s1 + 1] - off[s0]
        if v is None:
            ko[lo:hi] = segmented_sort(k[lo:hi], sub)
        else:
            for sg in range(s0, s1):
                a, b = int(off[sg]), int(off[sg + 1])
                ko[a:b], vo[a:b] = sort_pairs_u32(k[a:b], v[a:b])

    with ThreadPoolExecutor(max_workers=max(1, threads)) as pool:
        list(pool.map(one, range(len(cuts) - 1)))
    return (ko, vo) if v is not None else ko


def _sort_typed(kind, dtype, keys, vals):
    k = np.ascontiguousarray(np.asarray(keys, dtype=dtype)).view(np.uint32)
    v = _u32(vals) if vals is not None else None
    ko = np.empty_like(k)
    vo = np.empty_like(v) if v is not None else None
    if k.size and _load().oracle_sort_typed(kind, _p32(k), _p32(v), _p32(ko), _p32(vo), k.size) != 0:
        raise MemoryError("oracle_sort_typed")
    return (ko.view(dtype), vo) if v is not None else ko.view(dtype)


def sort_i32(keys, vals=None):
    """Ascending sort of int32 keys (signed order), stable with values."""
    return _sort_typed(1, np.int32, keys, vals)


def sort_f32(keys, vals=None):
    """Ascending sort of float32 keys in IEEE 754 totalOrder, stable with values."""
    return _sort_typed(2, np.float32, keys, vals)


def sort_u64(keys) -> np.ndarray:
    """Ascending sort of u64 keys (top-down merge sort)."""
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    out = np.empty_like(k)
    if k.size and _load().oracle_sort_u64(_p64(k), _p64(out), k.size) != 0:
        raise MemoryError("oracle_sort_u64")
    return out


def colored_prefix_sums(values, colors, d):
    """Per-color inclusive prefix sums (mod 2^32); colors >= d count as d - 1."""
    v = _u32(values)
    c = np.ascontiguousarray(np.asarray(colors, dtype=np.uint8))
    assert v.shape == c.shape
    out = np.empty_like(v)
    if _load().oracle_colored_prefix_sums(_p32(v), c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _p32(out),
                                          v.size, d) != 0:
        raise ValueError("colored_prefix_sums: d must be in [1, 256]")
    return out


def distribute_runs(keys, run_offsets, P, t, pivot_buckets=False):
    """Distribution of sorted runs into buckets by sampled splitters (Sec. 3.2).

    Returns (keys rearranged by (bucket, run), piece offsets with nb*s + 1
    entries, the P-1 splitters); nb = P, or 2P-1 with pivot buckets.
    """
    k = _u32(keys)
    off = np.ascontiguousarray(np.asarray(run_offsets, dtype=np.uint64))
    s = off.size - 1
    nb = 2 * P - 1 if pivot_buckets else P
    out = np.empty_like(k)
    piece = np.empty(nb * s + 1, dtype=np.uint64)
    spl = np.empty(max(P - 1, 1), dtype=np.uint32)
    rc = _load().oracle_distribute_runs(_p32(k), _p64(off), s, P, t, int(bool(pivot_buckets)), _p32(out),
                                        _p64(piece), _p32(spl))
    if rc == -2:
        raise ValueError("distribute_runs: bad arguments")
    if rc != 0:
        raise MemoryError("oracle_distribute_runs")
    return out, piece, spl[: P - 1]
