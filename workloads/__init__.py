"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module only draws numbers; it contains none of the sorting or merging
arithmetic of the method (the ``sorted`` inputs are ordered by numpy's own
sort, a library routine neither side under test uses).  Every generator but
``sorted``/``reverse`` is counter based: element ``i`` of a stream with seed
``s`` depends only on ``(s, i)``, so any slice can be regenerated
independently; both sides always see bit-identical inputs.

Base generator: the SplitMix64 output function (Steele, Lea & Flood, OOPSLA
2014; the constants are those of Vigna's public-domain reference), applied to
the counter ``(seed << 32) + i``.  A draw is the top 32 bits of the 64-bit
output.

Distributions (the paper's data sets are described in its experimental
section; the MI355X workloads add sorted, reverse, 16-distinct and Zipf):

* ``uniform``   -- u32 uniform over [0, 2^32).
* ``sorted``    -- the ``uniform`` draws in ascending order (numpy's library
                   sort of the same sample), so the multiset and its ties are
                   those of ``uniform``.  This one distribution is not counter
                   based: element i depends on the whole sample.
* ``reverse``   -- ``sorted`` read backwards (descending).
* ``distinct16``-- 16 distinct u32 values; each key picks one by the top 4 bits
                   of its draw.
* ``zipf``      -- Zipf(s=1.2) over 2^20 ranks by inverse CDF; rank r maps to
                   key ``((r-1) * 2654435761) mod 2^32`` (odd multiplier, so
                   the tie structure of the ranks is kept).
* ``paper_random``   -- uniform over [0, 10^6] (the paper's "random" set).
* ``paper_distinct`` -- a shuffled 1..n (the paper's "distinct" set).
* ``paper_01``       -- uniform 0/1 keys (the paper's "0-1" set).
* ``paper_dups``     -- k copies of each of n/k keys, shuffled ("defined
                        duplicates").

64-bit keys (``keys_u64``): ``uniform`` (a full 64-bit draw), ``hi16`` (high half
one of 16 values, low half uniform: ties in the high half), ``lo16`` (the
reverse), ``equal`` (one key), ``sorted`` / ``reverse`` (``sorted`` u32 in the high
half, a uniform low half: equal high halves are not in low-half order),
``extremes`` (drawn from 0, 1, 2^32 - 1, 2^32,
2^63 and 2^64 - 1).

Colored prefix sums take u32 values uniform over [0, 2^32) and uint8 colors
uniform over [0, m) by the multiply-shift map ``(draw * m) >> 32`` of a second
stream; ``m = d`` normally, ``m > d`` to exercise colors out of range.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "DISTRIBUTIONS",
    "splitmix64",
    "draws_u64",
    "draws_u32",
    "keys_u32",
    "pairs_u32",
    "segment_sizes",
    "sorted_runs",
    "request_stream",
    "colored_u32",
    "keys_u64",
]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DISTRIBUTIONS = ("uniform", "sorted", "reverse", "distinct16", "zipf")
PAPER_DISTRIBUTIONS = ("paper_random", "paper_distinct", "paper_01", "paper_dups")

_CHUNK = 1 << 22


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function of the (uint64) counter array ``x``."""
    with np.errstate(over="ignore"):
        z = x + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def draws_u64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """64-bit draws for counters ``(seed << 32) + i``, i in [start, start+n)."""
    out = np.empty(n, dtype=np.uint64)
    base = (int(seed) & 0xFFFFFFFF) << 32
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        ctr = np.arange(start + lo, start + hi, dtype=np.uint64) + np.uint64(base)
        out[lo:hi] = splitmix64(ctr)
    return out


def draws_u32(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Top 32 bits of :func:`draws_u64`."""
    out = np.empty(n, dtype=np.uint32)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        out[lo:hi] = (draws_u64(seed, hi - lo, start + lo) >> np.uint64(32)).astype(np.uint32)
    return out


def _zipf_cdf(s: float = 1.2, ranks: int = 1 << 20) -> np.ndarray:
    r = np.arange(1, ranks + 1, dtype=np.float64)
    w = r ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


_ZIPF_CACHE: dict = {}


def _shuffle_perm(seed: int, n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.permutation(n)


def keys_u32(dist: str, n: int, seed: int = 1) -> np.ndarray:
    """n u32 keys of distribution ``dist`` (see module docstring)."""
    n = int(n)
    if n == 0:
        return np.empty(0, dtype=np.uint32)
    if dist == "uniform":
        return draws_u32(seed, n)
    if dist in ("sorted", "reverse"):
        k = np.sort(draws_u32(seed, n))
        return k if dist == "sorted" else k[::-1].copy()
    if dist == "distinct16":
        vals = draws_u32(seed ^ 0x16, 16)
        sel = (draws_u32(seed, n) >> np.uint32(28)).astype(np.int64)
        return vals[sel]
    if dist == "zipf":
        if "cdf" not in _ZIPF_CACHE:
            _ZIPF_CACHE["cdf"] = _zipf_cdf()
        cdf = _ZIPF_CACHE["cdf"]
        out = np.empty(n, dtype=np.uint32)
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            u = (draws_u64(seed, hi - lo, lo) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
            r = np.searchsorted(cdf, u, side="right").astype(np.uint64)  # r - 1 in [0, 2^20)
            r = np.minimum(r, np.uint64(len(cdf) - 1))
            with np.errstate(over="ignore"):
                out[lo:hi] = ((r * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        return out
    if dist == "paper_random":
        return (draws_u64(seed, n) % np.uint64(1000001)).astype(np.uint32)
    if dist == "paper_distinct":
        return (_shuffle_perm(seed, n) + 1).astype(np.uint32)
    if dist == "paper_01":
        return (draws_u32(seed, n) >> np.uint32(31)).astype(np.uint32)
    if dist == "paper_dups":
        k = 4  # copies per key
        base = np.arange(n, dtype=np.uint64) // np.uint64(k)
        with np.errstate(over="ignore"):
            keys = ((base * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        return keys[_shuffle_perm(seed, n)]
    raise ValueError(f"unknown distribution {dist!r}")


def pairs_u32(dist: str, n: int, seed: int = 1):
    """(keys, values) with value = original index (as u32)."""
    keys = keys_u32(dist, n, seed)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def segment_sizes(count: int, lo: int = 32, hi: int = 1 << 20, seed: int = 1) -> np.ndarray:
    """``count`` sizes floor(exp(U(ln lo, ln hi))) from a seeded stream."""
    u = (draws_u64(seed ^ 0x5E6, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    s = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    return np.clip(s, lo, hi)


def sorted_runs(sizes, seed: int = 1, dist: str = "uniform"):
    """Concatenated keys made of ascending runs of the given sizes, plus offsets.

    Each run is a nondecreasing sequence built without a sort: running sums of
    small seeded increments (so runs may hold repeated keys when ``dist`` is
    ``"dups"``).
    """
    sizes = [int(s) for s in sizes]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(np.asarray(sizes, dtype=np.uint64))
    n = int(offs[-1])
    out = np.empty(n, dtype=np.uint32)
    for r, s in enumerate(sizes):
        if s == 0:
            continue
        d = draws_u64(seed * 7919 + r, s)
        if dist == "dups":
            inc = (d >> np.uint64(62)).astype(np.uint64)  # 0..3, many repeats
        else:
            span = max(1, ((1 << 32) - 1) // s)
            inc = d % np.uint64(span)
        k = np.cumsum(inc, dtype=np.uint64)
        out[int(offs[r]):int(offs[r + 1])] = np.minimum(k, np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out, offs


def request_stream(count: int, qps: float, lo: int = 1 << 10, hi: int = 1 << 24, seed: int = 1):
    """Poisson arrivals: (arrival_time_s, size, is_pairs, key_seed) per request."""
    d = draws_u64(seed ^ 0xA11, 3 * count).reshape(count, 3)
    u0 = ((d[:, 0] >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)
    gaps = -np.log(u0) / float(qps)
    t = np.cumsum(gaps)
    u1 = (d[:, 1] >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    sizes = np.floor(np.exp(math.log(lo) + u1 * (math.log(hi) - math.log(lo)))).astype(np.int64)
    pairs = (d[:, 2] >> np.uint64(63)).astype(bool)
    return [(float(t[i]), int(sizes[i]), bool(pairs[i]), seed * 100003 + i) for i in range(count)]


# ------------------------------------------------------------ torch (device) twins
#
# The same counter-based draws computed with torch int64 arithmetic, so large
# inputs can be generated directly in device memory.  torch has no logical
# right shift on int64, so shifts are masked; products wrap modulo 2^64 like
# the numpy uint64 version.  Bit-identical to draws_u32 / keys_u32("uniform").


def _t_srl(z, s):
    import torch

    return torch.bitwise_and(torch.bitwise_right_shift(z, s), (1 << (64 - s)) - 1)


def _t_u64(x: int):
    return x - (1 << 64) if x >= (1 << 63) else x


def draws_u64_torch(seed: int, n: int, device, start: int = 0):
    """int64 tensor on ``device`` holding the bits of draws_u64(seed, n, start)."""
    import torch

    base = ((int(seed) & 0xFFFFFFFF) << 32) + start
    g, m1, m2 = _t_u64(0x9E3779B97F4A7C15), _t_u64(0xBF58476D1CE4E5B9), _t_u64(0x94D049BB133111EB)
    z = torch.arange(0, n, dtype=torch.int64, device=device) + _t_u64(base % (1 << 64))
    z = z + g
    z = torch.bitwise_xor(z, _t_srl(z, 30)) * m1
    z = torch.bitwise_xor(z, _t_srl(z, 27)) * m2
    return torch.bitwise_xor(z, _t_srl(z, 31))


def draws_u32_torch(seed: int, n: int, device, start: int = 0, chunk: int = 1 << 26):
    """torch.uint32 tensor on ``device`` equal to draws_u32(seed, n, start)."""
    import torch

    out = torch.empty(n, dtype=torch.int32, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = _t_srl(draws_u64_torch(seed, hi - lo, device, start + lo), 32).to(torch.int32)
    return out.view(torch.uint32)


def keys_u32_torch(dist: str, n: int, device, seed: int = 1, chunk: int = 1 << 26):
    """Device twin of keys_u32 for the "uniform" and "zipf" distributions."""
    import torch

    if dist == "uniform":
        return draws_u32_torch(seed, n, device, chunk=chunk)
    if dist != "zipf":
        raise ValueError(f"no device generator for {dist!r}")
    if "cdf" not in _ZIPF_CACHE:
        _ZIPF_CACHE["cdf"] = _zipf_cdf()
    cdf = torch.from_numpy(_ZIPF_CACHE["cdf"]).to(device)
    out = torch.empty(n, dtype=torch.int32, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        u = _t_srl(draws_u64_torch(seed, hi - lo, device, lo), 11).to(torch.float64) * (2.0 ** -53)
        r = torch.searchsorted(cdf, u, right=True).clamp_(max=cdf.numel() - 1)
        out[lo:hi] = ((r * 2654435761) & 0xFFFFFFFF).to(torch.int32)
    return out.view(torch.uint32)


U64_DISTRIBUTIONS = ("uniform", "hi16", "lo16", "equal", "sorted", "reverse", "extremes")
_U64_EXTREMES = np.array([0, 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1], dtype=np.uint64)


def keys_u64(dist: str, n: int, seed: int = 1) -> np.ndarray:
    """n unsigned 64-bit keys of the named distribution (see the module doc)."""
    s32 = np.uint64(32)
    if dist == "uniform":
        return draws_u64(seed, n)
    if dist in ("hi16", "lo16"):
        few = ((draws_u32(seed, n) >> np.uint32(28)) * np.uint32(0x9E3779B9)).astype(np.uint64)  # odd: 16 values
        many = draws_u32(seed ^ 0x64, n).astype(np.uint64)
        return (few << s32) | many if dist == "hi16" else (many << s32) | few
    if dist == "equal":
        return np.full(n, 0x0123456789ABCDEF, dtype=np.uint64)
    if dist in ("sorted", "reverse"):
        k = (keys_u32(dist, n, seed).astype(np.uint64) << s32) | draws_u32(seed ^ 0x64, n).astype(np.uint64)
        return k
    if dist == "extremes":
        return _U64_EXTREMES[draws_u32(seed, n) % np.uint32(_U64_EXTREMES.size)]
    raise ValueError(f"unknown u64 distribution {dist!r}")


_COLOR_SEED = 0xC0105


def colored_u32(n: int, m: int, seed: int = 1):
    """(values u32, colors uint8 uniform over [0, m)), m <= 256."""
    assert 1 <= m <= 256
    vals = draws_u32(seed, n)
    cols = ((draws_u32(seed ^ _COLOR_SEED, n).astype(np.uint64) * np.uint64(m)) >> np.uint64(32)).astype(np.uint8)
    return vals, cols


def colored_u32_torch(n: int, m: int, device, seed: int = 1, chunk: int = 1 << 26):
    """Device twin of colored_u32 (torch.uint32 values, torch.uint8 colors)."""
    import torch

    assert 1 <= m <= 256
    vals = draws_u32_torch(seed, n, device, chunk=chunk)
    cols = torch.empty(n, dtype=torch.uint8, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        draw = _t_srl(draws_u64_torch(seed ^ _COLOR_SEED, hi - lo, device, lo), 32)
        cols[lo:hi] = _t_srl(draw * m, 32).to(torch.uint8)
    return vals, cols


def segment_offsets(sizes) -> np.ndarray:
    """Exclusive prefix sums (uint64) of segment sizes, with the total last."""
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(np.asarray(sizes, dtype=np.uint64))
    return offs
