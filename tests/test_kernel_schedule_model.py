"""CPU model of the HIP kernels' compare-exchange schedule and LDS addresses.

This is a design check of the GPU path, not the oracle: it replays, with
numpy, the exact sequence of register-local compare-exchanges, lane-dependent
complements and STRIDED/BLOCKED transposes that the block-sort and merge
kernels execute on a 64 x 64 tile (w = 64 lanes x 64 registers), and checks

* that the schedule sorts (0-1 principle inputs, random inputs, duplicates);
* that every LDS instruction of a transpose is conflict-free on the measured
  gfx950 geometry (32 banks x 4 bytes): 4-byte accesses (STRIDED, CROSS)
  touch 32 distinct banks in each 32-lane half; 16-byte accesses (BLOCKED,
  four registers per instruction) touch the 32 banks once in each group of 8
  consecutive lanes (one 128-byte pass);
* Batcher's network size (543 comparators for 64 keys) and that it sorts;
* the paper's Fig. 1 view of shared memory (element k in bank k mod w,
  column k div w) for the paper's w = 8 drawing.
"""

import itertools

import numpy as np
import pytest

W = 64  # lanes
E = 64  # registers per lane
T = W * E
PAD = 4  # LDS pad words per 64-word row
STRIDE = E + PAD  # LDS words per row
BANKS = 32
HALF = 32


# ------------------------------------------------------------ comparator lists


def oe_merge(lo, hi, r):
    step = 2 * r
    if step < hi - lo:
        yield from oe_merge(lo, hi, step)
        yield from oe_merge(lo + r, hi, step)
        for i in range(lo + r, hi - r, step):
            yield (i, i + r)
    else:
        yield (lo, lo + r)


def oe_sort(lo, hi):
    if hi - lo >= 1:
        mid = lo + (hi - lo) // 2
        yield from oe_sort(lo, mid)
        yield from oe_sort(mid + 1, hi)
        yield from oe_merge(lo, hi, 1)


def half_clean(d, db):
    """(a, b) pairs: smaller goes to a.  Mirrors half_clean<D, DB>."""
    out = []
    while True:
        for r in range(E):
            if r & d:
                continue
            if db >= 0 and (r >> db) & 1:
                out.append((r + d, r))
            else:
                out.append((r, r + d))
        if d == 1:
            break
        d //= 2
    return out


def apply(regs, pairs):
    """regs: (lanes, E) array; apply compare-exchanges on register pairs."""
    for a, b in pairs:
        x, y = regs[:, a].copy(), regs[:, b].copy()
        regs[:, a] = np.minimum(x, y)
        regs[:, b] = np.maximum(x, y)


def flip(regs, bits):
    m = np.where(bits & 1, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0)).astype(regs.dtype)
    regs ^= m[:, None]


# ---------------------------------------------------------------- layouts


def strided_pos(lane, r):
    return W * r + lane


def blocked_pos(lane, r):
    return E * lane + r


def lds_addr(p):
    return p + PAD * (p // 64)


def to_blocked(regs):
    lanes = np.arange(W)
    lds = {}
    for r in range(E):
        for l in lanes:
            lds[lds_addr(strided_pos(l, r))] = regs[l, r]
    out = np.empty_like(regs)
    for r in range(E):
        for l in lanes:
            out[l, r] = lds[lds_addr(blocked_pos(l, r))]
    return out


def to_strided(regs):
    lanes = np.arange(W)
    lds = {}
    for r in range(E):
        for l in lanes:
            lds[lds_addr(blocked_pos(l, r))] = regs[l, r]
    out = np.empty_like(regs)
    for r in range(E):
        for l in lanes:
            out[l, r] = lds[lds_addr(strided_pos(l, r))]
    return out


def fast_to_blocked(regs):
    # position p held at STRIDED (p % 64, p // 64) moves to BLOCKED (p // 64, p % 64)
    return regs.T.copy()


fast_to_strided = fast_to_blocked


# ----------------------------------------------------------- kernel schedules

OE64 = list(oe_sort(0, E - 1))


def sort_tile_model(tile):
    """tile: (T,) keys in input order; returns the kernel's output tile."""
    lanes = np.arange(W)
    regs = np.empty((W, E), dtype=tile.dtype)
    for r in range(E):  # load_tile: STRIDED
        regs[:, r] = tile[W * r + lanes]
    # sort_tile: the loaded registers are read as BLOCKED lines
    flip(regs, lanes)
    apply(regs, OE64)
    flip(regs, lanes)
    for j in range(1, 7):
        regs = fast_to_strided(regs)
        apply(regs, half_clean(1 << (j - 1), j if j < 6 else -1))
        regs = fast_to_blocked(regs)
        if j < 6:
            flip(regs, lanes >> j)
        apply(regs, half_clean(E // 2, -1))
        if j < 6:
            flip(regs, lanes >> j)
    regs = fast_to_strided(regs)
    out = np.empty_like(tile)
    for r in range(E):  # store_tile: STRIDED
        out[W * r + lanes] = regs[:, r]
    return out


def shear_tile_model(tile):
    """The ShearSort block sort (paper Sec. 3.1, Algorithm 1) as the kernel runs it:
    rows are BLOCKED lines, columns STRIDED lines; six iterations of (snake row
    sort, column sort) and a final ascending row sort."""
    lanes = np.arange(W)
    regs = np.empty((W, E), dtype=tile.dtype)
    for r in range(E):
        regs[:, r] = tile[W * r + lanes]
    for _ in range(6):
        flip(regs, lanes)  # odd rows descending (snake)
        apply(regs, OE64)
        flip(regs, lanes)
        regs = fast_to_strided(regs)
        apply(regs, OE64)  # columns ascending
        regs = fast_to_blocked(regs)
    apply(regs, OE64)  # final row sort, ascending: row-major order
    regs = fast_to_strided(regs)
    out = np.empty_like(tile)
    for r in range(E):
        out[W * r + lanes] = regs[:, r]
    return out


def merge_tile_model(a_piece, b_piece):
    """A ascending at [0, na), B reversed at the end, padding between."""
    na, nb = len(a_piece), len(b_piece)
    pad = np.iinfo(a_piece.dtype).max
    tile = np.full(T, pad, dtype=a_piece.dtype)
    tile[:na] = a_piece
    if nb:
        tile[T - nb:] = b_piece[::-1]
    lanes = np.arange(W)
    regs = np.empty((W, E), dtype=tile.dtype)
    for r in range(E):
        regs[:, r] = tile[W * r + lanes]
    apply(regs, half_clean(E // 2, -1))
    regs = fast_to_blocked(regs)
    apply(regs, half_clean(E // 2, -1))
    regs = fast_to_strided(regs)
    out = np.empty_like(tile)
    for r in range(E):
        out[W * r + lanes] = regs[:, r]
    return out[: na + nb]


# ---------------------------------------------------------------------- tests


def test_batcher_64_size_and_sorts():
    assert len(OE64) == 543
    rng = np.random.default_rng(1)
    for _ in range(200):
        x = rng.integers(0, 4, size=(1, E)).astype(np.uint32)
        y = x.copy()
        apply(y, OE64)
        assert np.array_equal(y[0], np.sort(x[0]))


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_batcher_sorts_every_01_input(n):
    net = list(oe_sort(0, n - 1))
    for bits in itertools.product((0, 1), repeat=n):
        x = np.array([bits], dtype=np.uint32)
        y = x.copy()
        for a, b in net:
            lo, hi = min(y[0, a], y[0, b]), max(y[0, a], y[0, b])
            y[0, a], y[0, b] = lo, hi
        assert list(y[0]) == sorted(bits)


def test_transpose_model_matches_index_permutation():
    regs = np.arange(T, dtype=np.uint32).reshape(W, E)
    assert np.array_equal(to_blocked(regs), fast_to_blocked(regs))
    assert np.array_equal(to_strided(regs), fast_to_strided(regs))


def b32_conflict_free(words):
    """4-byte accesses of 64 lanes: 32 distinct banks in each 32-lane half."""
    banks = np.asarray(words) % BANKS
    return all(len(set(banks[h * HALF:(h + 1) * HALF].tolist())) == HALF for h in range(W // HALF))


def b128_conflict_free(words):
    """16-byte accesses (words w..w+3, w a multiple of 4) of 64 lanes: every group
    of 8 consecutive lanes covers the 32 banks exactly once."""
    words = np.asarray(words)
    if np.any(words % 4):
        return False  # not 16-byte aligned
    for g in range(W // 8):
        banks = sorted(int((w + k) % BANKS) for w in words[8 * g:8 * g + 8] for k in range(4))
        if banks != list(range(BANKS)):
            return False
    return True


# Half-width transposes (9 KiB of LDS per wave): v_permlane32_swap on
# registers r and r + 32 gives register r the lower half-waves of both and
# register r + 32 their upper half-waves (the swap of the off-diagonal 32 x 32
# quadrants of M[register][lane]); each half-wave then transposes its two
# 32 x 32 blocks (registers 0..31, then 32..63) through a 32-row LDS matrix with
# rows of HALF_STRIDE words: STRIDED side word 36 r + l', BLOCKED side 36 l' + c.

HALF_STRIDE = 36


def permlane32_swap(x, y):
    """v_permlane32_swap_b32 on one register pair (lanes are array rows)."""
    nx, ny = x.copy(), y.copy()
    nx[HALF:], ny[:HALF] = y[:HALF], x[HALF:]
    return nx, ny


def swap_quadrants(regs):
    out = regs.copy()
    for r in range(E // 2):
        out[:, r], out[:, r + E // 2] = permlane32_swap(regs[:, r], regs[:, r + E // 2])
    return out


def half_word(lane, row, col):
    """LDS word of (row, col) of the lane's half-wave matrix."""
    return (lane // HALF) * HALF * HALF_STRIDE + HALF_STRIDE * row + col


def half_block_transpose(regs, r0, s2b):
    lanes = np.arange(W)
    lds = {}
    out = regs.copy()
    for k in range(HALF):
        for l in lanes:
            w = half_word(l, k, l % HALF) if s2b else half_word(l, l % HALF, k)
            lds[w] = regs[l, r0 + k]
    for k in range(HALF):
        for l in lanes:
            w = half_word(l, l % HALF, k) if s2b else half_word(l, k, l % HALF)
            out[l, r0 + k] = lds[w]
    return out


def to_blocked_half(regs):
    x = swap_quadrants(regs)
    return half_block_transpose(half_block_transpose(x, 0, True), E // 2, True)


def to_strided_half(regs):
    x = half_block_transpose(half_block_transpose(regs, 0, False), E // 2, False)
    return swap_quadrants(x)


def test_half_width_transposes_match_index_permutation():
    regs = np.arange(T, dtype=np.uint32).reshape(W, E)
    assert np.array_equal(to_blocked_half(regs), fast_to_blocked(regs))
    assert np.array_equal(to_strided_half(regs), fast_to_strided(regs))
    assert np.array_equal(to_strided_half(to_blocked_half(regs)), regs)


def test_half_width_transposes_conflict_free_and_fit():
    lanes = np.arange(W)
    for k in range(HALF):  # 4-byte STRIDED-side accesses
        assert b32_conflict_free(half_word(lanes, k, lanes % HALF)), k
    for c in range(0, HALF, 4):  # 16-byte BLOCKED-side accesses
        assert b128_conflict_free(half_word(lanes, lanes % HALF, c)), c
    words = {half_word(l, k, l % HALF) for l in range(W) for k in range(HALF)}
    assert len(words) == W * HALF and max(words) < 2 * HALF * HALF_STRIDE  # 2304 words = 9 KiB


def test_lds_transposes_conflict_free_on_gfx950_geometry():
    lanes = np.arange(W)
    for r in range(E):
        assert b32_conflict_free(lds_addr(strided_pos(lanes, r))), r
    for r in range(0, E, 4):  # BLOCKED side: four consecutive registers per 16-byte access
        assert b128_conflict_free(lds_addr(blocked_pos(lanes, r))), r
    # 4-byte BLOCKED accesses would conflict 4-way on this layout (the kernels never issue them)
    assert not b32_conflict_free(lds_addr(blocked_pos(lanes, 0)))
    # the unpadded layout would conflict 32-way for the BLOCKED accesses
    banks = (blocked_pos(lanes, 0)) % BANKS
    assert len(set(banks[:HALF].tolist())) == 1
    # the padded address map is injective on the tile and fits the LDS array
    addrs = lds_addr(np.arange(T))
    assert len(set(addrs.tolist())) == T and addrs.max() < W * STRIDE


@pytest.mark.parametrize("dist", ["random", "zero_one", "dups", "sorted", "reverse"])
def test_block_sort_schedule_sorts(dist):
    rng = np.random.default_rng(7)
    for _ in range(3):
        if dist == "random":
            x = rng.integers(0, 2**32, size=T, dtype=np.uint64).astype(np.uint32)
        elif dist == "zero_one":
            x = rng.integers(0, 2, size=T).astype(np.uint32)
        elif dist == "dups":
            x = rng.integers(0, 5, size=T).astype(np.uint32) * np.uint32(0x40000000)
        elif dist == "sorted":
            x = np.sort(rng.integers(0, 2**32, size=T, dtype=np.uint64).astype(np.uint32))
        else:
            x = np.sort(rng.integers(0, 2**32, size=T, dtype=np.uint64).astype(np.uint32))[::-1].copy()
        assert np.array_equal(sort_tile_model(x), np.sort(x))


def test_block_sort_schedule_01_principle_sampled():
    # 0-1 inputs with every possible count of ones at random positions
    rng = np.random.default_rng(3)
    for ones in list(range(0, 130)) + list(range(T - 130, T + 1)) + list(rng.integers(0, T, 60)):
        x = np.zeros(T, dtype=np.uint32)
        x[rng.permutation(T)[:ones]] = 1
        assert np.array_equal(sort_tile_model(x), np.sort(x))


def test_block_sort_schedule_stable_pairs():
    # (key, rank) composite packed into 64 bits: the network sorts by it, so
    # the order of equal keys follows the rank (load position).
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 3, size=T).astype(np.uint64)
    comp = (keys << np.uint64(32)) | np.arange(T, dtype=np.uint64)
    out = sort_tile_model(comp)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(out & np.uint64(0xFFFFFFFF), order.astype(np.uint64))


@pytest.mark.parametrize("na,nb", [(0, 4096), (4096, 0), (2048, 2048), (1, 4095), (4095, 1),
                                   (1000, 3096), (3000, 0), (0, 17), (5, 7), (2047, 2049)])
def test_merge_tile_schedule(na, nb):
    rng = np.random.default_rng(na * 7919 + nb)
    a = np.sort(rng.integers(0, 50, size=na).astype(np.uint32))
    b = np.sort(rng.integers(0, 50, size=nb).astype(np.uint32))
    assert np.array_equal(merge_tile_model(a, b), np.sort(np.concatenate([a, b])))


def test_merge_tile_schedule_01_exhaustive_boundaries():
    # 0-1 principle for merging: A = 0^x 1^(na-x), B = 0^y 1^(nb-y)
    for na, nb in [(4096, 0), (2048, 2048), (1024, 3072)]:
        for x in range(0, na + 1, max(1, na // 64)):
            for y in range(0, nb + 1, max(1, nb // 64)):
                a = np.array([0] * x + [1] * (na - x), dtype=np.uint32)
                b = np.array([0] * y + [1] * (nb - y), dtype=np.uint32)
                got = merge_tile_model(a, b)
                assert got.sum() == (na - x) + (nb - y) and np.all(np.diff(got.astype(np.int64)) >= 0)


def test_paper_fig1_bank_matrix_view():
    # Fig. 1 (w = 8 banks): A_k sits in bank k mod 8, column k div 8.
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "fig1_bank_matrix_w8.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for bank, *elems in rows:
        for col, name in enumerate(elems):
            k = int(name[2:])
            assert k % 8 == int(bank) and k // 8 == col


# ------------------------------------------------- group (multi-wave) sort


def lds_word(p):
    return p + PAD * (p // 64)


def group_sort_model(x, nw):
    """Replays k_block_sort_group<NW>: per-wave sorts, then cross-wave rounds
    through the BLOCKED / CROSS / STRIDED layouts with the kernel's LDS words."""
    lw = nw.bit_length() - 1
    lanes = np.arange(W)
    regs = []
    for w in range(nw):
        R = np.empty((W, E), dtype=x.dtype)
        for r in range(E):
            R[:, r] = x[T * w + W * r + lanes]
        flip(R, np.full(W, w & 1))
        flip(R, lanes)
        apply(R, OE64)
        flip(R, lanes)
        for j in range(1, 7):
            R = fast_to_strided(R)
            apply(R, half_clean(1 << (j - 1), j if j < 6 else -1))
            R = fast_to_blocked(R)
            if j < 6:
                flip(R, lanes >> j)
            apply(R, half_clean(E // 2, -1))
            if j < 6:
                flip(R, lanes >> j)
        flip(R, np.full(W, w & 1))
        regs.append(R)

    def move(src_pos, dst_pos):
        lds = {}
        for w in range(nw):
            for r in range(E):
                for l in range(W):
                    lds[lds_word(src_pos(w, l, r))] = regs[w][l, r]
        out = []
        for w in range(nw):
            R = np.empty((W, E), dtype=x.dtype)
            for r in range(E):
                for l in range(W):
                    R[l, r] = lds[lds_word(dst_pos(w, l, r))]
            out.append(R)
        return out

    blocked = lambda w, l, r: T * w + W * l + r
    strided = lambda w, l, r: T * w + W * r + l
    cross = lambda w, l, r: l + W * w + W * nw * r
    for J in range(7, 7 + lw):
        last = J == 6 + lw
        regs = move(blocked, cross)
        for R in regs:
            apply(R, half_clean(1 << (J - 1 - lw), -1 if last else J - lw))
        regs = move(cross, strided)
        for w, R in enumerate(regs):
            if not last:
                flip(R, np.full(W, (w >> (J - 6)) & 1))
            apply(R, half_clean(1 << (lw - 1), -1))
            R2 = fast_to_blocked(R)
            apply(R2, half_clean(E // 2, -1))
            if not last:
                flip(R2, np.full(W, (w >> (J - 6)) & 1))
            regs[w] = R2
    out = np.empty(nw * T, dtype=x.dtype)
    for w in range(nw):
        R = fast_to_strided(regs[w])
        for r in range(E):
            out[T * w + W * r + lanes] = R[:, r]
    return out


@pytest.mark.parametrize("nw", [4, 8])
def test_group_sort_schedule_sorts(nw):
    rng = np.random.default_rng(nw)
    for x in (rng.integers(0, 2**32, size=nw * T, dtype=np.uint64).astype(np.uint32),
              rng.integers(0, 2, size=nw * T).astype(np.uint32),
              np.arange(nw * T, dtype=np.uint32)[::-1].copy()):
        assert np.array_equal(group_sort_model(x, nw), np.sort(x))


@pytest.mark.parametrize("nw", [4, 8])
def test_group_layouts_conflict_free(nw):
    lanes = np.arange(W)
    layouts = {
        "blocked": lambda w, l, r: T * w + W * l + r,
        "strided": lambda w, l, r: T * w + W * r + l,
        "cross": lambda w, l, r: l + W * w + W * nw * r,
    }
    for name, pos in layouts.items():
        for w in range(nw):
            if name == "blocked":  # 16-byte accesses, four registers each
                for r in range(0, E, 4):
                    assert b128_conflict_free(lds_word(pos(w, lanes, r))), (name, w, r)
            else:
                for r in range(E):
                    assert b32_conflict_free(lds_word(pos(w, lanes, r))), (name, w, r)
    # every layout is a bijection onto the group tile, inside the LDS array
    for pos in layouts.values():
        ps = {pos(w, l, r) for w in range(nw) for l in range(W) for r in range(E)}
        assert ps == set(range(nw * T))
    assert lds_word(nw * T - 1) < nw * W * STRIDE


# -------------------------------------------- co-rank search from samples


def corank_brute(a, b, d):
    """Elements of A among the first d outputs of the stable merge (A first on ties)."""
    i = max(0, d - len(b))
    while i < min(d, len(a)) and not (a[i] > b[d - 1 - i]):
        i += 1
    return i


def corank_level(lo, hi, g, pred, probes_per_round=64):
    """Mirror of corank_level<G> (64 probes per round) and corank_level_half<G>
    (32) over candidates g*c in [lo, hi)."""
    P = probes_per_round
    sh = P.bit_length() - 1
    c0 = (lo + g - 1) // g
    c1 = (hi - 1) // g + 1 if hi > 0 else 0
    while c0 < c1:
        span = c1 - c0
        probes = [c0 + (span * k >> sh) for k in range(P)]
        fails = [not pred(g * c) for c in probes]
        cnt = sum(fails)
        assert fails == [True] * cnt + [False] * (P - cnt)  # monotone
        if cnt == 0:
            hi = min(hi, g * c0)
            break
        cf = probes[cnt - 1]
        lo = max(lo, g * cf + 1)
        if cnt < P:
            cn = probes[cnt]
            hi = min(hi, g * cn)
            c1 = cn
        c0 = cf + 1
    return lo, hi


def corank_sampled(arr, apos, na, nb, d, probes_per_round=64):
    """The three levels of k_partition_sampled on one array holding A then B."""
    f = arr[::64]
    l = arr[63::64]
    cf = arr[::4096]
    cl = arr[4095::4096]
    bpos = apos + na
    P = probes_per_round
    lo, hi = max(0, d - nb), min(d, na)
    lo, hi = corank_level(lo, hi, 4096, lambda i: cf[(apos + i) // 4096] > cl[(bpos + d - 1 - i) // 4096], P)
    assert hi - lo <= 4096
    lo, hi = corank_level(lo, hi, 64, lambda i: f[(apos + i) // 64] > l[(bpos + d - 1 - i) // 64], P)
    assert hi - lo <= 64
    lo, hi = corank_level(lo, hi, 1, lambda i: arr[apos + i] > arr[bpos + d - 1 - i], P)
    assert lo == hi
    return lo


@pytest.mark.parametrize("na,nb,levels", [(32768, 32768, 3), (32768, 5000, 7), (65536, 65536, 2), (32768, 0, 1),
                                          (32768, 32768, 40000)])
def test_corank_from_samples_matches_brute_force(na, nb, levels):
    rng = np.random.default_rng(na + nb + levels)
    apos = 3 * 65536  # runs start at multiples of 4096
    arr = np.zeros(apos + na + nb + 4096, dtype=np.int64)
    a = np.sort(rng.integers(0, levels, size=na))
    b = np.sort(rng.integers(0, levels, size=nb))
    arr[apos:apos + na] = a
    arr[apos + na:apos + na + nb] = b
    for d in range(0, na + nb, 4096):
        want = corank_brute(a, b, d)
        assert corank_sampled(arr, apos, na, nb, d) == want, d
        assert corank_sampled(arr, apos, na, nb, d, probes_per_round=32) == want, d


@pytest.mark.parametrize("dist", ["random", "zero_one", "dups", "reverse"])
def test_shear_sort_schedule_sorts(dist):
    rng = np.random.default_rng(17)
    if dist == "random":
        x = rng.integers(0, 2**32, size=T, dtype=np.uint64).astype(np.uint32)
    elif dist == "zero_one":
        x = rng.integers(0, 2, size=T).astype(np.uint32)
    elif dist == "dups":
        x = rng.integers(0, 5, size=T).astype(np.uint32)
    else:
        x = np.arange(T, dtype=np.uint32)[::-1].copy()
    assert np.array_equal(shear_tile_model(x), np.sort(x))


def test_shear_sort_schedule_01_principle_sampled():
    # ShearSort needs ceil(log2 64) = 6 iterations plus the final row phase
    # (2 log w + 1 line sorts, Sec. 3.1); 0-1 inputs with every count of ones
    # near the ends and random counts in between
    rng = np.random.default_rng(19)
    for ones in list(range(0, 70)) + list(range(T - 70, T + 1)) + list(rng.integers(0, T, 40)):
        x = np.zeros(T, dtype=np.uint32)
        x[rng.permutation(T)[:ones]] = 1
        assert np.array_equal(shear_tile_model(x), np.sort(x))


# ------------------------------------------------- fan-in 4 merge pass plan
#
# Model of the four-way merge pass: the merge of runs A, B, C, D (a group of
# four consecutive runs of length L) is the binary merge of AB = merge(A, B)
# and CD = merge(C, D).  The pass cuts the four-way merge path at every
# multiple of AB_STEP of AB (AB cuts) and at every multiple of CD_STEP of CD
# (CD cuts); each cut is found with binary co-ranks and single-run rank
# searches only.  Consecutive AB cuts bound a segment; a segment whose CD side
# is longer than CD_STEP is cut again at the CD cuts strictly inside it, so
# every merge item holds at most AB_STEP elements of AB and CD_STEP of CD and
# fits one tile (AB in the lower half, CD in the upper half).

AB_STEP = 1920
CD_STEP = 2048


def bitonic_tile_network(tile):
    """The merge network of a bitonic 4096-slot tile (STRIDED in, STRIDED out)."""
    lanes = np.arange(W)
    regs = np.empty((W, E), dtype=tile.dtype)
    for r in range(E):
        regs[:, r] = tile[W * r + lanes]
    apply(regs, half_clean(E // 2, -1))
    regs = fast_to_blocked(regs)
    apply(regs, half_clean(E // 2, -1))
    regs = fast_to_strided(regs)
    out = np.empty_like(tile)
    for r in range(E):
        out[W * r + lanes] = regs[:, r]
    return out


def rank_sampled(arr, rpos, nr, k, strict, probes_per_round=32):
    """Elements of the sorted run arr[rpos:rpos+nr] below k (strict: at most
    k): three levels over tile samples, block samples and keys."""
    cf, f = arr[::4096], arr[::64]
    pred = (lambda v: v > k) if strict else (lambda v: v >= k)
    lo, hi = 0, nr
    lo, hi = corank_level(lo, hi, 4096, lambda i: pred(cf[(rpos + i) // 4096]), probes_per_round)
    assert hi - lo <= 4096
    lo, hi = corank_level(lo, hi, 64, lambda i: pred(f[(rpos + i) // 64]), probes_per_round)
    assert hi - lo <= 64
    lo, hi = corank_level(lo, hi, 1, lambda i: pred(arr[rpos + i]), probes_per_round)
    assert lo == hi
    return lo


def corank_blocks(arr, apos, na, nb, d, probes_per_round=64):
    """corank_sampled for a diagonal that is a multiple of 64 only: the first
    level steps 4096 candidates at a time but reads block samples."""
    f, l = arr[::64], arr[63::64]
    bpos = apos + na
    lo, hi = max(0, d - nb), min(d, na)
    bp = lambda i: f[(apos + i) // 64] > l[(bpos + d - 1 - i) // 64]
    lo, hi = corank_level(lo, hi, 4096, bp, probes_per_round)
    lo, hi = corank_level(lo, hi, 64, bp, probes_per_round)
    lo, hi = corank_level(lo, hi, 1, lambda i: arr[apos + i] > arr[bpos + d - 1 - i], probes_per_round)
    assert lo == hi
    return lo


def tile_from_strided(regs):
    out = np.empty(W * E, dtype=regs.dtype)
    lanes = np.arange(W)
    for r in range(E):
        out[W * r + lanes] = regs[:, r]
    return out


def strided_from_tile(tile):
    lanes = np.arange(W)
    regs = np.empty((W, E), dtype=tile.dtype)
    for r in range(E):
        regs[:, r] = tile[W * r + lanes]
    return regs


def packed_item_model(pieces):
    """Both sides of at most 2048 keys: A ascending at the front of the lower
    half, B reversed at its back, C and D the same in the upper half; one
    network without the top stage merges both halves, a transpose reverses
    the upper half, and the full network merges the bitonic result."""
    a, b, c, d = pieces
    assert len(a) + len(b) <= 2048 and len(c) + len(d) <= 2048
    pad = np.iinfo(a.dtype).max
    tile = np.full(T, pad, dtype=a.dtype)
    tile[:len(a)] = a
    if len(b):
        tile[2048 - len(b):2048] = b[::-1]
    tile[2048:2048 + len(c)] = c
    if len(d):
        tile[T - len(d):] = d[::-1]
    regs = strided_from_tile(tile)
    apply(regs, half_clean(E // 4, -1))  # register bits 4..0 = position bits 10..6
    regs = fast_to_blocked(regs)
    apply(regs, half_clean(E // 2, -1))
    regs = fast_to_strided(regs)
    mid = tile_from_strided(regs)
    assert np.array_equal(mid[:2048], np.sort(tile[:2048]))
    assert np.array_equal(mid[2048:], np.sort(tile[2048:]))
    mid[2048:] = mid[2048:][::-1].copy()
    return bitonic_tile_network(mid)


def group_runs(n, L, g):
    base = 4 * L * g
    return base, [int(min(max(n - base - r * L, 0), L)) for r in range(4)]


def ceil_div(a, b):
    return -(-a // b)


def ab_segments(nab):
    return ceil_div(nab, AB_STEP) if nab > AB_STEP else 1


def cd_cuts(ncd):
    return (ncd - 1) // CD_STEP if ncd else 0


def cuts4_model(arr, n, L, g):
    """AB cuts P[0..J] and CD cuts Q[1..M] of group g, each as the counts
    (a, b, c, d) taken from A, B, C and D before the cut."""
    base, (na, nb, nc, nd) = group_runs(n, L, g)
    A, B, C, D = (base + r * L for r in range(4))
    J, M = ab_segments(na + nb), cd_cuts(nc + nd)
    P = [None] * (J + 1)
    P[0], P[J] = (0, 0, 0, 0), (na, nb, nc, nd)
    for j in range(1, J):
        x = AB_STEP * j
        a = corank_blocks(arr, A, na, nb, x)
        b = x - a
        k = arr[A + a] if a < na and (b >= nb or arr[A + a] <= arr[B + b]) else arr[B + b]
        P[j] = (a, b, rank_sampled(arr, C, nc, k, False), rank_sampled(arr, D, nd, k, False))
    Q = [None] * (M + 1)
    for m in range(1, M + 1):
        y = CD_STEP * m
        c = corank_blocks(arr, C, nc, nd, y)
        e = y - c
        k = arr[C + c] if c < nc and (e >= nd or arr[C + c] <= arr[D + e]) else arr[D + e]
        Q[m] = (rank_sampled(arr, A, na, k, True), rank_sampled(arr, B, nb, k, True), c, e)
    return P, Q


def items4_model(P, Q):
    """The merge items of one group, as (first cut, last cut), the way the
    work-group slots of the merge launch decode them: AB item j for every
    segment, CD item m for every CD cut strictly inside a long segment."""
    J, M = len(P) - 1, len(Q) - 1
    ycd = lambda p: p[2] + p[3]
    items = []
    for j in range(J):
        y0, y1 = ycd(P[j]), ycd(P[j + 1])
        items.append((P[j], Q[y0 // CD_STEP + 1] if y1 - y0 > CD_STEP else P[j + 1]))
    for m in range(1, M + 1):
        xq, gm = Q[m][0] + Q[m][1], CD_STEP * m
        jc = min(J - 1, xq // AB_STEP)
        before = jc > 0 and P[jc][0] + P[jc][1] == xq and ycd(P[jc]) > gm
        js = jc - 1 if before else jc
        y0, y1 = ycd(P[js]), ycd(P[js + 1])
        if not (y1 > y0 + CD_STEP and y0 < gm < y1):
            continue
        items.append((Q[m], Q[m + 1] if m < M and CD_STEP * (m + 1) < y1 else P[js + 1]))
    return items


def merge4_item_model(arr, n, L, g, c0, c1, out, smp):
    """One merge item: a copy (one piece), one binary merge network (two
    pieces) or the packed tile's two networks (three or four); samples at
    global positions."""
    base, _ = group_runs(n, L, g)
    starts = [base + r * L for r in range(4)]
    lens = [c1[i] - c0[i] for i in range(4)]
    assert min(lens) >= 0
    pieces = [arr[starts[r] + c0[r]:starts[r] + c0[r] + lens[r]] for r in range(4)]
    sx, sy = lens[0] + lens[1], lens[2] + lens[3]
    assert sx <= 2048 and sy <= 2048
    cnt = sx + sy
    nonempty = [p for p in pieces if len(p)]
    pad = np.iinfo(arr.dtype).max
    if len(nonempty) >= 3:
        tile = packed_item_model(pieces)
        smp["packed"] = smp.get("packed", 0) + 1
    elif len(nonempty) == 2:
        tile = np.full(T, pad, dtype=arr.dtype)
        tile[:cnt] = merge_tile_model(nonempty[0], nonempty[1])[:cnt]
    else:
        tile = np.full(T, pad, dtype=arr.dtype)
        tile[:cnt] = nonempty[0]
    obase = base + sum(c0)
    out[obase:obase + cnt] = tile[:cnt]
    for p in range(cnt):  # the kernel writes exactly these sample words
        gp = obase + p
        if gp % 64 == 0:
            smp["f"][gp // 64] = tile[p]
        if gp % 64 == 63:
            smp["l"][gp // 64] = tile[p]
        if gp % 4096 == 0:
            smp["cf"][gp // 4096] = tile[p]
        if gp % 4096 == 4095:
            smp["cl"][gp // 4096] = tile[p]


def merge4_pass_model(arr, n, L):
    """Every group's cuts and items; returns the output and its samples."""
    out = np.full_like(arr, -1)
    smp = {k: np.full(ceil_div(n, s), -1, dtype=arr.dtype) for k, s in (("f", 64), ("l", 64), ("cf", 4096),
                                                                          ("cl", 4096))}
    smp["packed"] = 0
    for g in range(ceil_div(n, 4 * L)):
        P, Q = cuts4_model(arr, n, L, g)
        items = sorted(items4_model(P, Q), key=lambda it: sum(it[0]))
        cur = (0, 0, 0, 0)
        for c0, c1 in items:  # the items tile the group's merge path exactly once
            assert c0 == cur, (g, c0, cur)
            assert all(c0[r] <= c1[r] for r in range(4)), (g, c0, c1)
            assert c1[0] + c1[1] - c0[0] - c0[1] <= AB_STEP and c1[2] + c1[3] - c0[2] - c0[3] <= CD_STEP
            merge4_item_model(arr, n, L, g, c0, c1, out, smp)
            cur = c1
        assert cur == P[-1]
    return out, smp


def _runs_input(n, L, dist, seed):
    rng = np.random.default_rng(seed)
    if dist == "random":
        keys = rng.integers(0, 2**32, size=n, dtype=np.int64)
    elif dist == "dups":
        keys = rng.integers(0, 3, size=n, dtype=np.int64)
    elif dist == "ascending":  # every run above the previous one
        keys = np.arange(n, dtype=np.int64)
    else:  # "descending": every run below the previous one
        keys = (n - np.arange(n, dtype=np.int64)) // L * L + (np.arange(n) % L)
    arr = np.zeros(ceil_div(n, 4096) * 4096 + 4096, dtype=np.int64)
    for s in range(0, n, L):
        arr[s:min(s + L, n)] = np.sort(keys[s:min(s + L, n)])
    # the samples the previous pass wrote are these views of its output (the
    # padding past n never reaches a search: brackets stay inside the runs)
    return arr


@pytest.mark.parametrize("n,L", [(4 * 8192, 8192), (4 * 8192 * 2 + 3 * 8192 + 100, 8192), (8192 + 5, 8192),
                                 (2 * 16384 + 4096, 16384), (4 * 4096 * 3 + 4096 * 2 + 1, 4096),
                                 (4 * 4096 + 2 * 4096 + 1000, 4096)])
@pytest.mark.parametrize("dist", ["random", "dups", "ascending", "descending"])
def test_merge4_pass_plan(n, L, dist):
    arr = _runs_input(n, L, dist, seed=n + L)
    out, smp = merge4_pass_model(arr, n, L)
    if dist == "random" and n >= 4 * L:
        assert smp["packed"] > 0  # the packed path is exercised
    want = np.concatenate([np.sort(arr[s:min(s + 4 * L, n)], kind="stable") for s in range(0, n, 4 * L)])
    assert np.array_equal(out[:n], want)
    # every sample word the next pass reads was written, with the right key
    # (last-of-block samples exist for full blocks: a search reads no other)
    res = out[:n]
    assert np.array_equal(smp["f"], res[::64])
    assert np.array_equal(smp["cf"], res[::4096])
    assert np.array_equal(smp["l"][: n // 64], res[63::64])
    assert np.array_equal(smp["cl"][: n // 4096], res[4095::4096])
    del smp["packed"]


@pytest.mark.parametrize("L", [65536, 1 << 19])
def test_merge4_items_balanced_on_random_keys(L):
    """Random runs: nearly every segment is one packed item of about
    2 AB_STEP outputs, however far the merge path strays from the diagonal
    (the CD side of a segment stays near AB_STEP keys)."""
    n = 4 * L
    arr = _runs_input(n, L, "random", seed=5)
    P, Q = cuts4_model(arr, n, L, 0)
    items = items4_model(P, Q)
    sizes = [sum(c1) - sum(c0) for c0, c1 in items]
    assert sum(sizes) == n
    assert len(items) <= 1.02 * len(P)
    assert np.median(sizes) > 3700
    packed = sum(1 for c0, c1 in items if sum(1 for r in range(4) if c1[r] > c0[r]) >= 3)
    assert packed >= 0.98 * len(items)


def test_merge4_long_segments_split_at_cd_cuts():
    """Runs that do not interleave (every C and D key below every A and B key,
    and the reverse): the segments with a long CD side are cut at every CD cut
    inside them, so no item exceeds CD_STEP keys of CD, and the items still
    tile the path exactly once."""
    L = 32768
    n = 4 * L
    for dist in ("ascending", "descending"):
        arr = _runs_input(n, L, dist, seed=3)
        P, Q = cuts4_model(arr, n, L, 0)
        items = items4_model(P, Q)
        assert len(items) >= ceil_div(2 * L, AB_STEP) + ceil_div(2 * L, CD_STEP) - 2
        assert all(c1[2] + c1[3] - c0[2] - c0[3] <= CD_STEP for c0, c1 in items)


# ---------------------------------------------- long ShearSort over NW waves
#
# Model of the h-wave ShearSort block sort (paper Sec. 3.1, sorting w^2 h keys
# with h waves): regs[v, l, r] is register r of lane l of wave v.  The grid
# has 64 rows and 64 NW columns; a lane's BLOCKED registers are its row's
# segment in that wave, its STRIDED registers (after the in-wave transpose) a
# column.  Rows are sorted by a register sort per segment and a bitonic
# network of merge-splits across the waves; the sorted grid, in row-major
# order, is moved into BLOCKED sub-tiles by a line permutation.


def _model_rows(regs, snake):
    nw = regs.shape[0]
    odd = (np.arange(64) & 1).astype(bool)
    if snake:
        regs[:, odd, :] = ~regs[:, odd, :]
    regs.sort(axis=2)
    k = 1
    while k < nw:
        j = k
        while j >= 1:
            new = regs.copy()
            for v in range(nw):
                q = v ^ j
                asc = (v & (2 * k)) == 0
                keep_low = (v < q) == asc
                b = regs[q, :, ::-1]
                m = np.minimum(regs[v], b) if keep_low else np.maximum(regs[v], b)
                new[v] = np.sort(m, axis=1)  # the in-lane bitonic merge
            regs[:] = new
            j //= 2
        k *= 2
    if snake:
        regs[:, odd, :] = ~regs[:, odd, :]


def long_shear_model(keys, nw):
    assert keys.size == nw * 4096
    # loaded STRIDED: wave v, lane l, register r holds position 4096 v + 64 r + l
    regs = keys.reshape(nw, 64, 64).transpose(0, 2, 1).copy()
    for _ in range(6):
        _model_rows(regs, True)
        regs = regs.transpose(0, 2, 1).copy()  # to_strided: lanes hold columns
        regs.sort(axis=2)
        regs = regs.transpose(0, 2, 1).copy()  # to_blocked
    _model_rows(regs, False)
    # grid position l * 64 NW + 64 v + r -> BLOCKED sub-tiles
    out = np.empty_like(regs)
    for vd in range(nw):
        for ld in range(64):
            line = 64 * vd + ld
            out[vd, ld] = regs[line % nw, line // nw]
    return out.reshape(-1)  # position 4096 v' + 64 l' + r


@pytest.mark.parametrize("nw", [2, 8])
def test_long_shear_model_sorts(nw):
    rng = np.random.default_rng(nw)
    n = nw * 4096
    cases = [rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32),
             rng.integers(0, 16, size=n).astype(np.uint32),
             np.arange(n, dtype=np.uint32)[::-1].copy()]
    padded = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    padded[n - 5000:] = 0xFFFFFFFF  # padding of a partial group
    cases.append(padded)
    for _ in range(6):  # 0-1 inputs with a random number of ones
        cases.append((rng.random(n) < rng.random()).astype(np.uint32))
    for keys in cases:
        assert np.array_equal(long_shear_model(keys, nw), np.sort(keys))


def test_long_shear_line_permutation_reads_are_conflict_free():
    """The line permutation reads word 4100 sv + 64 r + sl (sv = line mod 8,
    sl = line div 8, line = 64 v' + l'): every 32-lane half touches 32 banks."""
    for vd in range(8):
        for half in (0, 32):
            banks = set()
            for ld in range(half, half + 32):
                line = 64 * vd + ld
                banks.add((4100 * (line % 8) + 64 * 5 + line // 8) % 32)
            assert len(banks) == 32
