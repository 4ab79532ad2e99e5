"""C ABI checks that need no GPU: exported symbols, temp-size queries, pass
planning and argument validation (all return before any HIP call)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1306_5076_amd import _native

    return _native.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcf_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    from paper_1306_5076_amd._native import EXPORTED

    assert sorted(EXPORTED) == names


def q_sort(lib, n, pairs=False):
    need = ctypes.c_uint64(123)
    if pairs:
        st = lib.bcf_sort_pairs_u32(None, None, None, None, n, None, ctypes.byref(need), None)
    else:
        st = lib.bcf_sort_u32(None, None, n, None, ctypes.byref(need), None)
    return st, need.value


def test_tile_run_and_pass_count(lib):
    assert lib.bcf_tile_keys() == 4096
    assert lib.bcf_run_keys(0) == 32768 and lib.bcf_run_keys(1) == 16384
    small = 1 << 19  # default tuning: wave tiles (runs of 4096) up to 2^19 keys
    for pairs in (0, 1):
        R = lib.bcf_run_keys(pairs)
        assert lib.bcf_sort_passes(0, pairs) == 0
        assert lib.bcf_sort_passes(1, pairs) == 1
        assert lib.bcf_sort_passes(4096, pairs) == 1
        assert lib.bcf_sort_passes(4097, pairs) == 2
        # Lemma 2: 1 + O(log(n / M)) passes over the data, M the block-sort run:
        # binary passes (default) below 2^24 keys; from 2^24 keys, and for pairs
        # at every size, four-way passes while more than two runs remain, then
        # at most one binary pass
        for n in [2**12 + 1, 2**16, small, small + 1, 2**20, 2**24 - 1, 2**24, 2**25, 2**26, 2**28,
                  3 * R + 5 + small, 2**32 - 1]:
            m = 4096 if n <= small else R
            runs = -(-n // m)
            if not pairs and n < 2**24:
                want = int(np.ceil(np.log2(runs)))
            else:
                want = 0
                while runs > 1:
                    runs = -(-runs // (4 if runs > 2 else 2))
                    want += 1
            assert lib.bcf_sort_passes(n, pairs) == 1 + want, (n, pairs)
    assert lib.bcf_sort_passes(2**26, 0) == 1 + 6  # 2^11 runs: five four-way passes and one binary
    assert lib.bcf_sort_passes(2**28, 1) == 1 + 7  # 2^14 runs of pairs: seven four-way passes
    assert lib.bcf_sort_passes(3 * 4096, 0) == 3  # three runs, default below 2^24 keys: two binary passes
    assert lib.bcf_sort_passes(3 * 4096, 1) == 2  # three runs of pairs: one four-way pass


def test_pass_count_binary_fan_in(lib):
    from paper_1306_5076_amd._native import Tuning

    t = Tuning()
    lib.bcf_get_tuning(ctypes.byref(t))
    old = Tuning.from_buffer_copy(t)
    try:
        t.merge_fan_in = 2
        assert lib.bcf_set_tuning(ctypes.byref(t)) == 0
        for n in [2**12 + 1, 2**20, 2**26, 2**32 - 1]:
            m = 4096 if n <= 1 << 19 else 32768
            assert lib.bcf_sort_passes(n, 0) == 1 + int(np.ceil(np.log2(-(-n // m))))
        # the temp size does not depend on the fan-in
        need2 = q_sort(lib, 2**26)[1]
        t.merge_fan_in = 4  # four-way passes at every size
        assert lib.bcf_set_tuning(ctypes.byref(t)) == 0
        assert q_sort(lib, 2**26)[1] == need2
        assert lib.bcf_sort_passes(3 * 4096, 0) == 2  # three runs: one four-way pass
        assert lib.bcf_sort_passes(2**16, 0) == 1 + 2  # 16 runs of 4096: two four-way passes
        t.merge_fan_in = 3
        assert lib.bcf_set_tuning(ctypes.byref(t)) == 1
    finally:
        assert lib.bcf_set_tuning(ctypes.byref(old)) == 0


def merge4_cut_bytes_max(n):
    """Cut lists of the four-way passes: per group of four runs of L keys, the
    AB cuts (one every 1920 keys of A and B, and both ends) and the CD cuts
    (one every 2048 keys of C and D strictly inside, one unused slot), 16
    bytes each; the largest over the block-sort run lengths (wave tiles, key
    group tiles, pair group tiles)."""
    most = 0
    for run0 in (4096, 32768, 16384):
        run = run0
        while n > 2 * run:
            ab_segments = -(-2 * run // 1920)
            cd_cuts = (2 * run - 1) // 2048
            most = max(most, -(-n // (4 * run)) * (ab_segments + 1 + cd_cuts + 1) * 16)
            run *= 4
    return most


def test_temp_queries(lib):
    assert q_sort(lib, 0) == (0, 0)
    assert q_sort(lib, 4096) == (0, 0)  # one sorted run: no merge pass, no temp
    assert q_sort(lib, 4096, pairs=True) == (0, 0)
    st, need = q_sort(lib, 4097)
    assert st == 0 and need >= 4097 * 4 and need % 256 == 0
    st, need = q_sort(lib, 2**26, pairs=True)
    # two ping-pong arrays (keys, values), one u32 split per merge tile, two
    # sets of key samples (every 64-block: first and last; every tile: first
    # and last), and the four-way cut lists
    tiles, blocks = 2**26 // 4096, 2**26 // 64
    cuts = -(-merge4_cut_bytes_max(2**26) // 256) * 256
    assert st == 0 and need == 2 * 2**26 * 4 + tiles * 4 + 2 * (2 * blocks * 4 + 2 * tiles * 4) + cuts
    # keys: one ping-pong array, the splits, the samples, and the cut lists
    st, need = q_sort(lib, 2**26)
    assert st == 0 and need == 2**26 * 4 + tiles * 4 + 2 * (2 * blocks * 4 + 2 * tiles * 4) + cuts
    assert cuts < 2**26 * 4 // 64
    assert q_sort(lib, 2**32)[0] == 1  # above 2^32 - 1 keys: invalid


def test_typed_sort_queries_and_errors(lib):
    """int32 / float keys: the temp size is the u32 sort's; errors are returned
    before any launch (no device needed)."""
    for n in (0, 4096, 4097, 2**20 + 3, 2**26):
        need_u = ctypes.c_uint64(0)
        assert lib.bcf_sort_u32(None, None, n, None, ctypes.byref(need_u), None) == 0
        for f in (lib.bcf_sort_i32, lib.bcf_sort_f32):
            need = ctypes.c_uint64(7)
            assert f(None, None, n, None, ctypes.byref(need), None) == 0
            assert need.value == need_u.value
        need_p = ctypes.c_uint64(0)
        assert lib.bcf_sort_pairs_u32(None, None, None, None, n, None, ctypes.byref(need_p), None) == 0
        for f in (lib.bcf_sort_pairs_i32, lib.bcf_sort_pairs_f32):
            need = ctypes.c_uint64(7)
            assert f(None, None, None, None, n, None, ctypes.byref(need), None) == 0
            assert need.value == need_p.value
    fake = ctypes.c_void_p(4096)
    small = ctypes.c_uint64(16)
    assert lib.bcf_sort_f32(fake, fake, 10**6, fake, ctypes.byref(small), None) == 2  # temp too small
    assert lib.bcf_sort_i32(fake, fake, 10, fake, None, None) == 1  # NULL temp_bytes
    big = ctypes.c_uint64(1 << 40)
    assert lib.bcf_sort_i32(None, fake, 10**6, fake, ctypes.byref(big), None) == 1  # NULL keys
    assert lib.bcf_sort_pairs_f32(fake, None, fake, fake, 10**6, fake, ctypes.byref(big), None) == 1  # NULL vals
    assert lib.bcf_sort_f32(fake, fake, 2**32, fake, ctypes.byref(big), None) == 1  # too many keys


def test_colored_prefix_sums_queries_and_errors(lib):
    """Temp = two 256-aligned arrays of tiles x d words, tiles <= 2048 of whole
    8192-element pages; errors come back before any launch."""
    f = lib.bcf_colored_prefix_sums
    for n, d in ((1, 1), (8192, 5), (8193, 32), (2**22 + 5, 16), (2**29, 32), (2**32 - 1, 3)):
        need = ctypes.c_uint64(7)
        assert f(None, None, None, n, d, 1, None, ctypes.byref(need), None) == 0
        pages = -(-n // 8192)
        tile = -(-pages // 2048) * 8192
        tiles = -(-n // tile)
        assert tiles <= 2048 and (tiles - 1) * tile < n <= tiles * tile
        assert need.value == 2 * (-(-(tiles * d * 4) // 256) * 256), (n, d)
    need = ctypes.c_uint64(7)
    assert f(None, None, None, 0, 4, 0, None, ctypes.byref(need), None) == 0 and need.value == 0
    for d in (0, 33, 256):
        assert f(None, None, None, 100, d, 1, None, ctypes.byref(need), None) == 1
    assert f(None, None, None, 2**32, 4, 1, None, ctypes.byref(need), None) == 1
    fake, odd = ctypes.c_void_p(4096), ctypes.c_void_p(4100)
    big = ctypes.c_uint64(1 << 30)
    assert f(fake, fake, fake, 100, 4, 1, fake, None, None) == 1  # NULL temp_bytes
    assert f(None, fake, fake, 100, 4, 1, fake, ctypes.byref(big), None) == 1  # NULL values
    assert f(fake, odd, fake, 100, 4, 1, fake, ctypes.byref(big), None) == 1  # colors not 16-byte aligned
    small = ctypes.c_uint64(16)
    assert f(fake, fake, fake, 10**6, 4, 1, fake, ctypes.byref(small), None) == 2  # temp too small


def test_u64_sort_queries_and_errors(lib):
    """Temp = one 256-aligned u64 ping-pong array once there is a merge pass
    (more than one 4096-key tile); errors before any launch."""
    f = lib.bcf_sort_u64
    for n in (0, 1, 4096, 4097, 2**20 + 3, 2**26, 2**32 - 1):
        need = ctypes.c_uint64(7)
        assert f(None, None, n, None, ctypes.byref(need), None) == 0
        assert need.value == (0 if n <= 4096 else -(-8 * n // 256) * 256), n
    need = ctypes.c_uint64(0)
    assert f(None, None, 2**32, None, ctypes.byref(need), None) == 1  # too many keys
    fake = ctypes.c_void_p(4096)
    assert f(fake, fake, 10, fake, None, None) == 1  # NULL temp_bytes
    big = ctypes.c_uint64(1 << 40)
    assert f(None, fake, 10**6, fake, ctypes.byref(big), None) == 1  # NULL keys_in
    small = ctypes.c_uint64(16)
    assert f(fake, fake, 10**6, fake, ctypes.byref(small), None) == 2  # temp too small


def test_argument_errors(lib):
    need = ctypes.c_uint64(16)
    fake = ctypes.c_void_p(4096)
    # temp too small (returns before any launch)
    assert lib.bcf_sort_u32(fake, fake, 10**6, fake, ctypes.byref(need), None) == 2
    # NULL temp_bytes
    assert lib.bcf_sort_u32(fake, fake, 10, fake, None, None) == 1
    # NULL keys with a real temp buffer
    big = ctypes.c_uint64(1 << 40)
    assert lib.bcf_sort_u32(None, fake, 10**6, fake, ctypes.byref(big), None) == 1
    for s in range(6):
        assert lib.bcf_status_string(s).startswith(b"BCF_")


def _offs(a):
    a = np.asarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def test_merge_runs_validation_and_query(lib):
    need = ctypes.c_uint64(0)
    a, p = _offs([0, 5, 3, 9])  # decreasing offset
    assert lib.bcf_merge_runs_host(None, None, p, 3, None, None, None, ctypes.byref(need), None) == 1
    a, p = _offs([1, 5])  # off[0] != 0
    assert lib.bcf_merge_runs_host(None, None, p, 1, None, None, None, ctypes.byref(need), None) == 1
    a, p = _offs([0, 5000, 5000, 9000])
    assert lib.bcf_merge_runs_host(None, None, p, 3, None, None, None, ctypes.byref(need), None) == 0
    assert need.value >= 9000 * 4
    # k == 0 is a no-op
    assert lib.bcf_merge_runs_host(None, None, None, 0, None, None, None, ctypes.byref(need), None) == 0


def test_device_offset_calls_refuse_before_any_device_access(lib):
    """The calls with device offsets: k == 0 / nseg == 0 are no-ops with a zero
    temp size, and a NULL offset array or NULL temp_bytes is refused, all
    without touching the device."""
    need = ctypes.c_uint64(7)
    assert lib.bcf_merge_runs(None, None, None, 0, None, None, None, ctypes.byref(need), None) == 0
    assert need.value == 0
    assert lib.bcf_merge_runs(None, None, None, 3, None, None, None, ctypes.byref(need), None) == 1
    assert lib.bcf_merge_runs(None, None, ctypes.c_void_p(0x1000), 3, None, None, None, None, None) == 1
    for f in (lib.bcf_segmented_sort,):
        need = ctypes.c_uint64(7)
        assert f(None, None, None, 0, None, ctypes.byref(need), None) == 0 and need.value == 0
        assert f(None, None, None, 4, None, ctypes.byref(need), None) == 1
        assert f(None, None, ctypes.c_void_p(0x1000), 4, None, None, None) == 1
    need = ctypes.c_uint64(7)
    assert lib.bcf_segmented_sort_pairs(None, None, None, None, None, 0, None, ctypes.byref(need), None) == 0
    assert need.value == 0
    assert lib.bcf_segmented_sort_pairs(None, None, None, None, None, 2, None, ctypes.byref(need), None) == 1


def test_sort_pb_query_and_validation(lib):
    """bcf_sort_u32_pb: the temp query is host-only (the run offsets are
    uniform); sizes and the distribution's limits are checked first."""
    need = ctypes.c_uint64(0)
    q = lambda n, P, rk, pb: lib.bcf_sort_u32_pb(None, None, n, P, rk, pb, None, ctypes.byref(need), None)  # noqa
    assert q(0, 256, 1 << 18, 1) == 0 and need.value == 0
    assert q(1 << 26, 256, 1 << 18, 1) == 0
    n = 1 << 26
    assert need.value >= 2 * n * 4  # the distributed keys and the bucket merge's ping-pong buffer
    with_pivots = need.value
    assert q(1 << 26, 256, 1 << 18, 0) == 0 and need.value < with_pivots  # P instead of 2P - 1 buckets' pieces
    assert q(1 << 26, 0, 1 << 18, 0) == 1 and q(1 << 26, 65537, 1 << 18, 0) == 1  # P in 1..65536
    assert q(1 << 26, 256, 0, 0) == 1  # run_keys >= 1
    assert q(1 << 26, 65536, 1 << 12, 1) == 1  # 16384 runs x 65536 candidates > 2^26
    assert q(1 << 32, 256, 1 << 18, 1) == 1  # more than 2^32 - 1 keys
    buf = ctypes.c_void_p(0x100000)
    tb = ctypes.c_uint64(1 << 40)
    assert lib.bcf_sort_u32_pb(buf, buf, 1 << 20, 16, 1 << 16, 1, ctypes.c_void_p(0x200000), ctypes.byref(tb),
                               None) == 1  # in place is refused


def test_segmented_validation_and_query(lib):
    need = ctypes.c_uint64(0)
    a, p = _offs([0, 10, 5])
    assert lib.bcf_segmented_sort_host(None, None, p, 2, None, ctypes.byref(need), None) == 1
    a, p = _offs([0, 0, 1, 4096, 4096 + 8193])
    assert lib.bcf_segmented_sort_host(None, None, p, 4, None, ctypes.byref(need), None) == 0
    assert need.value > 0


def test_segmented_execute_needs_its_upload(lib):
    """bcf_segmented_execute into a temp buffer that no upload planned (for
    these offsets) is refused before any launch."""
    a, p = _offs([0, 100, 5000, 40000])
    need = ctypes.c_uint64(0)
    assert lib.bcf_segmented_upload(p, 3, 0, None, ctypes.byref(need), None) == 0
    fake_temp = ctypes.c_void_p(0x10000)  # never dereferenced: refused first
    tb = ctypes.c_uint64(need.value)
    dummy = ctypes.c_void_p(0x20000)
    assert lib.bcf_segmented_execute(dummy, None, dummy, None, p, 3, fake_temp, ctypes.byref(tb), None) == 1


def test_tuning_roundtrip():
    import paper_1306_5076_amd as bcf

    before = bcf.get_tuning()
    assert set(before) == {"merge_variant", "nontemporal", "sampled_partition", "tile_samples",
                           "group_min_keys", "check_runs", "block_sort", "fused_partition", "merge_fan_in"}
    assert before["block_sort"] == 0 and before["merge_variant"] == 3 and before["fused_partition"] == 1
    assert before["merge_fan_in"] == 0
    with bcf.tuning(fused_partition=0):
        assert bcf.get_tuning()["fused_partition"] == 0
    with bcf.tuning(merge_variant=2, group_min_keys=12345, check_runs=1, block_sort=2, merge_fan_in=2):
        t = bcf.get_tuning()
        assert t["merge_variant"] == 2 and t["group_min_keys"] == 12345 and t["check_runs"] == 1
        assert t["block_sort"] == 2 and t["merge_fan_in"] == 2
        # wave tiles hand runs of 4096 keys to the merge passes
        assert bcf.run_keys() == 4096 and bcf.run_keys(pairs=True) == 4096
        assert bcf.sort_passes(1 << 26) == 1 + 14
    with bcf.tuning(block_sort=2):  # 2^14 runs: seven four-way passes
        assert bcf.sort_passes(1 << 26) == 1 + 7 and bcf.sort_passes(1 << 26, pairs=True) == 1 + 7
    assert bcf.get_tuning() == before
    assert bcf.run_keys() == 32768 and bcf.sort_passes(1 << 26) == 1 + 6
    with bcf.tuning(merge_fan_in=2):
        assert bcf.sort_passes(1 << 26) == 1 + 11
    # default block sort: wave tiles up to 2^19 keys, group tiles above; binary
    # passes below 2^24 keys
    assert bcf.sort_passes(1 << 19) == 1 + 7 and bcf.sort_passes((1 << 19) + 1) == 1 + 5
    with bcf.tuning(merge_fan_in=4):  # 128 runs -> 32 -> 8 -> 2 -> 1; 17 runs -> 5 -> 2 -> 1
        assert bcf.sort_passes(1 << 19) == 1 + 4 and bcf.sort_passes((1 << 19) + 1) == 1 + 3
    for v in (3, 4):  # group tiles (merge rounds or the long ShearSort): runs of 32768 keys
        with bcf.tuning(block_sort=v):
            assert bcf.sort_passes(1 << 16) == 1 + 1 and bcf.sort_passes(1 << 15) == 1
            assert bcf.run_keys() == 32768 and bcf.run_keys(pairs=True) == 16384
    from paper_1306_5076_amd import BcfError

    for bad in ({"merge_variant": 7}, {"block_sort": 5}, {"block_sort": -1}, {"merge_fan_in": 3}):
        with pytest.raises(BcfError):
            bcf.set_tuning(**bad)
    assert bcf.get_tuning() == before


def test_distribute_runs_validation_and_query(lib):
    need = ctypes.c_uint64(0)
    q = lambda p, s, P, t, pb=0: lib.bcf_distribute_runs(None, p, s, P, t, pb, None, None, None, None,  # noqa: E731
                                                           ctypes.byref(need), None)
    a, p = _offs([0, 5, 3])  # decreasing offset
    assert q(p, 2, 4, 4) == 1
    a, p = _offs([1, 5])  # off[0] != 0
    assert q(p, 1, 4, 4) == 1
    a, p = _offs([0, 100, 300])
    assert q(p, 2, 0, 4) == 1 and q(p, 2, 4, 0) == 1  # P, t >= 1
    assert q(p, 2, (1 << 16) + 1, 4) == 1 and q(p, 2, 4, (1 << 16) + 1) == 1
    assert q(p, 2, 1 << 16, 1 << 16) == 0  # 2 runs x 65536 candidates
    assert q(p, 2, 16, 16) == 0 and need.value >= 2 * 16 * 2 * 8
    small = need.value
    assert q(p, 2, 16, 16, 1) == 0 and need.value > small  # 31 buckets' pieces
    a, p = _offs(list(range(0, 1025)))  # 1024 one-key runs
    assert q(p, 1024, 1 << 16, 1 << 10) == 1  # 1024 * 65536 pieces > 2^24
    # s == 0 is a no-op
    assert lib.bcf_distribute_runs(None, None, 0, 4, 4, 0, None, None, None, None, ctypes.byref(need), None) == 0
    assert need.value == 0
    # in place is refused before any launch
    a, p = _offs([0, 64])
    buf = ctypes.c_void_p(0x100000)
    tb = ctypes.c_uint64(1 << 30)
    assert lib.bcf_distribute_runs(buf, p, 1, 4, 4, 0, buf, ctypes.c_void_p(0x200000), None, ctypes.c_void_p(0x300000),
                                   ctypes.byref(tb), None) == 1


def test_merge_run_groups_validation_and_query(lib):
    need = ctypes.c_uint64(0)
    a, p = _offs([0, 10, 20, 30])
    g = (ctypes.c_uint32 * 3)(0, 2, 3)
    assert lib.bcf_merge_run_groups(None, None, p, 3, g, 2, None, None, None, ctypes.byref(need), None) == 0
    assert need.value >= 30 * 4
    bad = (ctypes.c_uint32 * 3)(0, 2, 2)  # last start != k
    assert lib.bcf_merge_run_groups(None, None, p, 3, bad, 2, None, None, None, ctypes.byref(need), None) == 1
    dec = (ctypes.c_uint32 * 3)(0, 3, 2)  # decreasing
    assert lib.bcf_merge_run_groups(None, None, p, 3, dec, 2, None, None, None, ctypes.byref(need), None) == 1
    assert lib.bcf_merge_run_groups(None, None, p, 3, None, 2, None, None, None, ctypes.byref(need), None) == 1


def test_noalloc_sort_limits_without_gpu(lib):
    """bcf_sort_u32_noalloc refuses sizes past BCF_NOALLOC_MAX_KEYS and NULL
    pointers before touching the device; n == 0 is a no-op."""
    text = open(HEADER).read()
    m = re.search(r"#define\s+BCF_NOALLOC_MAX_KEYS\s+\(1ull\s*<<\s*(\d+)\)", text)
    assert m is not None
    max_keys = 1 << int(m.group(1))
    assert lib.bcf_sort_u32_noalloc(None, None, 0, None) == 0
    assert lib.bcf_sort_u32_noalloc(None, None, max_keys + 1, None) == 1
    assert lib.bcf_sort_u32_noalloc(None, None, 2**40, None) == 1
    assert lib.bcf_sort_u32_noalloc(None, None, 5, None) == 1
    # the library array holds bcf_sort_u32's temp for the largest size it serves
    st, need = q_sort(lib, max_keys)
    assert st == 0 and need <= 18 << 20
