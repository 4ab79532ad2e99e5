"""The allocation-free key sort (bcf_sort_u32_noalloc) against bcf_sort_u32,
through the C ABI: the same result on the same inputs, on two calls in a row
(the second smaller, so that it runs on what the first left in the library's
device array), and sizes past the array's limit refused before any launch."""

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MAX_KEYS = 1 << 22  # BCF_NOALLOC_MAX_KEYS


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1306_5076_amd import _native

    return torch, torch.device("cuda:0"), _native.load()


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _sort_with_temp(torch, dev, lib, kin):
    """bcf_sort_u32 with a caller-provided temp buffer (the allocating entry point)."""
    n = kin.numel()
    need = ctypes.c_uint64(0)
    assert lib.bcf_sort_u32(None, None, n, None, ctypes.byref(need), None) == 0
    temp = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    out = torch.empty_like(kin)
    have = ctypes.c_uint64(temp.numel())
    st = lib.bcf_sort_u32(ctypes.c_void_p(kin.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                          ctypes.c_void_p(temp.data_ptr()), ctypes.byref(have), _stream(torch))
    assert st == 0, st
    torch.cuda.synchronize()
    return out


def _sort_noalloc(torch, lib, kin, out):
    st = lib.bcf_sort_u32_noalloc(ctypes.c_void_p(kin.data_ptr()), ctypes.c_void_p(out.data_ptr()), kin.numel(),
                                  _stream(torch))
    assert st == 0, st
    torch.cuda.synchronize()


@pytest.mark.parametrize("sizes,dist", [((MAX_KEYS, 3 * 4096 + 123), "uniform"),
                                        ((1_000_003, 4097), "zipf"),
                                        ((65_536 + 17, 1), "distinct16")])
def test_noalloc_matches_sort_u32_twice(env, sizes, dist):
    torch, dev, lib = env
    for call, n in enumerate(sizes):
        print(f"noalloc call {call}: n={n} dist={dist}", flush=True)
        keys = workloads.keys_u32(dist, n, seed=11 + call)
        kin = torch.from_numpy(keys).to(dev)
        want = _sort_with_temp(torch, dev, lib, kin)
        got = torch.empty_like(kin)
        _sort_noalloc(torch, lib, kin, got)
        assert torch.equal(got, want), (call, n)
        assert torch.equal(kin.cpu(), torch.from_numpy(keys))  # input untouched


def test_noalloc_in_place_and_limits(env):
    torch, dev, lib = env
    keys = workloads.keys_u32("uniform", 100_000, seed=5)
    kin = torch.from_numpy(keys).to(dev)
    want = _sort_with_temp(torch, dev, lib, kin)
    _sort_noalloc(torch, lib, kin, kin)
    assert torch.equal(kin, want)
    # past the limit: refused, output untouched
    big = torch.zeros(MAX_KEYS + 1, dtype=torch.uint32, device=dev)
    out = torch.full_like(big, 7)
    st = lib.bcf_sort_u32_noalloc(ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(out.data_ptr()), MAX_KEYS + 1,
                                  _stream(torch))
    assert st == 1  # BCF_ERR_INVALID
    torch.cuda.synchronize()
    assert bool((out == 7).all())
    assert lib.bcf_sort_u32_noalloc(None, None, 0, None) == 0
