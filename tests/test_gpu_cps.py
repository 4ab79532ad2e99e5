"""GPU parity of colored prefix sums (the paper's bank-conflict example,
Sec. 1.2 and its appendix) against the CPU oracle: bit-exact, both LDS counter
layouts, at sizes that span many 8192-element pages, several tiles and a
ragged tail; plus clamped colors, in-place calls and argument errors."""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def bcf():
    import paper_1306_5076_amd as bcf
    from paper_1306_5076_amd import _native

    _native.load()
    return bcf


def first_diff(got, want):
    idx = np.flatnonzero(got != want)
    return None if idx.size == 0 else (int(idx[0]), int(got[idx[0]]), int(want[idx[0]]))


SIZES = [1, 31, 32, 33, 8191, 8192, 8193, 100_003, (1 << 22) + 5, (1 << 24) + 8192 * 3 + 9]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("d", [1, 2, 5, 16, 32])
def test_colored_prefix_sums_vs_oracle(torch_dev, bcf, n, d):
    torch, dev = torch_dev
    v, c = workloads.colored_u32(n, d, seed=n % 1009 + d)
    want = oracle.colored_prefix_sums(v, c, d)
    tv, tc = torch.from_numpy(v).to(dev), torch.from_numpy(c).to(dev)
    for cf in (True, False):
        got = bcf.colored_prefix_sums(tv, tc, d, conflict_free=cf).cpu().numpy()
        assert first_diff(got, want) is None, (n, d, cf)


@pytest.mark.parametrize("d", [1, 3, 32])
def test_colored_prefix_sums_clamps_colors(torch_dev, bcf, d):
    torch, dev = torch_dev
    n = 300_001
    v, c = workloads.colored_u32(n, 256, seed=d)
    want = oracle.colored_prefix_sums(v, c, d)
    tv, tc = torch.from_numpy(v).to(dev), torch.from_numpy(c).to(dev)
    for cf in (True, False):
        got = bcf.colored_prefix_sums(tv, tc, d, conflict_free=cf).cpu().numpy()
        assert first_diff(got, want) is None, (d, cf)


def test_colored_prefix_sums_in_place_and_full_size(torch_dev, bcf):
    torch, dev = torch_dev
    n, d = (1 << 29) - 3, 32  # the full demonstration size, checked on a prefix and sampled tiles
    tv, tc = workloads.colored_u32_torch(n, d, dev, seed=5)
    got = bcf.colored_prefix_sums(tv, tc, d).cpu().numpy()
    head = 1 << 21
    want = oracle.colored_prefix_sums(tv[:head].cpu().numpy(), tc[:head].cpu().numpy(), d)
    assert first_diff(got[:head], want) is None
    # any window [lo, hi): its sums = the window's own colored sums plus, per
    # color, the last result of that color before lo (0 if none) -- checked on
    # the CPU from the last element of each color before the window
    vn, cn = tv.cpu().numpy(), tc.cpu().numpy()
    for lo in (n // 3 + 11, n - 100_000):
        hi = min(n, lo + 100_000)
        local = oracle.colored_prefix_sums(vn[lo:hi], cn[lo:hi], d)
        base = np.zeros(d, dtype=np.uint32)
        back = lo - (1 << 16)  # every color occurs in the 2^16 elements before lo
        for col in range(d):
            idx = np.flatnonzero(cn[back:lo] == col)
            assert idx.size
            base[col] = got[back + idx[-1]]
        assert first_diff(got[lo:hi], local + base[cn[lo:hi]]) is None, lo
    # in place (out is values), the other layout
    small = 1_000_003
    v, c = workloads.colored_u32(small, 7, seed=3)
    t = torch.from_numpy(v).to(dev)
    bcf.colored_prefix_sums(t, torch.from_numpy(c).to(dev), 7, conflict_free=False, out=t)
    assert first_diff(t.cpu().numpy(), oracle.colored_prefix_sums(v, c, 7)) is None


def test_colored_prefix_sums_errors(torch_dev, bcf):
    torch, dev = torch_dev
    from paper_1306_5076_amd import BcfError

    v = torch.zeros(4096, dtype=torch.uint32, device=dev)
    c = torch.zeros(4096, dtype=torch.uint8, device=dev)
    for d in (0, 33):
        with pytest.raises(BcfError):
            bcf.colored_prefix_sums(v, c, d)
    with pytest.raises(BcfError):  # colors not 16-byte aligned
        bcf.colored_prefix_sums(v[:4000], torch.zeros(4005, dtype=torch.uint8, device=dev)[5:], 4)
    with pytest.raises(ValueError):
        bcf.colored_prefix_sums(v, c[:100], 4)
    out = bcf.colored_prefix_sums(v[:0], c[:0], 4)
    assert out.numel() == 0
