"""GPU parity of the unsigned 64-bit key sort against the CPU oracle: bit-exact
on every u64 distribution (ties in either half, one key, extreme values) at
edge sizes (one tile, wave tiles up to 2^19 keys, group tiles of 16384 above,
partial last groups), a 2^24 and the 2^26 benchmark size, in place, and
argument errors."""

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


@pytest.mark.parametrize("dist", workloads.U64_DISTRIBUTIONS)
@pytest.mark.parametrize("n", [1, 2, 3, 4095, 4096, 4097, 16385, 100_003, 1 << 19, (1 << 19) + 1,
                               (1 << 19) + 3 * 4096 + 5, (1 << 20) + 7])
def test_sort_u64_vs_oracle(torch_dev, bcf, n, dist):
    torch, dev = torch_dev
    keys = workloads.keys_u64(dist, n, seed=n % 101)
    got = bcf.sort_u64(torch.from_numpy(keys).to(dev)).cpu().numpy()
    assert first_diff(got, oracle.sort_u64(keys)) is None, (n, dist)


@pytest.mark.parametrize("n,dist", [((1 << 24) + 5, "hi16"), ((1 << 24) + 5, "lo16"), (1 << 26, "uniform")])
def test_sort_u64_large(torch_dev, bcf, n, dist):
    torch, dev = torch_dev
    keys = workloads.keys_u64(dist, n, seed=2)
    got = bcf.sort_u64(torch.from_numpy(keys).to(dev)).cpu().numpy()
    assert first_diff(got, oracle.sort_u64(keys)) is None


def test_sort_u64_in_place_workspace_and_errors(torch_dev, bcf):
    torch, dev = torch_dev
    ws = bcf.Workspace(dev)
    for n in (300_001, 5000):  # the second call reuses the larger workspace
        keys = workloads.keys_u64("extremes", n, seed=n)
        t = torch.from_numpy(keys).to(dev)
        bcf.sort_u64(t, out=t, workspace=ws)
        assert first_diff(t.cpu().numpy(), oracle.sort_u64(keys)) is None
    with pytest.raises(TypeError):
        bcf.sort_u64(torch.zeros(10, dtype=torch.int64, device=dev))
    assert bcf.sort_u64(torch.zeros(0, dtype=torch.uint64, device=dev)).numel() == 0
