"""GPU parity of the segmented sort at its full configured size: 10,000
arrays with sizes log-uniform in [32, 2^20] (about 10^9 keys in total), uniform
keys, seed 1.  Keys and stable key/value pairs, run eagerly and as a captured
graph replayed on new data, each compared with the oracle segment by segment
(the oracle's plain merge sort of every segment, spread over the host cores).
"""

import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

NSEG = 10_000
LO, HI = 32, 1 << 20
THREADS = max(1, min(16, os.cpu_count() or 1))


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


@pytest.fixture(scope="module")
def segments():
    sizes = workloads.segment_sizes(NSEG, lo=LO, hi=HI, seed=1)
    offs = workloads.segment_offsets(sizes)
    return sizes, offs


def _first_bad_segment(got, want, offs):
    if np.array_equal(got, want):
        return None
    bad = int(np.flatnonzero(got != want)[0])
    sg = int(np.searchsorted(offs, bad, side="right")) - 1
    return sg, bad, int(got[bad]), int(want[bad])


def _keys_on_device(torch, dev, n, seed):
    k = workloads.keys_u32_torch("uniform", n, dev, seed=seed)
    return k, k.cpu().numpy()


def test_segmented_keys_full_size_eager_and_graph(torch_dev, bcf, segments):
    torch, dev = torch_dev
    sizes, offs = segments
    n = int(offs[-1])
    print(f"segmented keys: {NSEG} segments, {n} keys", flush=True)
    kin, keys = _keys_on_device(torch, dev, n, seed=1)
    out = bcf.segmented_sort(kin, offs)
    torch.cuda.synchronize()
    want = oracle.segmented_sort_threads(keys, offs, THREADS)
    assert _first_bad_segment(out.cpu().numpy(), want, offs) is None

    plan = bcf.SegmentedPlan(offs, dev)
    gout = torch.empty_like(kin)
    graph = plan.capture(kin, gout)
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(gout, out)
    # new data in the same buffers, eager work in between
    kin.copy_(workloads.keys_u32_torch("uniform", n, dev, seed=2))
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    want2 = oracle.segmented_sort_threads(kin.cpu().numpy(), offs, THREADS)
    assert _first_bad_segment(gout.cpu().numpy(), want2, offs) is None


def test_segmented_pairs_full_size_eager_and_graph(torch_dev, bcf, segments):
    torch, dev = torch_dev
    sizes, offs = segments
    n = int(offs[-1])
    print(f"segmented pairs: {NSEG} segments, {n} pairs", flush=True)
    kin, keys = _keys_on_device(torch, dev, n, seed=3)
    vals = np.arange(n, dtype=np.uint32)  # value = original index
    vin = torch.from_numpy(vals).to(dev)
    ko, vo = bcf.segmented_sort(kin, offs, vals=vin)
    torch.cuda.synchronize()
    wk, wv = oracle.segmented_sort_threads(keys, offs, THREADS, vals=vals)
    assert _first_bad_segment(ko.cpu().numpy(), wk, offs) is None
    assert _first_bad_segment(vo.cpu().numpy(), wv, offs) is None

    plan = bcf.SegmentedPlan(offs, dev, pairs=True)
    gko, gvo = torch.empty_like(kin), torch.empty_like(vin)
    graph = plan.capture(kin, gko, vin, gvo)
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(gko, ko) and torch.equal(gvo, vo), rep
