"""Host-side planning logic of the Python binding (no GPU)."""

import numpy as np
import pytest


@pytest.mark.parametrize("pb", [False, True])
@pytest.mark.parametrize("s,P", [(3, 4), (1, 2), (5, 1), (7, 3)])
def test_bucket_groups_for_the_merge_after_a_distribution(s, P, pb):
    """Group b = the s pieces of bucket b; a pivot bucket is a single run."""
    from paper_1306_5076_amd.api import bucket_groups

    nb = 2 * P - 1 if pb else P
    rng = np.random.default_rng(s * 10 + P)
    po = np.concatenate([[0], np.cumsum(rng.integers(0, 5, nb * s))]).astype(np.uint64)
    offs, starts = bucket_groups(po, s, P, pb)
    assert offs[0] == 0 and offs[-1] == po[-1] and np.all(np.diff(offs.astype(np.int64)) >= 0)
    assert starts[0] == 0 and starts[-1] == offs.size - 1 and starts.size == nb + 1
    for b in range(nb):
        runs = offs[starts[b]:starts[b + 1] + 1]
        if pb and b % 2 == 1:
            assert runs.tolist() == [po[b * s], po[(b + 1) * s]]
        else:
            assert runs.tolist() == po[b * s:(b + 1) * s + 1].tolist()
