"""Colored prefix sums timing sweep: the paper's bank-conflict demonstration
(Sec. 1.2 and its appendix) on gfx950.  Times both LDS counter layouts of
``colored_prefix_sums`` over the number of colors d at N elements (the paper
uses N = 2^29) with inputs resident in HBM.

    python -m paper_1306_5076_amd.cps_demo [--n N] [--colors 1,2,4,8,16,32] [--reps R]

prints one JSON object.  The algorithmic HBM traffic of one call is 14 bytes
per element: phase 1 reads values and colors (5 B), phase 3 reads them again
and writes the sums (9 B); phase 2 touches tiles x d words only.
"""

from __future__ import annotations

import argparse
import json

BYTES_PER_ELEMENT = 14


def sweep(n=1 << 29, colors=(1, 2, 4, 8, 16, 32), reps=5, device="cuda:0", seed=1):
    import torch

    import workloads
    from . import api
    from .autotune import time_ms

    dev = torch.device(device)
    out = None
    ws = api.Workspace(dev)
    res = {"n": n, "bytes_per_element": BYTES_PER_ELEMENT, "per_d": {}}
    for d in colors:
        vals, cols = workloads.colored_u32_torch(n, d, dev, seed=seed)
        out = torch.empty_like(vals) if out is None else out
        row = {}
        for cf in (True, False):
            fn = lambda: api.colored_prefix_sums(vals, cols, d, conflict_free=cf, out=out, workspace=ws)
            ms = time_ms(fn, reps=reps, warmup=1)
            row["conflict_free" if cf else "naive"] = {
                "ms": round(ms, 4), "GB_per_s": round(BYTES_PER_ELEMENT * n / ms / 1e6, 1)}
        row["naive_over_cf"] = round(row["naive"]["ms"] / row["conflict_free"]["ms"], 3)
        res["per_d"][str(d)] = row
        del vals, cols
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 29)
    ap.add_argument("--colors", default="1,2,4,8,16,32")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    print(json.dumps(sweep(a.n, tuple(int(x) for x in a.colors.split(",")), a.reps)), flush=True)


if __name__ == "__main__":
    main()
