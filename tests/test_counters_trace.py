"""The kernel-trace summariser (CPU only): a synthetic rocprofv3 trace with
other kernels between the library's calls, grouped into calls."""

import csv
import os

from paper_1306_5076_amd import counters


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def test_per_call_groups_library_launches(tmp_path):
    # three calls of plan, block sort, two merges; a generator kernel before
    # each call; the last call cut short (one merge missing)
    t, rows = 0, []

    def launch(name, us):
        nonlocal t
        rows.append([name, t, t + us * 1000])
        t += us * 1000 + 10

    for c in range(3):
        launch("void at::native::fill_kernel<int>(int)", 50)
        launch("bcf::k_plan_zero(bcf::PlanArgs)", 2)
        launch("void bcf::k_block_sort_group<8>(bcf::Src)", 100 + c)
        launch("void bcf::k_merge4<true>(bcf::Merge4Src)", 30)
        if c < 2:
            launch("void bcf::k_merge4<true>(bcf::Merge4Src)", 40)
    _write(tmp_path / "x_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    _write(tmp_path / "x_kernel_stats.csv", ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"],
           [["bcf::k_merge4(bcf::Merge4Src)", 5, 34000, 30000, 40000, 50.0]])
    text = counters.trace_markdown(str(tmp_path), "cmd", "T", per_call=True)
    assert "median over 2 calls of 4 launches" in text
    assert "| `bcf::k_merge4<true>` | 2 | 70.0 |" in text
    assert "| `bcf::k_block_sort_group<8>` | 1 | 100.5 |" in text
    assert "| all library kernels | 4 | 172.5 | 100 % |" in text
    assert "fill_kernel" not in text.split("## One call")[1]
