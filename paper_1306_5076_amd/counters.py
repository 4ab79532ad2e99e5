"""Summaries of rocprofv3 runs of ``bench.py`` for the ``profiles/`` folder.

Measurement tooling, not part of the sort path: it reads the CSV files that
``rocprofv3 --kernel-trace --stats`` and ``rocprofv3 --pmc ...`` wrote and
turns them into the short summaries that ``bench.py`` and the design notes
quote.

* ``trace``   -- per-kernel launch statistics and, for the merge passes of
  one sort, the median duration at every pass position;
* ``traffic`` -- HBM bytes per dispatch from a ``FETCH_SIZE`` run and a
  ``WRITE_SIZE`` run.  The counters are in KiB per dispatch and are scaled by
  what they read for a plain device-to-device copy of known size in the same
  run (``bench.py --copy-calibration``): the scale makes that copy read and
  write exactly its size;
* ``lds``     -- ``SQ_LDS_BANK_CONFLICT`` and ``SQ_INSTS_LDS`` per dispatch.

Every JSON summary records the hash of the kernel sources it was measured
with; ``bench.py`` uses a summary only while the sources still hash the same.

    python -m paper_1306_5076_amd.counters trace   DIR OUT.md  --command "..."
    python -m paper_1306_5076_amd.counters traffic FETCH_DIR WRITE_DIR OUT.json --n N --command "..."
    python -m paper_1306_5076_amd.counters lds     DIR OUT.json --command "..."
    python -m paper_1306_5076_amd.counters summary TRAFFIC.json LDS.json OUT.md --algorithmic-bytes B
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
# every source of the library (kernels and the host code that picks launch
# shapes), so that any change to them marks committed counter summaries stale
KERNEL_SOURCES = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")) + glob.glob(os.path.join(PKG, "csrc", "*.hpp")))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the library's sources (file names
    and contents, in name order)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without the return type and the argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):  # cut at the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def _one_csv(directory: str, suffix: str) -> str:
    found = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not found:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return found[0]


def _rows(directory: str, suffix: str):
    with open(_one_csv(directory, suffix)) as f:
        return list(csv.DictReader(f))


def counter_per_kernel(directory: str, counter: str) -> dict:
    """{kernel: [value of `counter` per dispatch]} from a --pmc run."""
    out: dict[str, list[float]] = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_dir: str, write_dir: str, n_copy_keys: int, command: str = "") -> dict:
    fetch = counter_per_kernel(fetch_dir, "FETCH_SIZE")
    write = counter_per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = 4.0 * n_copy_keys
    cf, cw = fetch.get(COPY_KERNEL), write.get(COPY_KERNEL)
    if not cf or not cw:
        raise ValueError(f"no {COPY_KERNEL} dispatch to calibrate with (run bench.py --copy-calibration)")
    # the calibration copies are the largest copy dispatches; small host-device
    # copies of descriptors in the same run are left out
    cf = [x for x in cf if x >= 0.5 * max(cf)]
    cw = [x for x in cw if x >= 0.5 * max(cw)]
    fetch_scale = copy_bytes / (statistics.mean(cf) * 1024.0)
    write_scale = copy_bytes / (statistics.mean(cw) * 1024.0)
    per = {}
    for k in sorted(set(fetch) & set(write)):
        if k == COPY_KERNEL or not k.startswith(("bcf::", "k_dist_")):
            continue
        fk, wk = statistics.mean(fetch[k]), statistics.mean(write[k])
        per[k] = {
            "fetch_kib_raw": round(fk, 1),
            "write_kib_raw": round(wk, 1),
            "read_bytes": int(fk * 1024 * fetch_scale),
            "write_bytes": int(wk * 1024 * write_scale),
            "dispatches": len(fetch[k]),
        }
    return {
        "kernel_source_hash": kernel_source_hash(),
        "command": command,
        "fetch_scale": round(fetch_scale, 4),
        "write_scale": round(write_scale, 4),
        "calibration": f"{COPY_KERNEL} of {n_copy_keys} u32 ({int(copy_bytes)} bytes read and written): "
        "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled so that the copy reads and writes exactly its size",
        "per_kernel": per,
    }


def lds(directory: str, command: str = "") -> dict:
    conf = counter_per_kernel(directory, "SQ_LDS_BANK_CONFLICT")
    insts = counter_per_kernel(directory, "SQ_INSTS_LDS")
    per = {}
    for k in sorted(set(conf) & set(insts)):
        if not k.startswith(("bcf::", "k_dist_")):
            continue
        per[k] = {"SQ_LDS_BANK_CONFLICT": statistics.mean(conf[k]), "SQ_INSTS_LDS": statistics.mean(insts[k]),
                  "dispatches": len(conf[k])}
    return {"kernel_source_hash": kernel_source_hash(), "command": command, "per_kernel": per}


def counters_markdown(traffic_json: str, lds_json: str, algorithmic_bytes: float) -> str:
    """One page from a traffic summary and an LDS summary (both JSON)."""
    with open(traffic_json) as f:
        t = json.load(f)
    with open(lds_json) as f:
        ld = json.load(f)
    out = [f"# Counters (kernel source hash {t['kernel_source_hash']})", "",
           "Commands (repository root on the GPU box, library built in-tree; each counter set in its own run):",
           "", "    " + ld.get("command", ""), "", "    " + t.get("command", ""), "",
           "## LDS bank conflicts (per dispatch, averaged)", "",
           "| kernel | dispatches | SQ_INSTS_LDS | SQ_LDS_BANK_CONFLICT |", "|---|---|---|---|"]
    for k, v in ld["per_kernel"].items():
        out.append(f"| `{k}` | {v['dispatches']} | {v['SQ_INSTS_LDS']:.0f} | {v['SQ_LDS_BANK_CONFLICT']:.0f} |")
    out += ["", f"## HBM traffic per dispatch (FETCH_SIZE x {t['fetch_scale']}, WRITE_SIZE x {t['write_scale']})", "",
            t["calibration"] + ".", "",
            "| kernel | dispatches | read MB | written MB | algorithmic MB (read + write) |", "|---|---|---|---|---|"]
    for k, v in t["per_kernel"].items():
        alg = f"{algorithmic_bytes / 1e6:.1f}" if k.startswith(("bcf::k_merge", "bcf::k_block_sort")) else "-"
        out.append(f"| `{k}` | {v['dispatches']} | {v['read_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | {alg} |")
    return "\n".join(out) + "\n"


def _is(kind: str, name: str) -> bool:
    n = short_name(name)
    if kind == "block":
        return n.startswith("bcf::k_block_sort")
    if kind == "merge":
        return n.startswith("bcf::k_merge")
    return False


def _per_call_lines(trace) -> list[str]:
    """Library launches grouped into calls: a call starts at each launch of
    the run's first library kernel.  Per kernel: launches per call and median
    time per call over the calls with the most common launch count."""
    lib = [r for r in trace if short_name(r["Kernel_Name"]).startswith("bcf::")]
    if not lib:
        return []
    first = lib[0]["Kernel_Name"]
    calls = []
    for r in lib:
        if r["Kernel_Name"] == first:
            calls.append([])
        calls[-1].append((short_name(r["Kernel_Name"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    size = statistics.mode(len(c) for c in calls)
    full = [c for c in calls if len(c) == size]
    names = list(dict.fromkeys(n for n, _ in full[0]))
    per = {n: [sum(t for m, t in c if m == n) for c in full] for n in names}
    count = {n: sum(1 for m, _ in full[0] if m == n) for n in names}
    total = statistics.median(sum(t for _, t in c) for c in full)
    lines = ["", f"## One call, by kernel (median over {len(full)} calls of {size} launches)", "",
             "| kernel | launches per call | median us per call | share of the call |", "|---|---|---|---|"]
    for n in sorted(names, key=lambda n: -statistics.median(per[n])):
        med = statistics.median(per[n])
        lines.append(f"| `{n}` | {count[n]} | {med / 1e3:.1f} | {100 * med / total:.1f} % |")
    lines.append(f"| all library kernels | {size} | {total / 1e3:.1f} | 100 % |")
    return lines


def trace_markdown(directory: str, command: str, title: str, n_keys: int | None = None, elem_bytes: int = 4,
                   per_call: bool = False) -> str:
    stats = _rows(directory, "kernel_stats.csv")
    lines = [f"# {title}", "", "Command (repository root on the GPU box, library built in-tree beforehand):", "",
             "    " + command.replace("\n", "\n    "), "", f"Kernel source hash: `{kernel_source_hash()}`", "",
             "## Per kernel (all launches of the run)", "",
             "| kernel | calls | average us | min us | max us | share of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} % |")
    try:
        trace = _rows(directory, "kernel_trace.csv")
    except FileNotFoundError:
        trace = []
    if trace and per_call:
        trace.sort(key=lambda r: int(r["Start_Timestamp"]))
        lines += _per_call_lines(trace)
    elif trace:
        trace.sort(key=lambda r: int(r["Start_Timestamp"]))
        sorts, cur = [], None
        for r in trace:
            if _is("block", r["Kernel_Name"]):
                cur = {"block": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), "merges": []}
                sorts.append(cur)
            elif _is("merge", r["Kernel_Name"]) and cur is not None:
                cur["merges"].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        if sorts:
            npass = statistics.mode(len(s["merges"]) for s in sorts)
            full = [s for s in sorts if len(s["merges"]) == npass]
            lines += ["", f"## One sort, launch by launch (median over {len(full)} sorts)", "",
                      "| launch | kernel | median us |" + (" algorithmic GB/s |" if n_keys else ""),
                      "|---|---|---|" + ("---|" if n_keys else "")]
            med = statistics.median(s["block"] for s in full) / 1e3
            gbs = f" {2 * elem_bytes * n_keys / (med * 1e-6) / 1e9:.0f} |" if n_keys else ""
            lines.append(f"| 0 | block sort | {med:.1f} |{gbs}")
            for i in range(npass):
                med = statistics.median(s["merges"][i] for s in full) / 1e3
                gbs = f" {2 * elem_bytes * n_keys / (med * 1e-6) / 1e9:.0f} |" if n_keys else ""
                lines.append(f"| {i + 1} | merge pass {i + 1} | {med:.1f} |{gbs}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("out")
    t.add_argument("--command", default="")
    t.add_argument("--title", default="Kernel trace")
    t.add_argument("--n", type=int, default=None, help="keys per sort, for algorithmic GB/s")
    t.add_argument("--elem-bytes", type=int, default=4, help="bytes per element moved (keys 4, key/value pairs 8)")
    t.add_argument("--per-call", action="store_true",
                   help="group the library's launches into calls (each starting at the run's first library "
                        "kernel) and list time per kernel per call, in place of the block-sort / merge-pass table")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("out")
    f.add_argument("--n", type=int, required=True, help="u32 elements of the calibration copy")
    f.add_argument("--command", default="")
    ld = sub.add_parser("lds")
    ld.add_argument("dir")
    ld.add_argument("out")
    ld.add_argument("--command", default="")
    sm = sub.add_parser("summary")
    sm.add_argument("traffic_json")
    sm.add_argument("lds_json")
    sm.add_argument("out")
    sm.add_argument("--algorithmic-bytes", type=float, required=True,
                    help="read + write bytes one merge or block-sort launch must move")
    a = ap.parse_args(argv)
    if a.what == "summary":
        with open(a.out, "w") as fh:
            fh.write(counters_markdown(a.traffic_json, a.lds_json, a.algorithmic_bytes))
    elif a.what == "trace":
        text = trace_markdown(a.dir, a.command, a.title, a.n, a.elem_bytes, a.per_call)
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        rec = traffic(a.fetch_dir, a.write_dir, a.n, a.command) if a.what == "traffic" else lds(a.dir, a.command)
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
    print(a.out)


if __name__ == "__main__":
    main()
