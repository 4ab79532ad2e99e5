"""Build the HIP library (libbcf.so) and the LDS probe for gfx950 with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).  Objects are compiled
in parallel, then linked into ``paper_1306_5076_amd/libbcf.so``.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbcf.so")
PROBE_SRC = os.path.join(PKG, "probes", "lds_bank_probe.hip")
PROBE_BIN = os.path.join(PKG, "probes", "lds_bank_probe")

ARCH = os.environ.get("BCF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]
SOURCES = ["bcf_kernels.hip", "bcf_api.hip", "bcf_cps.hip", "bcf_u64.hip", "bcf_dist.hip", "bcf_noalloc.hip", "bcf_plan.hip"]
# The key/value networks compare elements as doubles (v_min_f64 / v_max_f64)
# that are never NaN; with the IEEE mode bit clear the compiler does not
# quieten (canonicalise) every value read back from LDS before comparing it.
EXTRA = {"bcf_kernels.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"]}


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = [os.path.join(BUILD, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = [[HIPCC, *COMMON, *EXTRA.get(s, []), "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    jobs.append([HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", PROBE_SRC, "-o", PROBE_BIN])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(_run, jobs))
    tmp = LIB + ".tmp"
    outs.append(_run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]))
    os.replace(tmp, LIB)
    if verbose:
        print("\n".join(o for o in outs if o.strip()), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
