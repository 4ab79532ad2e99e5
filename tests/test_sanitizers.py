"""Host-code sanitizer runs (CPU only): the oracle under gcc's
AddressSanitizer + UndefinedBehaviorSanitizer, and the host side of the C ABI
(argument checks, temp queries, the host planners) built by hipcc with the
sanitizers on the host pass only (``-Xarch_host``), driven by small native
programs under ``tests/sanitize/``.  GPU code is never instrumented."""

import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(SAN, "_build")
CSRC = os.path.join(ROOT, "paper_1306_5076_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIB_SOURCES = ["bcf_kernels.hip", "bcf_api.hip", "bcf_cps.hip", "bcf_u64.hip", "bcf_dist.hip", "bcf_noalloc.hip",
               "bcf_plan.hip"]
HOST_SAN = ["-Xarch_host", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}"
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(SAN, "oracle_check.c"),
          os.path.join(ROOT, "oracle", "bcf_oracle.c")])
    assert "ok" in _run([exe], env=ENV, timeout=300)


def _source_hash():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)) + ["../../include/bcf.h", "../../tests/sanitize/abi_host_check.cpp"]:
        p = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(p):
            h.update(name.encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_abi_under_asan_ubsan():
    """The library's host code built with ASan + UBSan (cached by source hash
    under tests/sanitize/_build), then driven through every host-only path."""
    tag = _source_hash()
    exe = os.path.join(BUILD, f"abi_host_check_{tag}")
    if not os.path.exists(exe):
        if os.path.isdir(BUILD):
            shutil.rmtree(BUILD)
        os.makedirs(BUILD)
        common = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", *HOST_SAN,
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-I", os.path.join(ROOT, "include"), "-I", CSRC]
        procs, objs = [], []
        for s in LIB_SOURCES:
            o = os.path.join(BUILD, s.replace(".hip", ".o"))
            objs.append(o)
            procs.append(subprocess.Popen([*common, "-c", os.path.join(CSRC, s), "-o", o],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        for p in procs:
            out, _ = p.communicate()
            assert p.returncode == 0, out[-4000:]
        drv = os.path.join(BUILD, "drv.o")
        _run([HIPCC, "--cuda-host-only", "-O1", "-std=c++17", *HOST_SAN, "-I", os.path.join(ROOT, "include"),
              "-c", "-x", "c++", os.path.join(SAN, "abi_host_check.cpp"), "-o", drv])
        _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", drv, *objs, "-o", exe + ".tmp"])
        os.replace(exe + ".tmp", exe)
    assert "ok" in _run([exe], env=ENV, timeout=300)
