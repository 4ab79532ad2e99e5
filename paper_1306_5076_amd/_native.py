"""ctypes view of libbcf.so (the C ABI declared in include/bcf.h).

Only argument marshalling lives here: every step of a sort runs in the HIP
kernels of the library.  There is no fallback: if the library is missing or a
call fails, an exception is raised.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbcf.so")

BCF_OK = 0
STATUS_NAMES = {
    0: "BCF_OK",
    1: "BCF_ERR_INVALID",
    2: "BCF_ERR_TEMP_TOO_SMALL",
    3: "BCF_ERR_NOMEM",
    4: "BCF_ERR_DEVICE",
    5: "BCF_ERR_UNSORTED_RUN",
}

# every symbol include/bcf.h declares
EXPORTED = (
    "bcf_sort_u32",
    "bcf_sort_u32_noalloc",
    "bcf_sort_pairs_u32",
    "bcf_sort_i32",
    "bcf_sort_f32",
    "bcf_sort_pairs_i32",
    "bcf_sort_pairs_f32",
    "bcf_colored_prefix_sums",
    "bcf_sort_u64",
    "bcf_merge_runs",
    "bcf_merge_runs_host",
    "bcf_distribute_runs",
    "bcf_merge_run_groups",
    "bcf_sort_u32_pb",
    "bcf_segmented_sort",
    "bcf_segmented_sort_pairs",
    "bcf_segmented_sort_host",
    "bcf_segmented_sort_pairs_host",
    "bcf_segmented_upload",
    "bcf_segmented_execute",
    "bcf_status_string",
    "bcf_tile_keys",
    "bcf_run_keys",
    "bcf_sort_passes",
    "bcf_get_tuning",
    "bcf_set_tuning",
    "bcf_profile_enable",
    "bcf_profile_collect",
)


class BcfError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {msg}")
        self.status = status


class Tuning(ctypes.Structure):
    """Mirror of bcf_tuning (include/bcf.h)."""

    _fields_ = [
        ("merge_variant", ctypes.c_int32),
        ("nontemporal", ctypes.c_int32),
        ("sampled_partition", ctypes.c_int32),
        ("tile_samples", ctypes.c_int32),
        ("group_min_keys", ctypes.c_uint64),
        ("check_runs", ctypes.c_int32),
        ("block_sort", ctypes.c_int32),
        ("fused_partition", ctypes.c_int32),
        ("merge_fan_in", ctypes.c_int32),
    ]


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (after torch, so that both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library not built: {path}. Run __graft_entry__.build() (hipcc, gfx950) first."
        )
    try:  # torch first: its libamdhip64 then also serves libbcf.so
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.bcf_sort_u32.argtypes = [vp, vp, u64, vp, u64p, vp]
    lib.bcf_sort_pairs_u32.argtypes = [vp, vp, vp, vp, u64, vp, u64p, vp]
    lib.bcf_sort_u32_noalloc.argtypes = [vp, vp, u64, vp]
    lib.bcf_sort_u32_noalloc.restype = ctypes.c_int
    for f in ("bcf_sort_i32", "bcf_sort_f32"):
        getattr(lib, f).argtypes = [vp, vp, u64, vp, u64p, vp]
        getattr(lib, f).restype = ctypes.c_int
    for f in ("bcf_sort_pairs_i32", "bcf_sort_pairs_f32"):
        getattr(lib, f).argtypes = [vp, vp, vp, vp, u64, vp, u64p, vp]
        getattr(lib, f).restype = ctypes.c_int
    lib.bcf_colored_prefix_sums.argtypes = [vp, vp, vp, u64, u32, ctypes.c_int, vp, u64p, vp]
    lib.bcf_colored_prefix_sums.restype = ctypes.c_int
    lib.bcf_sort_u64.argtypes = [vp, vp, u64, vp, u64p, vp]
    lib.bcf_sort_u64.restype = ctypes.c_int
    lib.bcf_merge_runs.argtypes = [vp, vp, vp, u32, vp, vp, vp, u64p, vp]  # device offsets
    lib.bcf_merge_runs_host.argtypes = [vp, vp, u64p, u32, vp, vp, vp, u64p, vp]
    lib.bcf_sort_u32_pb.argtypes = [vp, vp, u64, u32, u32, ctypes.c_int, vp, u64p, vp]
    lib.bcf_distribute_runs.argtypes = [vp, u64p, u32, u32, u32, ctypes.c_int, vp, vp, vp, vp, u64p, vp]
    lib.bcf_merge_run_groups.argtypes = [vp, vp, u64p, u32, ctypes.POINTER(u32), u32, vp, vp, vp, u64p, vp]
    lib.bcf_segmented_sort.argtypes = [vp, vp, vp, u32, vp, u64p, vp]  # device offsets
    lib.bcf_segmented_sort_pairs.argtypes = [vp, vp, vp, vp, vp, u32, vp, u64p, vp]
    lib.bcf_segmented_sort_host.argtypes = [vp, vp, u64p, u32, vp, u64p, vp]
    lib.bcf_segmented_sort_pairs_host.argtypes = [vp, vp, vp, vp, u64p, u32, vp, u64p, vp]
    lib.bcf_segmented_upload.argtypes = [u64p, u32, ctypes.c_int, vp, u64p, vp]
    lib.bcf_segmented_execute.argtypes = [vp, vp, vp, vp, u64p, u32, vp, u64p, vp]
    for f in ("bcf_sort_u32", "bcf_sort_pairs_u32", "bcf_merge_runs", "bcf_merge_runs_host", "bcf_distribute_runs",
              "bcf_merge_run_groups", "bcf_sort_u32_pb", "bcf_segmented_sort", "bcf_segmented_sort_pairs",
              "bcf_segmented_sort_host", "bcf_segmented_sort_pairs_host", "bcf_segmented_upload",
              "bcf_segmented_execute"):
        getattr(lib, f).restype = ctypes.c_int
    lib.bcf_status_string.argtypes = [ctypes.c_int]
    lib.bcf_status_string.restype = ctypes.c_char_p
    lib.bcf_tile_keys.argtypes = []
    lib.bcf_tile_keys.restype = u32
    lib.bcf_run_keys.argtypes = [ctypes.c_int]
    lib.bcf_run_keys.restype = u32
    lib.bcf_sort_passes.argtypes = [u64, ctypes.c_int]
    lib.bcf_sort_passes.restype = u32
    lib.bcf_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.bcf_get_tuning.restype = None
    lib.bcf_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.bcf_set_tuning.restype = ctypes.c_int
    lib.bcf_profile_enable.argtypes = [ctypes.c_int]
    lib.bcf_profile_enable.restype = None
    lib.bcf_profile_collect.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int]
    lib.bcf_profile_collect.restype = ctypes.c_int
    _lib = lib
    return lib


def check(fn: str, status: int):
    if status != BCF_OK:
        msg = load().bcf_status_string(status).decode()
        raise BcfError(fn, status, msg)
