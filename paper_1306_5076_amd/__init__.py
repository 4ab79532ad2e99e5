"""MI355X (gfx950) bank-conflict-free comparison sort.

HIP kernels behind a C ABI (include/bcf.h, libbcf.so); this package adds the
torch-tensor front end.  Importing it does not touch the GPU.
"""

import importlib

from ._native import EXPORTED, LIB_PATH, BcfError  # noqa: F401

_API = (
    "Workspace",
    "sort_u32",
    "sort_pairs_u32",
    "sort_i32",
    "sort_f32",
    "sort_pairs_i32",
    "sort_pairs_f32",
    "colored_prefix_sums",
    "sort_u64",
    "merge_runs",
    "distribute_runs",
    "merge_run_groups",
    "sort_u32_pb",
    "segmented_sort",
    "SegmentedPlan",
    "tile_keys",
    "run_keys",
    "sort_passes",
    "profile_enable",
    "profile_collect",
    "get_tuning",
    "set_tuning",
    "tuning",
)


def __getattr__(name):
    if name in _API:
        return getattr(importlib.import_module(__name__ + ".api"), name)
    raise AttributeError(name)
