"""ctypes binding of libbsort.so: the C ABI of include/bsort.h, same names,
argument marshalling only.  Every step of the sort runs in the library's
HIP kernels; there is no fallback: if the library is missing this module
raises on import."""
from __future__ import annotations

import ctypes
import os

# torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
# first makes libbsort.so bind to that already-loaded copy, so the process
# has exactly one HIP runtime and torch's streams and memory are valid here.
import torch  # noqa: F401

from .build import LIB

if not os.path.exists(LIB):
    raise ImportError(
        f"libbsort.so not found at {LIB}; build it with "
        "`python -m paper_2603_08929_amd.build` (hipcc, gfx950)")

lib = ctypes.CDLL(LIB)

# status codes and flags (include/bsort.h)
OK, EINVAL, ESCRATCH, ETOOBIG, EHIP, ENODEV, ENOSPACE = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 64 << 20
DESCENDING, NO_SKIP, NO_FINISH, IDX64, KEYS_UNCHANGED = 1, 2, 4, 8, 16
PLAIN = NO_SKIP | NO_FINISH
KEY_U, KEY_I, KEY_F = 0, 1, 2

_vp, _u64, _u32, _i, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t

TYPED = ["u8", "u16", "u32", "u64", "i8", "i16", "i32", "i64", "f8", "f16", "f32", "f64"]
SYMBOLS = ["bsort_scratch_bytes", "bsort_sort", "bsort_segmented", "bsort_segmented_f32",
           "bsort_segmented_i32", "bsort_backward_scatter", "bsort_strerror",
           "bsort_device_status", "bsort_level_stats", "bsort_timing_arm",
           "bsort_timing_read", "bsort_timing_disarm", "bsort_config_count",
           "bsort_config_name", "bsort_config_override", "bsort_tuned_config",
           "bsort_autotune", "bsort_autotune_reset", "bsort_graph_create",
           "bsort_graph_launch", "bsort_graph_destroy", "bsort_pairs_scratch_bytes",
           "bsort_sort_pairs", "bsort_segmented_pairs", "bsort_gather",
           "bsort_scratch_bytes128", "bsort_sort128", "bsort_sort_layout",
           "bsort_inplace_scratch_bytes", "bsort_sort_inplace", "bsort_segmented_inplace",
           "bsort_scatter", "bsort_autotune_save", "bsort_autotune_load",
           "bsort_segmented_noalloc", "bsort_levels", "bsort_level_bytes"] + \
    [f"bsort_{t}" for t in TYPED]

lib.bsort_scratch_bytes.argtypes = [_i, _u64, _u64, _i, _u32]
lib.bsort_scratch_bytes.restype = _sz
for t in TYPED:
    fn = getattr(lib, f"bsort_{t}")
    fn.argtypes = [_vp, _u64, _u32, _vp, _vp, _sz, _vp]
    fn.restype = _i
lib.bsort_sort.argtypes = [_vp, _i, _i, _u64, _u32, _vp, _vp, _sz, _vp]
lib.bsort_sort.restype = _i
lib.bsort_segmented.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _vp, _vp, _sz, _vp]
lib.bsort_segmented.restype = _i
lib.bsort_segmented_noalloc.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _vp, _vp]
lib.bsort_segmented_noalloc.restype = _i
lib.bsort_levels.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _i, _vp, _vp, _sz, _vp]
lib.bsort_levels.restype = _i
lib.bsort_level_bytes.argtypes = [_vp, _vp, _vp, _vp, _i]
lib.bsort_level_bytes.restype = _i
for t in ("f32", "i32"):
    fn = getattr(lib, f"bsort_segmented_{t}")
    fn.argtypes = [_vp, _vp, _u64, _u64, _u32, _vp, _vp, _sz, _vp]
    fn.restype = _i
lib.bsort_backward_scatter.argtypes = [_vp, _vp, _u64, _u64, _i, _vp, _u32, _vp]
lib.bsort_backward_scatter.restype = _i
lib.bsort_pairs_scratch_bytes.argtypes = [_i, _u64, _u64, _i, _i, _u32]
lib.bsort_pairs_scratch_bytes.restype = _sz
lib.bsort_sort_pairs.argtypes = [_vp, _i, _i, _u64, _u32, _vp, _i, _vp, _vp, _sz, _vp]
lib.bsort_sort_pairs.restype = _i
lib.bsort_segmented_pairs.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _vp, _i, _vp, _vp,
                                      _sz, _vp]
lib.bsort_segmented_pairs.restype = _i
lib.bsort_gather.argtypes = [_vp, _i, _vp, _vp, _u64, _u64, _u32, _vp, _vp]
lib.bsort_gather.restype = _i
lib.bsort_scatter.argtypes = [_vp, _i, _vp, _vp, _u64, _u64, _u32, _vp, _vp]
lib.bsort_scatter.restype = _i
lib.bsort_autotune_save.argtypes = [ctypes.c_char_p]
lib.bsort_autotune_save.restype = _i
lib.bsort_autotune_load.argtypes = [ctypes.c_char_p]
lib.bsort_autotune_load.restype = _i
lib.bsort_scratch_bytes128.argtypes = [_u64, _i, _u32]
lib.bsort_scratch_bytes128.restype = _sz
lib.bsort_sort128.argtypes = [_vp, _i, _u64, _u32, _vp, _vp, _sz, _vp]
lib.bsort_sort128.restype = _i
lib.bsort_sort_layout.argtypes = [_vp, _i, _i, _u64, _u32, ctypes.POINTER(ctypes.c_uint8), _vp,
                                  _vp, _sz, _vp]
lib.bsort_sort_layout.restype = _i
lib.bsort_inplace_scratch_bytes.argtypes = [_i, _u64, _u64, _u32]
lib.bsort_inplace_scratch_bytes.restype = _sz
lib.bsort_sort_inplace.argtypes = [_vp, _i, _i, _u64, _u32, _vp, _sz, _vp]
lib.bsort_sort_inplace.restype = _i
lib.bsort_segmented_inplace.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _vp, _sz, _vp]
lib.bsort_segmented_inplace.restype = _i
lib.bsort_strerror.argtypes = [_i]
lib.bsort_strerror.restype = ctypes.c_char_p
lib.bsort_device_status.argtypes = [_vp, _vp]
lib.bsort_device_status.restype = _i
lib.bsort_level_stats.argtypes = [_vp, _vp, _vp, _vp, _vp, _i, _vp, _vp]
lib.bsort_level_stats.restype = _i
lib.bsort_timing_arm.argtypes = [_i]
lib.bsort_timing_arm.restype = _i
lib.bsort_timing_read.argtypes = [_vp, _vp, _i]
lib.bsort_timing_read.restype = _i
lib.bsort_timing_disarm.argtypes = []
lib.bsort_timing_disarm.restype = None
lib.bsort_config_count.argtypes = []
lib.bsort_config_count.restype = _i
lib.bsort_config_name.argtypes = [_i]
lib.bsort_config_name.restype = ctypes.c_char_p
lib.bsort_config_override.argtypes = [_i]
lib.bsort_config_override.restype = _i
lib.bsort_tuned_config.argtypes = [_i, _i, _u64, _u64]
lib.bsort_tuned_config.restype = _i
lib.bsort_autotune.argtypes = [_vp, _i, _i, _vp, _u64, _u64, _u32, _vp, _vp, _sz, _vp, _i]
lib.bsort_autotune.restype = _i
lib.bsort_autotune_reset.argtypes = []
lib.bsort_autotune_reset.restype = None
lib.bsort_graph_create.argtypes = [ctypes.POINTER(_vp), _vp, _i, _i, _vp, _u64, _u64, _u32, _vp,
                                   _vp, _sz]
lib.bsort_graph_create.restype = _i
lib.bsort_graph_launch.argtypes = [_vp, _vp]
lib.bsort_graph_launch.restype = _i
lib.bsort_graph_destroy.argtypes = [_vp]
lib.bsort_graph_destroy.restype = _i


def strerror(rc: int) -> str:
    return lib.bsort_strerror(rc).decode()


def check(rc: int, what: str) -> None:
    if rc != OK:
        raise RuntimeError(f"{what} failed: {strerror(rc)} (status {rc})")


# the same names as the C ABI
bsort_scratch_bytes = lib.bsort_scratch_bytes
bsort_sort = lib.bsort_sort
bsort_segmented = lib.bsort_segmented
bsort_segmented_noalloc = lib.bsort_segmented_noalloc
bsort_levels = lib.bsort_levels
bsort_level_bytes = lib.bsort_level_bytes
bsort_segmented_f32 = lib.bsort_segmented_f32
bsort_segmented_i32 = lib.bsort_segmented_i32
bsort_backward_scatter = lib.bsort_backward_scatter
bsort_strerror = lib.bsort_strerror
bsort_device_status = lib.bsort_device_status
bsort_level_stats = lib.bsort_level_stats
bsort_timing_arm = lib.bsort_timing_arm
bsort_timing_read = lib.bsort_timing_read
bsort_timing_disarm = lib.bsort_timing_disarm
bsort_config_count = lib.bsort_config_count
bsort_config_name = lib.bsort_config_name
bsort_config_override = lib.bsort_config_override
bsort_tuned_config = lib.bsort_tuned_config
bsort_autotune = lib.bsort_autotune
bsort_autotune_reset = lib.bsort_autotune_reset
bsort_graph_create = lib.bsort_graph_create
bsort_graph_launch = lib.bsort_graph_launch
bsort_graph_destroy = lib.bsort_graph_destroy
bsort_pairs_scratch_bytes = lib.bsort_pairs_scratch_bytes
bsort_sort_pairs = lib.bsort_sort_pairs
bsort_segmented_pairs = lib.bsort_segmented_pairs
bsort_gather = lib.bsort_gather
bsort_scatter = lib.bsort_scatter
bsort_autotune_save = lib.bsort_autotune_save
bsort_autotune_load = lib.bsort_autotune_load
bsort_scratch_bytes128 = lib.bsort_scratch_bytes128
bsort_sort128 = lib.bsort_sort128
bsort_sort_layout = lib.bsort_sort_layout
bsort_inplace_scratch_bytes = lib.bsort_inplace_scratch_bytes
bsort_sort_inplace = lib.bsort_sort_inplace
bsort_segmented_inplace = lib.bsort_segmented_inplace
for _t in TYPED:
    globals()[f"bsort_{_t}"] = getattr(lib, f"bsort_{_t}")
