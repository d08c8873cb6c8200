"""Helpers for the GPU parity tests: move raw key patterns to the device,
call the C ABI (through the ctypes binding), and get the oracle's answer
for the same input."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2603_08929_amd import _lib
from paper_2603_08929_amd.workloads import DTYPES

# dtype name -> typed C entry point
ENTRY = {"u8": "bsort_u8", "u16": "bsort_u16", "u32": "bsort_u32", "u64": "bsort_u64",
         "i8": "bsort_i8", "i16": "bsort_i16", "i32": "bsort_i32", "i64": "bsort_i64",
         "e4m3": "bsort_f8", "e5m2": "bsort_f8", "f16": "bsort_f16", "bf16": "bsort_f16",
         "f32": "bsort_f32", "f64": "bsort_f64"}
FAMILY = {"U": _lib.KEY_U, "I": _lib.KEY_I, "F": _lib.KEY_F}
CARRIER = {8: torch.int8, 16: torch.int16, 32: torch.int32, 64: torch.int64}
SIGNED_NP = {8: np.int8, 16: np.int16, 32: np.int32, 64: np.int64}


def key_bytes(name: str) -> int:
    return DTYPES[name][0] // 8


def to_device(bits: np.ndarray, name: str) -> torch.Tensor:
    w = DTYPES[name][0]
    arr = np.ascontiguousarray(bits.astype(DTYPES[name][2])).view(SIGNED_NP[w])
    return torch.from_numpy(arr.copy()).to("cuda")


def from_device(t: torch.Tensor, name: str) -> np.ndarray:
    return t.cpu().numpy().view(DTYPES[name][2])


def stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def gpu_sort(name: str, bits: np.ndarray, asc: bool = True, flags: int = 0,
             idx: str = "u32", poison: int = None, scratch_extra: int = 0):
    """Sort through the typed C entry point.  idx in {None, 'u32', 'i64'}.
    Returns (keys as raw patterns, indices as int64 numpy or None)."""
    n = bits.size
    keys = to_device(bits, name)
    fl = flags | (0 if asc else _lib.DESCENDING)
    ind = None
    if idx == "u32":
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
    elif idx == "i64":
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        fl |= _lib.IDX64
    need = _lib.bsort_scratch_bytes(key_bytes(name), n, 1, int(ind is not None), fl)
    scratch = torch.empty(max(need + scratch_extra, 256), dtype=torch.uint8, device="cuda")
    if poison is not None:
        scratch.fill_(poison)
    fn = getattr(_lib, ENTRY[name])
    rc = fn(keys.data_ptr(), n, fl, ind.data_ptr() if ind is not None else None,
            scratch.data_ptr(), scratch.numel(), stream())
    _lib.check(rc, ENTRY[name])
    torch.cuda.synchronize()
    status = _lib.bsort_device_status(scratch.data_ptr(), stream()) if n else 0
    assert status == 0, f"device status {status}"
    out_i = None
    if ind is not None:
        out_i = ind.cpu().numpy()
        out_i = (out_i.view(np.uint32).astype(np.int64) if idx == "u32" else out_i)
    return from_device(keys, name), out_i


def gpu_segmented(name: str, bits: np.ndarray, lengths, asc: bool = True, flags: int = 0,
                  idx: str = "u32"):
    n = bits.size
    keys = to_device(bits, name)
    offs = np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))])
    assert offs[-1] == n
    offsets = torch.from_numpy(offs).to("cuda")
    fl = flags | (0 if asc else _lib.DESCENDING)
    ind = None
    if idx == "u32":
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
    elif idx == "i64":
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        fl |= _lib.IDX64
    B = len(lengths)
    need = _lib.bsort_scratch_bytes(key_bytes(name), n, B, int(ind is not None), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    rc = _lib.bsort_segmented(keys.data_ptr(), FAMILY[DTYPES[name][1]], key_bytes(name),
                              offsets.data_ptr(), B, n, fl,
                              ind.data_ptr() if ind is not None else None,
                              scratch.data_ptr(), scratch.numel(), stream())
    _lib.check(rc, "bsort_segmented")
    torch.cuda.synchronize()
    status = _lib.bsort_device_status(scratch.data_ptr(), stream()) if n else 0
    assert status == 0, f"device status {status}"
    out_i = None
    if ind is not None:
        out_i = ind.cpu().numpy()
        out_i = (out_i.view(np.uint32).astype(np.int64) if idx == "u32" else out_i)
    return from_device(keys, name), out_i, offs


def oracle_sort(name: str, bits: np.ndarray, asc: bool = True):
    k, i = oracle.sort_dtype(bits.astype(np.uint64), name, asc=asc)
    return k.astype(DTYPES[name][2]), i


def gpu_levels(name: str, bits: np.ndarray, levels: int, asc: bool = True, idx: str = "u32",
               lengths=None):
    """The sort stopped after `levels` global levels (bsort_levels), one array
    or back-to-back segments of the given lengths.  Returns (keys as raw
    patterns, indices as int64 numpy or None)."""
    n = bits.size
    keys = to_device(bits, name)
    fl = _lib.PLAIN | (0 if asc else _lib.DESCENDING)
    ind = None
    if idx == "u32":
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
    elif idx == "i64":
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        fl |= _lib.IDX64
    offsets, B = None, 1
    if lengths is not None:
        offs = np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))])
        assert offs[-1] == n
        offsets = torch.from_numpy(offs).to("cuda")
        B = len(lengths)
    need = _lib.bsort_scratch_bytes(key_bytes(name), n, B, int(ind is not None), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    rc = _lib.bsort_levels(keys.data_ptr(), FAMILY[DTYPES[name][1]], key_bytes(name),
                           offsets.data_ptr() if offsets is not None else None, B, n, fl,
                           levels, ind.data_ptr() if ind is not None else None,
                           scratch.data_ptr(), scratch.numel(), stream())
    _lib.check(rc, "bsort_levels")
    torch.cuda.synchronize()
    status = _lib.bsort_device_status(scratch.data_ptr(), stream()) if n else 0
    assert status == 0, f"device status {status}"
    out_i = None
    if ind is not None:
        out_i = ind.cpu().numpy()
        out_i = (out_i.view(np.uint32).astype(np.int64) if idx == "u32" else out_i)
    return from_device(keys, name), out_i


def oracle_snapshots(name: str, bits: np.ndarray, asc: bool = True):
    """The oracle's breadth-first snapshots: row d is the array after every
    partition on the top d bits.  Returns (keys (w+1, n), idx (w+1, n))."""
    w, mode, mant = oracle.DTYPES[name]
    _, _, snap, snap_i = oracle.sort(bits.astype(np.uint64), w, mode, asc=asc, mant_bits=mant,
                                     snapshots=True)
    return snap.astype(DTYPES[name][2]), snap_i
