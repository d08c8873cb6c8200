"""bsort oracle -- TEST INFRASTRUCTURE ONLY.

ctypes loader for the plain single-threaded C oracle in ``bsort_oracle.c``
(written from Algorithms 1-5 of the bsort paper).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package;
the GPU library never does.

Key interpretation: every key is a raw w-bit pattern carried in a uint64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsort_oracle.c")

UNSIGNED, SIGNED, FLOAT = 0, 1, 2
LOMUTO, STABLE = 0, 1

_libs = {}


def lib_path(mutant: int = 0) -> str:
    name = "libbsort_oracle.so" if mutant == 0 else f"libbsort_oracle_mut{mutant}.so"
    return os.path.join(_HERE, name)


def build(mutant: int = 0) -> str:
    """Compile the oracle (or a deliberately wrong mutant of it) with gcc."""
    out = lib_path(mutant)
    cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           f"-DBSO_MUTANT={mutant}", "-o", out + ".tmp", _SRC]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(out + ".tmp", out)
    return out


def _load(mutant: int = 0) -> ctypes.CDLL:
    if mutant in _libs:
        return _libs[mutant]
    path = lib_path(mutant)
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(mutant)
    lib = ctypes.CDLL(path)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.bso_sort.argtypes = [u64p, i64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p, i64p]
    lib.bso_sort.restype = ctypes.c_int
    lib.bso_select.argtypes = [u64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, i64p]
    lib.bso_select.restype = ctypes.c_int
    lib.bso_permute_backward.argtypes = [dp, i64p, ctypes.c_uint64, ctypes.c_uint64, dp]
    lib.bso_permute_backward.restype = ctypes.c_int
    lib.bso_sort128.argtypes = [u64p, u64p, i64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int]
    lib.bso_sort128.restype = ctypes.c_int
    _libs[mutant] = lib
    return lib


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def sort(keys, w: int, mode: int, asc: bool = True, mant_bits: int = 0,
         flavour: int = STABLE, with_idx: bool = True, snapshots: bool = False,
         mutant: int = 0):
    """Sort w-bit patterns.  Returns (keys, idx) or, with snapshots=True,
    (keys, idx, snap, snap_idx) where snap has shape (w+1, n)."""
    lib = _load(mutant)
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).copy()
    n = k.size
    idx = np.arange(n, dtype=np.int64) if with_idx else None
    snap = np.zeros((w + 1, n), dtype=np.uint64) if snapshots else None
    snap_i = np.zeros((w + 1, n), dtype=np.int64) if (snapshots and with_idx) else None
    rc = lib.bso_sort(_ptr(k, ctypes.c_uint64), _ptr(idx, ctypes.c_int64), n, w, mode,
                      mant_bits, int(bool(asc)), flavour, _ptr(snap, ctypes.c_uint64),
                      _ptr(snap_i, ctypes.c_int64))
    if rc != 0:
        raise ValueError(f"bso_sort rejected its arguments (rc={rc})")
    if snapshots:
        return k, idx, snap, snap_i
    return k, idx


def select(keys, w: int, mode: int, asc: bool, j: int, mant_bits: int = 0) -> Tuple[int, int]:
    """(key, source index) at sorted position j of a stable sort."""
    lib = _load()
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    ko = ctypes.c_uint64(0)
    io = ctypes.c_int64(0)
    rc = lib.bso_select(_ptr(k, ctypes.c_uint64), k.size, w, mode, mant_bits,
                        int(bool(asc)), j, ctypes.byref(ko), ctypes.byref(io))
    if rc != 0:
        raise ValueError(f"bso_select rejected its arguments (rc={rc})")
    return int(ko.value), int(io.value)


def sort128(lo, hi, mode: int, asc: bool = True, mant_bits: int = 112):
    """Stable sort of 128-bit patterns hi * 2^64 + lo (uint64 arrays).
    Returns (lo, hi, idx)."""
    lib = _load()
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.uint64)).copy()
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.uint64)).copy()
    if lo.shape != hi.shape:
        raise ValueError("lo and hi differ in shape")
    idx = np.arange(lo.size, dtype=np.int64)
    rc = lib.bso_sort128(_ptr(lo, ctypes.c_uint64), _ptr(hi, ctypes.c_uint64),
                         _ptr(idx, ctypes.c_int64), lo.size, mode, mant_bits, int(bool(asc)))
    if rc != 0:
        raise ValueError(f"bso_sort128 rejected its arguments (rc={rc})")
    return lo, hi, idx


def sort_layout(keys, w: int, mode: int, bit_order, asc: bool = True):
    """Stable sort of w-bit patterns whose order bits are stored in another
    layout: order bit w-1-i lives in stored bit bit_order[i].  Pure Python
    (small inputs): Algorithm 1's split on the stored bit of each order bit,
    Algorithm 2's recursion to the next lower order bit, and the top levels
    of Algorithms 3 and 4 (sign pass in the inverse direction; for floats
    the negative half also inverted).  Returns (keys, idx)."""
    a = [int(k) for k in np.asarray(keys, dtype=np.uint64)]
    idx = list(range(len(a)))
    stored = [int(bit_order[w - 1 - b]) for b in range(w)]  # stored bit of order bit b

    def split(b, ps, pe, up):
        m = 1 << stored[b]
        first = [i for i in range(ps, pe) if ((a[i] & m) == 0) == up]
        second = [i for i in range(ps, pe) if ((a[i] & m) == 0) != up]
        ka = [a[i] for i in first + second]
        ki = [idx[i] for i in first + second]
        a[ps:pe], idx[ps:pe] = ka, ki
        return ps + len(first)

    def bqs(b, ps, pe, up):
        if pe - ps < 2 or b < 0:
            return
        k = split(b, ps, pe, up)
        bqs(b - 1, ps, k, up)
        bqs(b - 1, k, pe, up)

    n = len(a)
    if mode == UNSIGNED:
        bqs(w - 1, 0, n, asc)
    elif n >= 2:
        k = split(w - 1, 0, n, not asc)
        if mode == SIGNED:
            bqs(w - 2, 0, k, asc)
            bqs(w - 2, k, n, asc)
        else:
            neg = (0, k) if asc else (k, n)
            pos = (k, n) if asc else (0, k)
            bqs(w - 2, neg[0], neg[1], not asc)
            bqs(w - 2, pos[0], pos[1], asc)
    return np.array(a, dtype=np.uint64), np.array(idx, dtype=np.int64)


def permute_backward(grad_out: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """grad_in[r, idx[r, j]] = grad_out[r, j] (float64)."""
    lib = _load()
    g = np.ascontiguousarray(grad_out, dtype=np.float64)
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    rows, cols = g.shape
    out = np.zeros_like(g)
    rc = lib.bso_permute_backward(_ptr(g, ctypes.c_double), _ptr(ix, ctypes.c_int64),
                                  rows, cols, _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("idx is not a permutation of each row")
    return out


# Key interpretation per dtype name: (w, mode, mantissa bits).
DTYPES = {
    "u8": (8, UNSIGNED, 0), "u16": (16, UNSIGNED, 0), "u32": (32, UNSIGNED, 0),
    "u64": (64, UNSIGNED, 0),
    "i8": (8, SIGNED, 0), "i16": (16, SIGNED, 0), "i32": (32, SIGNED, 0),
    "i64": (64, SIGNED, 0),
    "e4m3": (8, FLOAT, 3), "e5m2": (8, FLOAT, 2), "f16": (16, FLOAT, 10),
    "bf16": (16, FLOAT, 7), "f32": (32, FLOAT, 23), "f64": (64, FLOAT, 52),
}
# 128-bit keys (sort128): mode and mantissa bits
DTYPES128 = {"u128": (UNSIGNED, 0), "i128": (SIGNED, 0), "f128": (FLOAT, 112)}


def sort_dtype(bits: np.ndarray, dtype: str, asc: bool = True, flavour: int = STABLE):
    """Sort raw bit patterns of a named dtype; returns (bits, idx)."""
    w, mode, mant = DTYPES[dtype]
    return sort(bits, w, mode, asc=asc, mant_bits=mant, flavour=flavour)
