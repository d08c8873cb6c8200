"""Seeded synthetic inputs (numpy PCG64), returned as raw key bit patterns.

These generators are the only code that both the GPU path's tests/benchmark
and the CPU oracle consume; they draw numbers and pack bits and do none of
the sort's arithmetic.  The paper sorts synthetic arrays of char, short,
int, long long, float and double (Section IV-B, Table 2) without saying how
they were distributed; these recipes stand in for them:

* integers: uniform over the full range of the type;
* floats: N(0, 1) draws rounded to the type (fp16 / bf16 round to nearest
  even from float32), optionally with signed zeros, subnormals and
  infinities planted at seeded positions;
* heavy duplicates: uint32 uniform in [0, 16);
* presorted / reverse-sorted uint32;
* batched: log-uniform lengths in [1, 2^20].
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

# name -> (bits, family, numpy raw dtype, numpy value dtype or None)
DTYPES: Dict[str, Tuple[int, str, type, object]] = {
    "u8": (8, "U", np.uint8, np.uint8), "u16": (16, "U", np.uint16, np.uint16),
    "u32": (32, "U", np.uint32, np.uint32), "u64": (64, "U", np.uint64, np.uint64),
    "i8": (8, "I", np.uint8, np.int8), "i16": (16, "I", np.uint16, np.int16),
    "i32": (32, "I", np.uint32, np.int32), "i64": (64, "I", np.uint64, np.int64),
    "e4m3": (8, "F", np.uint8, None), "e5m2": (8, "F", np.uint8, None),
    "f16": (16, "F", np.uint16, np.float16), "bf16": (16, "F", np.uint16, None),
    "f32": (32, "F", np.uint32, np.float32), "f64": (64, "F", np.uint64, np.float64),
}


def raw_dtype(name: str):
    return DTYPES[name][2]


def uniform_bits(name: str, n: int, seed: int) -> np.ndarray:
    """Every bit pattern equally likely (uniform over the integer range)."""
    bits, _, raw, _ = DTYPES[name]
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, size=n, dtype=np.uint64, endpoint=False
                        ).astype(raw) if bits < 64 else \
        rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


def normal_bits(name: str, n: int, seed: int) -> np.ndarray:
    """N(0, 1) values rounded to the float type, as bit patterns."""
    rng = np.random.default_rng(seed)
    if name == "f64":
        return rng.standard_normal(n).view(np.uint64)
    x = rng.standard_normal(n, dtype=np.float32)
    if name == "f32":
        return x.view(np.uint32)
    if name == "f16":
        return x.astype(np.float16).view(np.uint16)
    if name == "bf16":
        u = x.view(np.uint32).astype(np.uint64)
        # round to nearest even on the upper 16 bits (no NaNs in N(0,1) draws)
        r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
        return r.astype(np.uint16)
    raise ValueError(name)


def plant_specials(bits: np.ndarray, name: str, frac: float, seed: int) -> np.ndarray:
    """Overwrite frac*n positions each (disjoint, seeded) with signed zeros
    (half negative), subnormals (random sign, nonzero random mantissa) and
    infinities (half negative)."""
    w, fam, raw, _ = DTYPES[name]
    assert fam == "F"
    mant = {"f16": 10, "bf16": 7, "f32": 23, "f64": 52, "e5m2": 2, "e4m3": 3}[name]
    n = bits.size
    m = int(round(frac * n))
    if m == 0:
        return bits
    rng = np.random.default_rng(seed)
    out = bits.copy()
    pos = rng.choice(n, size=3 * m, replace=False)
    one = np.uint64(1)
    sign = one << np.uint64(w - 1)
    signs = lambda: np.where(rng.integers(0, 2, m) == 1, sign, np.uint64(0))
    expo_all = ((one << np.uint64(w - 1 - mant)) - one) << np.uint64(mant)
    zeros = signs()
    subs = rng.integers(1, 1 << mant, size=m, dtype=np.uint64) | signs()
    infs = expo_all | signs()
    out[pos[:m]] = zeros.astype(raw)
    out[pos[m:2 * m]] = subs.astype(raw)
    out[pos[2 * m:]] = infs.astype(raw)
    return out


def plant_nans(bits: np.ndarray, name: str, frac: float, seed: int) -> np.ndarray:
    """Overwrite frac*n seeded positions with NaN patterns: all exponent bits
    set, a nonzero random mantissa (quiet and signalling payloads alike), a
    random sign."""
    w, fam, raw, _ = DTYPES[name]
    assert fam == "F"
    mant = {"f16": 10, "bf16": 7, "f32": 23, "f64": 52, "e5m2": 2}[name]
    n = bits.size
    m = int(round(frac * n))
    if m == 0:
        return bits
    rng = np.random.default_rng(seed)
    out = bits.copy()
    pos = rng.choice(n, size=m, replace=False)
    one = np.uint64(1)
    sign = one << np.uint64(w - 1)
    expo_all = ((one << np.uint64(w - 1 - mant)) - one) << np.uint64(mant)
    payload = rng.integers(1, 1 << mant, size=m, dtype=np.uint64)
    signs = np.where(rng.integers(0, 2, m) == 1, sign, np.uint64(0))
    out[pos] = (expo_all | payload | signs).astype(raw)
    return out


def all_patterns(name: str, dup_frac: float, seed: int) -> np.ndarray:
    """Every bit pattern of an 8- or 16-bit dtype once, plus dup_frac * 2^w
    seeded repeats, in a seeded random order."""
    w, _, raw, _ = DTYPES[name]
    assert w <= 16
    rng = np.random.default_rng(seed)
    every = np.arange(1 << w, dtype=np.uint64)
    extra = rng.integers(0, 1 << w, size=int(dup_frac * (1 << w)), dtype=np.uint64)
    out = np.concatenate([every, extra])
    return out[rng.permutation(out.size)].astype(raw)


def heavy_duplicates_u32(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 16, size=n, dtype=np.uint32)


def presorted_u32(n: int, seed: int, reverse: bool = False) -> np.ndarray:
    x = np.sort(np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64)
                ).astype(np.uint32)
    return x[::-1].copy() if reverse else x


def batched_lengths(num: int = 4096, max_len: int = 1 << 20, seed: int = 2) -> np.ndarray:
    """L_i = floor(exp(u_i * ln(max_len + 1))), u ~ U[0, 1): log-uniform in
    [1, max_len]."""
    u = np.random.default_rng(seed).random(num)
    return np.floor(np.exp(u * np.log(max_len + 1.0))).astype(np.int64)


def mixed_bits(name: str, n: int, seed: int) -> np.ndarray:
    """Test input: uniform patterns for integers; N(0,1) for floats with
    specials; plus duplicated runs, so every path (ties, signs, specials)
    is exercised."""
    w, fam, raw, _ = DTYPES[name]
    if fam == "F" and name not in ("e4m3", "e5m2"):
        bits = plant_specials(normal_bits(name, n, seed), name, 0.01, seed + 1)
    else:
        bits = uniform_bits(name, n, seed)
    if n >= 8:
        rng = np.random.default_rng(seed + 2)
        k = n // 8
        bits[rng.choice(n, size=k, replace=False)] = bits[rng.choice(n, size=k)]
    return np.ascontiguousarray(bits.astype(raw))
