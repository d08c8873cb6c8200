"""Pins of the oracle's 128-bit sort (the method at w = 128, which the
paper's Section III-C says carries over to any word size).

- Brute force with numeric semantics: the keys are read as numbers --
  unsigned and two's-complement integers as Python ints, binary128 floats
  decoded exactly to fractions with the special values of Section III-C
  (-NaN first by descending payload, -inf, ..., -0 < +0, ..., +inf, +NaN by
  ascending payload) -- and Python's stable sort orders them.
- The same closed form through numpy's stable lexsort at larger sizes.
- Agreement with the 64-bit oracle where the two meet: sign-extended 64-bit
  integers, and binary64 values widened exactly to binary128.
- Independence of the mantissa width passed to Algorithm 5.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1
TOP = 1 << 127


def split(v):
    return np.array([x & M64 for x in v], dtype=np.uint64), \
        np.array([x >> 64 for x in v], dtype=np.uint64)


def join(lo, hi):
    return [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]


def numeric_key(v, mode):
    if mode == oracle.UNSIGNED:
        return v
    if mode == oracle.SIGNED:
        return v - (1 << 128) if v & TOP else v
    s, e, f = v >> 127, (v >> 112) & 0x7FFF, v & ((1 << 112) - 1)
    if e == 0x7FFF and f:
        return (0, -f) if s else (4, f)
    if e == 0x7FFF:
        return (1,) if s else (3,)
    mag = Fraction(f, 1 << (112 + 16382)) if e == 0 else \
        Fraction((1 << 112) + f) * Fraction(2) ** (e - 16383 - 112)
    val = -mag if s else mag
    return (2, val, -1 if (s and val == 0) else 0)


def f128(sign, exp, frac):
    return (sign << 127) | (exp << 112) | frac


def special_pool(rng):
    """binary128 patterns: zeros, subnormals, normals sharing high words,
    infinities and NaNs."""
    pool = [f128(0, 0, 0), f128(1, 0, 0), f128(0, 0, 1), f128(1, 0, 1),
            f128(0, 0, (1 << 112) - 1), f128(0, 16383, 0), f128(1, 16383, 0),
            f128(0, 16383, 1), f128(0, 16383, 1 << 64), f128(1, 16383, 1 << 64),
            f128(0, 16384, 5), f128(1, 1, 0), f128(0, 0x7FFE, (1 << 112) - 1),
            f128(0, 0x7FFF, 0), f128(1, 0x7FFF, 0), f128(0, 0x7FFF, 1), f128(1, 0x7FFF, 1),
            f128(0, 0x7FFF, 1 << 111), f128(1, 0x7FFF, (1 << 112) - 1)]
    for _ in range(8):
        pool.append(int(rng.integers(0, 1 << 63)) << 64 | int(rng.integers(0, 1 << 63)))
    return pool


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.SIGNED, oracle.FLOAT])
def test_brute_force_numeric_order(mode):
    rng = np.random.default_rng(60 + mode)
    pool = special_pool(rng) + [TOP, TOP - 1, 0, 1, M64, M64 + 1, (1 << 128) - 1]
    for trial in range(300):
        n = int(rng.integers(1, 9))
        v = [pool[int(i)] for i in rng.integers(0, len(pool), size=n)]
        lo, hi = split(v)
        for asc in (True, False):
            want = sorted(range(n), key=lambda i: numeric_key(v[i], mode), reverse=not asc)
            slo, shi, idx = oracle.sort128(lo, hi, mode, asc=asc)
            assert list(idx) == want, (trial, asc, [hex(x) for x in v])
            assert join(slo, shi) == [v[i] for i in want]


def order_key(lo, hi, mode, asc):
    """(v_lo, v_hi): the unsigned order key of Section III's mapping."""
    if mode == oracle.SIGNED:
        hi = hi ^ np.uint64(1 << 63)
    elif mode == oracle.FLOAT:
        neg = (hi >> np.uint64(63)) != 0
        lo, hi = np.where(neg, ~lo, lo), np.where(neg, ~hi, hi | np.uint64(1 << 63))
    if not asc:
        lo, hi = ~lo, ~hi
    return lo, hi


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.SIGNED, oracle.FLOAT])
def test_closed_form_large(mode):
    rng = np.random.default_rng(70 + mode)
    n = 20000
    pool = special_pool(rng)
    v = [pool[int(i)] for i in rng.integers(0, len(pool), size=n // 4)]
    lo, hi = split(v)
    # plus random patterns, half of them sharing a few high words
    rl = rng.integers(0, 1 << 63, size=3 * n // 4, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=3 * n // 4, dtype=np.uint64)
    rh = rng.integers(0, 1 << 63, size=3 * n // 4, dtype=np.uint64) * np.uint64(2)
    rh[::2] = np.array([0x8000000000000000, 0x3FFF000000000000, 7], dtype=np.uint64)[
        rng.integers(0, 3, size=rh[::2].size)]
    lo, hi = np.concatenate([lo, rl]), np.concatenate([hi, rh])
    perm = rng.permutation(lo.size)
    lo, hi = lo[perm], hi[perm]
    for asc in (True, False):
        vlo, vhi = order_key(lo, hi, mode, asc)
        want = np.lexsort((vlo, vhi))  # stable: equal keys keep input order
        slo, shi, idx = oracle.sort128(lo, hi, mode, asc=asc)
        np.testing.assert_array_equal(idx, want)
        np.testing.assert_array_equal(slo, lo[want])
        np.testing.assert_array_equal(shi, hi[want])


def widen_f64(b):
    """Exact binary64 -> binary128 conversion of a bit pattern."""
    s, e, f = b >> 63, (b >> 52) & 0x7FF, b & ((1 << 52) - 1)
    if e == 0x7FF:
        return f128(s, 0x7FFF, f << 60)
    if e == 0:
        if f == 0:
            return f128(s, 0, 0)
        top = f.bit_length() - 1           # value = f * 2^-1074
        exp = top - 1074 + 16383
        return f128(s, exp, (f - (1 << top)) << (112 - top))
    return f128(s, e - 1023 + 16383, f << 60)


def test_agrees_with_64_bit_oracle():
    rng = np.random.default_rng(80)
    n = 5000
    u = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    u[::3] = u[rng.integers(0, n, size=u[::3].size)]  # duplicates
    for asc in (True, False):
        # unsigned: high word zero
        _, _, idx = oracle.sort128(u, np.zeros(n, dtype=np.uint64), oracle.UNSIGNED, asc=asc)
        np.testing.assert_array_equal(idx, oracle.sort(u, 64, oracle.UNSIGNED, asc=asc)[1])
        # signed: sign extension keeps the order
        hi = np.where((u >> np.uint64(63)) != 0, np.uint64(M64), np.uint64(0))
        _, _, idx = oracle.sort128(u, hi, oracle.SIGNED, asc=asc)
        np.testing.assert_array_equal(idx, oracle.sort(u, 64, oracle.SIGNED, asc=asc)[1])
    # floats: binary64 values (with specials) widened exactly
    vals = rng.standard_normal(n) * np.exp2(rng.integers(-1080, 1020, size=n).astype(np.float64))
    b = vals.view(np.uint64).copy()
    specials = np.array([0, 1 << 63, 1, (1 << 63) | 1, 0x7FF0000000000000, 0xFFF0000000000000,
                         0x7FF8000000000001, 0xFFF8000000000002, 0x000FFFFFFFFFFFFF],
                        dtype=np.uint64)
    b[:specials.size] = specials
    b = b[rng.permutation(n)]
    w = [widen_f64(int(x)) for x in b]
    lo, hi = split(w)
    for asc in (True, False):
        _, _, idx = oracle.sort128(lo, hi, oracle.FLOAT, asc=asc)
        np.testing.assert_array_equal(idx, oracle.sort(b, 64, oracle.FLOAT, asc=asc,
                                                       mant_bits=52)[1])


def test_mantissa_width_does_not_matter():
    rng = np.random.default_rng(90)
    pool = special_pool(rng)
    v = [pool[int(i)] for i in rng.integers(0, len(pool), size=3000)]
    lo, hi = split(v)
    ref = oracle.sort128(lo, hi, oracle.FLOAT, mant_bits=112)[2]
    for mb in (0, 1, 50, 111, 126):
        np.testing.assert_array_equal(oracle.sort128(lo, hi, oracle.FLOAT, mant_bits=mb)[2], ref)
