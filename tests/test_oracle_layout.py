"""Pins of the oracle's sort for keys whose order bits are stored in
another layout (Section III-C: other arrangements sort with small changes).

- The identity layout gives the C oracle's sort.
- A concrete format with the sign in the lowest stored bit (half precision
  stored as exponent | mantissa | sign), decoded to exact numbers and
  ordered by Python's stable sort, brute force over small multisets.
- Any layout gives the C oracle's sort of the keys with their bits moved
  into order (plain bit manipulation written here).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def to_order_bits(keys, w, bit_order):
    """order word: bit w-1-i is stored bit bit_order[i]."""
    out = np.zeros_like(keys)
    for i, sb in enumerate(bit_order):
        out |= ((keys >> np.uint64(sb)) & np.uint64(1)) << np.uint64(w - 1 - i)
    return out


# half precision stored as exponent (bits 15..11) | mantissa (10..1) | sign (0)
SIGN_LOW_HALF = [0] + list(range(15, 10, -1)) + list(range(10, 0, -1))


def decode_sign_low_half(v):
    s, e, f = v & 1, (v >> 11) & 0x1F, (v >> 1) & 0x3FF
    if e == 0x1F and f:
        return (0, -f) if s else (4, f)
    if e == 0x1F:
        return (1,) if s else (3,)
    mag = Fraction(f, 1 << 24) if e == 0 else Fraction(1024 + f, 1 << 10) * Fraction(2) ** (e - 15)
    val = -mag if s else mag
    return (2, val, -1 if (s and val == 0) else 0)


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.SIGNED, oracle.FLOAT])
def test_identity_layout_is_the_standard_sort(mode):
    rng = np.random.default_rng(110 + mode)
    for w in (8, 16, 32):
        keys = rng.integers(0, 1 << w, size=500, dtype=np.uint64)
        keys[::5] = keys[0]
        mant = {8: 3, 16: 10, 32: 23}[w]
        for asc in (True, False):
            k, i = oracle.sort_layout(keys, w, mode, list(range(w - 1, -1, -1)), asc=asc)
            rk, ri = oracle.sort(keys, w, mode, asc=asc, mant_bits=mant)
            np.testing.assert_array_equal(i, ri)
            np.testing.assert_array_equal(k, rk)


def test_sign_in_lowest_bit_brute_force():
    rng = np.random.default_rng(120)
    pool = [0, 1, 2, 3, 0x7C00 << 0, (0x1F << 11), (0x1F << 11) | 1, (0x1F << 11) | 2,
            (0x1F << 11) | 3, (15 << 11), (15 << 11) | 1, (15 << 11) | (1 << 1), (16 << 11) | 1,
            (1 << 11), (1 << 11) | 1, 0xFFFF, 0xFFFE]
    pool += [int(x) for x in rng.integers(0, 1 << 16, size=10)]
    for trial in range(300):
        n = int(rng.integers(1, 9))
        v = [pool[int(j)] for j in rng.integers(0, len(pool), size=n)]
        for asc in (True, False):
            want = sorted(range(n), key=lambda j: decode_sign_low_half(v[j]), reverse=not asc)
            k, i = oracle.sort_layout(np.array(v, dtype=np.uint64), 16, oracle.FLOAT,
                                      SIGN_LOW_HALF, asc=asc)
            assert list(i) == want, (trial, asc, v)
            assert list(k) == [v[j] for j in want]


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.SIGNED, oracle.FLOAT])
def test_any_layout_is_the_sort_of_the_reordered_bits(mode):
    rng = np.random.default_rng(130 + mode)
    for w in (8, 16, 32, 64):
        order = [int(x) for x in rng.permutation(w)]
        keys = rng.integers(0, 1 << 63, size=400, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=400, dtype=np.uint64)
        if w < 64:
            keys &= np.uint64((1 << w) - 1)
        keys[::7] = keys[1]
        for asc in (True, False):
            k, i = oracle.sort_layout(keys, w, mode, order, asc=asc)
            _, ri = oracle.sort(to_order_bits(keys, w, order), w, mode, asc=asc,
                                mant_bits=w // 2)
            np.testing.assert_array_equal(i, ri)
            np.testing.assert_array_equal(k, keys[ri])
