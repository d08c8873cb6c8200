"""Independent numeric interpretation of key bit patterns, used to pin the
oracle.  Nothing here reorders bits or flips directions the way bsort does:
it decodes each pattern to the number it denotes (exactly, with Fraction)
and orders by that number, using the special-value rules of Section III-C
of the bsort paper:

* +inf/-inf sit inside their sign's partition, beyond every finite value;
* NaNs sit at the extremities (negative-signed NaNs first, positive-signed
  last when ascending), ordered among themselves by their payload;
* -0 < +0.

The order among NaNs of one sign follows the reading that the inverse
direction used for the negative half applies to all of its lower bits, so
ascending puts -NaN payloads largest-first and +NaN payloads smallest-first.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Callable, List, Sequence


def to_signed(k: int, w: int) -> int:
    """Two's-complement value of a w-bit pattern."""
    return k - (1 << w) if k >> (w - 1) else k


def from_signed(v: int, w: int) -> int:
    return v & ((1 << w) - 1)


def decode_float(k: int, w: int, mant: int, ieee_specials: bool = True):
    """Decode a sign|exponent|mantissa pattern.

    Returns (kind, sign, value) with kind in {"num", "inf", "nan"}; value is
    an exact Fraction for numbers and the payload (mantissa) for NaNs.
    ieee_specials=False decodes the OCP e4m3 ("fn") layout: no infinities,
    and only the all-ones exponent with all-ones mantissa is NaN.
    """
    e_bits = w - 1 - mant
    sign = (k >> (w - 1)) & 1
    e = (k >> mant) & ((1 << e_bits) - 1)
    m = k & ((1 << mant) - 1)
    bias = (1 << (e_bits - 1)) - 1
    e_max = (1 << e_bits) - 1
    if ieee_specials and e == e_max:
        return ("inf", sign, None) if m == 0 else ("nan", sign, m)
    if not ieee_specials and e == e_max and m == (1 << mant) - 1:
        return ("nan", sign, m)
    if e == 0:
        mag = Fraction(m, 1 << mant) * Fraction(2) ** (1 - bias)
    else:
        mag = (1 + Fraction(m, 1 << mant)) * Fraction(2) ** (e - bias)
    return ("num", sign, -mag if sign else mag)


def float_order_key(k: int, w: int, mant: int, ieee_specials: bool = True):
    """Ascending total-order key of a float pattern (see module doc)."""
    kind, sign, val = decode_float(k, w, mant, ieee_specials)
    if kind == "nan":
        return (0, -val, 0) if sign else (4, val, 0)
    if kind == "inf":
        return (1, 0, 0) if sign else (3, 0, 0)
    # numbers: by value, then -0 before +0
    return (2, val, 0 if sign else 1)


def order_key_fn(mode: str, w: int, mant: int = 0,
                 ieee_specials: bool = True) -> Callable[[int], object]:
    if mode == "unsigned":
        return lambda k: k
    if mode == "signed":
        return lambda k: to_signed(k, w)
    if mode == "float":
        return lambda k: float_order_key(k, w, mant, ieee_specials)
    raise ValueError(mode)


def expected_stable(keys: Sequence[int], keyfn: Callable[[int], object],
                    asc: bool) -> List[int]:
    """Stable sort permutation by the numeric order (Python's sort is
    stable, also with reverse=True)."""
    return sorted(range(len(keys)), key=lambda i: keyfn(keys[i]),
                  reverse=not asc)
