"""Exhaustive and large random pins of the oracle against numpy's own
numeric interpretation of the bit patterns (library decoders and numpy's
stable argsort), not against any bit-flipping formula.

* every 8-bit pattern (u8, i8, e4m3, e5m2) and every 16-bit pattern (u16,
  i16, fp16, bf16), shuffled with duplicates, in both directions;
* random 32- and 64-bit inputs with signed zeros, subnormals and
  infinities mixed in;
* NaN placement at the extremities (Section III-C).
"""
import numpy as np
import pytest

import oracle
from numeric_order import decode_float


def _shuffled_all(w, seed):
    rng = np.random.default_rng(seed)
    pats = np.arange(1 << w, dtype=np.uint64)
    dup = rng.integers(0, 1 << w, size=(1 << w) // 4, dtype=np.uint64)
    return rng.permutation(np.concatenate([pats, dup]))


def _stable_ref_int(vals, asc):
    v = vals.astype(np.int64)
    return np.argsort(v if asc else -v, kind="stable")


@pytest.mark.parametrize("dtype,npdt", [("u8", np.uint8), ("i8", np.int8),
                                        ("u16", np.uint16), ("i16", np.int16)])
@pytest.mark.parametrize("asc", [True, False])
def test_exhaustive_integers(dtype, npdt, asc):
    w = oracle.DTYPES[dtype][0]
    pats = _shuffled_all(w, 1)
    vals = pats.astype(np.dtype(f"u{w // 8}")).view(npdt)
    keys, idx = oracle.sort_dtype(pats, dtype, asc=asc)
    ref = _stable_ref_int(vals, asc)
    assert (idx == ref).all()
    assert (keys == pats[ref]).all()


def _float_values(pats, dtype):
    """numpy's (or, for fp8, an exact) decoding of the patterns."""
    if dtype == "f16":
        return pats.astype(np.uint16).view(np.float16).astype(np.float64)
    if dtype == "bf16":
        return (pats.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    if dtype == "f32":
        return pats.astype(np.uint32).view(np.float32).astype(np.float64)
    if dtype == "f64":
        return pats.view(np.float64)
    mant = oracle.DTYPES[dtype][2]
    ieee = dtype != "e4m3"
    out = np.empty(pats.size, dtype=np.float64)
    for i, p in enumerate(pats.tolist()):
        kind, sign, val = decode_float(p, 8, mant, ieee_specials=ieee)
        out[i] = (np.nan if kind == "nan" else
                  (-np.inf if sign else np.inf) if kind == "inf" else float(val))
    return out


def _stable_ref_float(pats, vals, w, asc):
    """Stable order by value with -0 < +0 for non-NaN entries (numpy's
    lexsort is stable); NaNs are checked separately."""
    sign = ((pats >> np.uint64(w - 1)) & np.uint64(1)).astype(np.int64)
    if asc:
        return np.lexsort((1 - sign, vals))
    return np.lexsort((sign, -vals))


def _check_float_output(pats, keys, idx, vals_fn, w, asc):
    assert (keys == pats[idx]).all()
    assert np.array_equal(np.sort(idx), np.arange(pats.size))
    vals = vals_fn(keys)
    nan = np.isnan(vals)
    sign = (keys >> np.uint64(w - 1)) & np.uint64(1)
    lo_nan = nan & (sign == (1 if asc else 0))   # NaNs that lead the output
    hi_nan = nan & (sign == (0 if asc else 1))   # NaNs that close it
    n_lo, n_hi = int(lo_nan.sum()), int(hi_nan.sum())
    assert lo_nan[:n_lo].all() and hi_nan[keys.size - n_hi:].all()
    mid = slice(n_lo, keys.size - n_hi)
    # numbers: ordered by value, -0 before +0, stable among equal patterns
    pm, im = pats[idx[mid]], idx[mid]
    order = _stable_ref_float(pm, vals_fn(pm), w, asc)
    assert (order == np.arange(pm.size)).all()
    # NaN runs: ordered by payload, largest first in the leading run and
    # smallest first in the closing one (in both directions: descending is
    # the exact reverse of ascending), stable among equal payloads
    mbits = np.uint64((1 << (w - 1)) - 1)
    for sl, desc_payload in ((slice(0, n_lo), True), (slice(keys.size - n_hi, keys.size), False)):
        pay = (keys[sl] & mbits).astype(np.float64)
        ref = np.argsort(-pay if desc_payload else pay, kind="stable")
        assert (ref == np.arange(pay.size)).all()
        ii = idx[sl]
        same = keys[sl][1:] == keys[sl][:-1]
        assert (ii[1:][same] > ii[:-1][same]).all()


@pytest.mark.parametrize("dtype", ["e4m3", "e5m2", "f16", "bf16"])
@pytest.mark.parametrize("asc", [True, False])
def test_exhaustive_floats(dtype, asc):
    w = oracle.DTYPES[dtype][0]
    pats = _shuffled_all(w, 2)
    keys, idx = oracle.sort_dtype(pats, dtype, asc=asc)
    _check_float_output(pats, keys, idx, lambda p: _float_values(p, dtype), w, asc)
    # the exhaustive set pins the special-value rules directly
    vals = _float_values(keys, dtype)
    fin = vals[~np.isnan(vals)]
    if asc:
        assert (fin[1:] >= fin[:-1]).all()
    else:
        assert (fin[1:] <= fin[:-1]).all()


def _specials(rng, n, w, npflt):
    bits = rng.standard_normal(n).astype(npflt).view(np.dtype(f"u{w // 8}")).astype(np.uint64)
    m = n // 50
    pos = rng.choice(n, size=4 * m, replace=False)
    one = np.uint64(1)
    sign = one << np.uint64(w - 1)
    mant = {32: 23, 64: 52}[w]
    expo_all = ((one << np.uint64(w - 1 - mant)) - one) << np.uint64(mant)
    bits[pos[:m]] = np.where(rng.integers(0, 2, m) == 1, sign, np.uint64(0))        # +-0
    sub = rng.integers(1, 1 << mant, size=m, dtype=np.uint64)
    bits[pos[m:2 * m]] = sub | np.where(rng.integers(0, 2, m) == 1, sign, np.uint64(0))  # subnormals
    bits[pos[2 * m:3 * m]] = expo_all | np.where(rng.integers(0, 2, m) == 1, sign, np.uint64(0))  # +-inf
    bits[pos[3 * m:]] = bits[rng.choice(n, size=m)]                                  # duplicates
    return bits


@pytest.mark.parametrize("dtype,npflt", [("f32", np.float32), ("f64", np.float64)])
@pytest.mark.parametrize("asc", [True, False])
def test_random_wide_floats(dtype, npflt, asc):
    w = oracle.DTYPES[dtype][0]
    rng = np.random.default_rng(3)
    pats = _specials(rng, 20000, w, npflt)
    keys, idx = oracle.sort_dtype(pats, dtype, asc=asc)
    _check_float_output(pats, keys, idx, lambda p: _float_values(p, dtype), w, asc)


def test_nan_patterns_wide():
    rng = np.random.default_rng(4)
    for dtype, npflt in (("f32", np.float32), ("f64", np.float64)):
        w = oracle.DTYPES[dtype][0]
        pats = _specials(rng, 3000, w, npflt)
        mant = oracle.DTYPES[dtype][2]
        one = np.uint64(1)
        expo_all = ((one << np.uint64(w - 1 - mant)) - one) << np.uint64(mant)
        nan_pos = rng.choice(pats.size, 60, replace=False)
        payload = rng.integers(1, 1 << min(mant, 20), size=60, dtype=np.uint64)
        sgn = np.where(rng.integers(0, 2, 60) == 1, one << np.uint64(w - 1), np.uint64(0))
        pats[nan_pos] = expo_all | payload | sgn
        pats[nan_pos[:10]] = pats[nan_pos[10]]  # duplicate NaNs
        for asc in (True, False):
            keys, idx = oracle.sort_dtype(pats, dtype, asc=asc)
            _check_float_output(pats, keys, idx, lambda p: _float_values(p, dtype), w, asc)


@pytest.mark.parametrize("dtype,npdt", [("u32", np.uint32), ("i32", np.int32),
                                        ("u64", np.uint64), ("i64", np.int64)])
@pytest.mark.parametrize("asc", [True, False])
def test_random_wide_integers(dtype, npdt, asc):
    w = oracle.DTYPES[dtype][0]
    rng = np.random.default_rng(9)
    n = 30000
    raw = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    pats = raw >> np.uint64(64 - w) if w < 64 else raw
    pats[::5] = pats[1::5][: pats[::5].size]  # duplicates
    vals = pats.astype(np.dtype(f"u{w // 8}")).view(npdt)
    keys, idx = oracle.sort_dtype(pats, dtype, asc=asc)
    if asc:
        ref = np.argsort(vals, kind="stable")
    else:
        # stable descending: rank values from the top, ties in input order
        uniq, inv = np.unique(vals, return_inverse=True)
        ref = np.lexsort((np.arange(n), uniq.size - 1 - inv))
    assert (idx == ref).all()
    assert (keys == pats[ref]).all()
