"""GPU check of the per-level property of Theorem 3's induction (P_E(k):
after the k most significant bits, the array is ordered by its k-bit
prefix).  bsort_levels stops the device sort after k global levels; its
output must

  - equal the oracle's breadth-first snapshot after k bits, element by
    element (keys bit-exact, indices exact), and
  - independently of the oracle: be ordered by the top k bits of the order
    key (non-increasing when descending), keys with an equal prefix in input
    order, and keys[j] == input[idx[j]] with idx a permutation.

Every k from 0 (the input, identity indices) to w (the full sort).  The
prefix-order checker itself is checked on the CPU against the oracle's
snapshots, with a planted mistake that it must catch."""
import numpy as np
import pytest

from paper_2603_08929_amd import _lib
from paper_2603_08929_amd.workloads import DTYPES, mixed_bits

gpu_util = pytest.importorskip("gpu_util")


def order_key(name: str, bits: np.ndarray) -> np.ndarray:
    """The unsigned key whose natural order is the dtype's total order:
    the sign bit inverted for integers; for floats every bit of a negative
    pattern inverted, the sign bit of a positive one set."""
    w, fam = DTYPES[name][0], DTYPES[name][1]
    k = bits.astype(np.uint64)
    mask = np.uint64((1 << w) - 1) if w < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    sign = np.uint64(1 << (w - 1))
    if fam == "I":
        return k ^ sign
    if fam == "F":
        neg = (k & sign) != 0
        return np.where(neg, ~k & mask, k | sign)
    return k


def check_prefix_order(name, src, got_k, got_i, levels, asc, label):
    n = src.size
    w = DTYPES[name][0]
    if got_i is not None:
        assert np.array_equal(np.sort(got_i), np.arange(n)), f"{label}: indices not a permutation"
        assert np.array_equal(got_k, src[got_i]), f"{label}: keys do not follow the indices"
    if n < 2 or got_i is None:
        return
    if levels == 0:
        assert np.array_equal(got_i, np.arange(n)), f"{label}: level 0 moved keys"
        return
    pre = order_key(name, got_k) >> np.uint64(w - levels)
    lo, hi = pre[:-1], pre[1:]
    bad = np.nonzero(hi < lo if asc else hi > lo)[0]
    tie = lo == hi
    assert bad.size == 0, f"{label}: prefix order broken at {bad[:5]}"
    unstable = np.nonzero(tie & (np.diff(got_i) <= 0))[0]
    assert unstable.size == 0, f"{label}: equal prefixes out of input order at {unstable[:5]}"


def _check_equal(got_k, got_i, exp_k, exp_i, label):
    bad = np.nonzero(got_k != exp_k)[0]
    assert bad.size == 0, (f"{label}: {bad.size} key mismatches, first at {bad[:5]}: "
                           f"got {got_k[bad[:5]]} expected {exp_k[bad[:5]]}")
    if got_i is not None:
        bad = np.nonzero(got_i != exp_i)[0]
        assert bad.size == 0, (f"{label}: {bad.size} index mismatches, first at {bad[:5]}: "
                               f"got {got_i[bad[:5]]} expected {exp_i[bad[:5]]}")


@pytest.mark.parametrize("name", ["u8", "i16", "e5m2", "bf16", "f32", "i64"])
@pytest.mark.parametrize("asc", [True, False])
def test_checker_on_oracle_snapshots(name, asc):
    """CPU: every oracle snapshot row passes the prefix-order check at its
    level; a row with two keys of different prefixes swapped fails it."""
    import oracle
    n = 3001
    w, mode, mant = oracle.DTYPES[name]
    raw = DTYPES[name][2]
    bits = mixed_bits(name, n, seed=13 + w)
    _, _, snap, snap_i = oracle.sort(bits.astype(np.uint64), w, mode, asc=asc, mant_bits=mant,
                                     snapshots=True)
    for lv in range(w + 1):
        check_prefix_order(name, bits, snap[lv].astype(raw), snap_i[lv], lv, asc, f"lv={lv}")
    for lv in (1, w // 2, w):
        k, i = snap[lv].astype(raw), snap_i[lv].copy()
        pre = order_key(name, k) >> np.uint64(w - lv)
        j = int(np.nonzero(pre[1:] != pre[:-1])[0][0])
        k[[j, j + 1]] = k[[j + 1, j]]
        i[[j, j + 1]] = i[[j + 1, j]]
        with pytest.raises(AssertionError):
            check_prefix_order(name, bits, k, i, lv, asc, f"planted lv={lv}")
        # two keys of one prefix out of input order
        k, i = snap[lv].astype(raw), snap_i[lv].copy()
        pre = order_key(name, k) >> np.uint64(w - lv)
        j = int(np.nonzero(pre[1:] == pre[:-1])[0][0])
        k[[j, j + 1]] = k[[j + 1, j]]
        i[[j, j + 1]] = i[[j + 1, j]]
        with pytest.raises(AssertionError):
            check_prefix_order(name, bits, k, i, lv, asc, f"planted tie lv={lv}")


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["u32", "i32", "f32", "f16", "u64"])
@pytest.mark.parametrize("asc", [True, False])
def test_every_level_matches_the_oracle_snapshot(name, asc):
    n = 200003
    w = DTYPES[name][0]
    bits = mixed_bits(name, n, seed=4242 + w)
    snap, snap_i = gpu_util.oracle_snapshots(name, bits, asc)
    for lv in range(w + 1):
        idx_kinds = ("u32", "i64", None) if lv in (1, w // 2, w - 1) else ("u32",)
        for idx in idx_kinds:
            label = f"{name} n={n} asc={asc} levels={lv} idx={idx}"
            print(label, flush=True)
            k, i = gpu_util.gpu_levels(name, bits, lv, asc, idx)
            _check_equal(k, i, snap[lv], snap_i[lv], label)
            check_prefix_order(name, bits, k, i, lv, asc, label)


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["u8", "u16", "i8", "i16", "i64", "e4m3", "e5m2", "bf16",
                                  "f64"])
@pytest.mark.parametrize("asc", [True, False])
def test_every_level_other_dtypes(name, asc):
    n = 30011
    w = DTYPES[name][0]
    bits = mixed_bits(name, n, seed=77 + w)
    snap, snap_i = gpu_util.oracle_snapshots(name, bits, asc)
    for lv in range(w + 1):
        label = f"{name} n={n} asc={asc} levels={lv}"
        print(label, flush=True)
        k, i = gpu_util.gpu_levels(name, bits, lv, asc, "u32")
        _check_equal(k, i, snap[lv], snap_i[lv], label)
        check_prefix_order(name, bits, k, i, lv, asc, label)


@pytest.mark.gpu
@pytest.mark.parametrize("asc", [True, False])
def test_levels_segmented(asc):
    lengths = [0, 1, 4999, 70001, 2, 0, 125000]
    n = sum(lengths)
    name = "f32"
    bits = mixed_bits(name, n, seed=91)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    snaps = [gpu_util.oracle_snapshots(name, bits[offs[s]:offs[s + 1]], asc)
             for s in range(len(lengths))]
    for lv in (0, 1, 2, 9, 17, 31, 32):
        label = f"segmented f32 asc={asc} levels={lv}"
        print(label, flush=True)
        k, i = gpu_util.gpu_levels(name, bits, lv, asc, "u32", lengths=lengths)
        for s in range(len(lengths)):
            a, b = offs[s], offs[s + 1]
            _check_equal(k[a:b], i[a:b], snaps[s][0][lv], snaps[s][1][lv], f"{label} seg={s}")
            check_prefix_order(name, bits[a:b], k[a:b], i[a:b], lv, asc, f"{label} seg={s}")


@pytest.mark.gpu
def test_full_level_count_is_the_full_sort():
    bits = mixed_bits("u32", 100003, seed=5)
    exp_k, exp_i = gpu_util.oracle_sort("u32", bits, True)
    k, i = gpu_util.gpu_levels("u32", bits, 32, True, "u32")
    _check_equal(k, i, exp_k, exp_i, "levels=32")
    k2, i2 = gpu_util.gpu_sort("u32", bits, True, _lib.PLAIN, "u32")
    _check_equal(k, i, k2, i2, "levels=32 vs bsort_u32 PLAIN")
