"""Brute force: every permutation of small multisets, in every key mode and
direction, against the numeric order of the decoded values (Section III's
ordering rules; see numeric_order.py).  Keys must come out in that order and
the payload must be the stable permutation (equal patterns keep input order
in both directions).  Also pins the per-level invariant P_E(k) of Theorem 3
and the quickselect entry point."""
import itertools

import numpy as np
import pytest

import oracle
from numeric_order import expected_stable, from_signed, order_key_fn

# (name, w, mode, mant, multisets of patterns)
CASES = [
    ("u3", 3, oracle.UNSIGNED, 0, [[0, 7, 3, 3, 5, 1, 0], [2, 2, 2, 5, 1, 6]]),
    ("u4", 4, oracle.UNSIGNED, 0, [[15, 8, 7, 0, 8, 1]]),
    ("i4", 4, oracle.SIGNED, 0, [[from_signed(v, 4) for v in (-8, -1, 3, -7, 2, 6, 3)],
                                 [from_signed(v, 4) for v in (7, -8, 0, -1, 0, 1)]]),
    ("i3", 3, oracle.SIGNED, 0, [[from_signed(v, 3) for v in (-4, 3, -1, 0, 0, 1, -4)]]),
    # 6-bit toy float of Fig. 3 (1/3/2): -inf, -2.5, -0, +0, subnormal, 1.75,
    # +inf, NaNs of both signs with different payloads, duplicates
    ("toy6", 6, oracle.FLOAT, 2, [[0b111100, 0b110001, 0b100000, 0b000000, 0b000001,
                                   0b001111, 0b011100],
                                  [0b111101, 0b111111, 0b011110, 0b011101, 0b100000,
                                   0b000000, 0b100000]]),
    ("toy5", 5, oracle.FLOAT, 1, [[0b11100, 0b11101, 0b01101, 0b00001, 0b10001, 0b00000,
                                   0b10000]]),
]


@pytest.mark.parametrize("name,w,mode,mant,multisets", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("asc", [True, False])
def test_all_permutations(name, w, mode, mant, multisets, asc):
    mname = {oracle.UNSIGNED: "unsigned", oracle.SIGNED: "signed",
             oracle.FLOAT: "float"}[mode]
    keyfn = order_key_fn(mname, w, mant)
    for ms in multisets:
        seen = set()
        for perm in itertools.permutations(range(len(ms))):
            arr = [ms[p] for p in perm]
            t = tuple(arr)
            if t in seen:
                continue
            seen.add(t)
            exp_idx = expected_stable(arr, keyfn, asc)
            for flavour in (oracle.STABLE, oracle.LOMUTO):
                keys, idx = oracle.sort(arr, w, mode, asc=asc, mant_bits=mant,
                                        flavour=flavour)
                assert keys.tolist() == [arr[i] for i in exp_idx], (name, arr, flavour)
                if flavour == oracle.STABLE:
                    assert idx.tolist() == exp_idx, (name, arr)


@pytest.mark.parametrize("name,w,mode,mant,multisets", CASES, ids=[c[0] for c in CASES])
def test_level_invariant(name, w, mode, mant, multisets):
    """Theorem 3's P_E(k): after the partitions on the top d bits, the array
    is ordered by the value those d bits denote (the key with its lower bits
    cleared), and inside a run of equal d-bit prefixes the input order is
    kept (stable flavour)."""
    mname = {oracle.UNSIGNED: "unsigned", oracle.SIGNED: "signed",
             oracle.FLOAT: "float"}[mode]
    keyfn = order_key_fn(mname, w, mant)
    rng = np.random.default_rng(5)
    for ms in multisets:
        for _ in range(30):
            arr = [ms[i] for i in rng.permutation(len(ms))]
            for asc in (True, False):
                _, _, snap, snap_i = oracle.sort(arr, w, mode, asc=asc, mant_bits=mant,
                                                 snapshots=True)
                for d in range(1, w + 1):
                    low = w - d
                    pre = [(int(k) >> low) << low for k in snap[d]]
                    ks = [keyfn(p) for p in pre]
                    for i in range(len(arr) - 1):
                        if asc:
                            assert ks[i] <= ks[i + 1], (name, arr, d)
                        else:
                            assert ks[i] >= ks[i + 1], (name, arr, d)
                        if pre[i] == pre[i + 1]:
                            assert snap_i[d][i] < snap_i[d][i + 1], (name, arr, d)


@pytest.mark.parametrize("dtype", ["u8", "i16", "f32", "f64", "i64", "bf16"])
def test_select_matches_sort(dtype):
    w, mode, mant = oracle.DTYPES[dtype]
    rng = np.random.default_rng(7)
    n = 501
    keys = rng.integers(0, 1 << min(w, 63), size=n, dtype=np.uint64)
    if w == 64:
        keys |= rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63)
    keys[::7] = keys[3]  # duplicates
    mname = {oracle.UNSIGNED: "unsigned", oracle.SIGNED: "signed", oracle.FLOAT: "float"}[mode]
    keyfn = order_key_fn(mname, w, mant)
    kl = [int(k) for k in keys]
    for asc in (True, False):
        sk, si = oracle.sort(keys, w, mode, asc=asc, mant_bits=mant)
        # the numeric order written out independently of the oracle
        perm = expected_stable(kl, keyfn, asc)
        for j in [0, 1, n // 2, n - 2, n - 1] + rng.integers(0, n, 10).tolist():
            k, i = oracle.select(keys, w, mode, asc, int(j), mant_bits=mant)
            assert k == int(sk[j]) and i == int(si[j])
            assert i == perm[j] and k == kl[perm[j]]


def test_permute_backward():
    """Pinned by two properties of the derivative of values = x[idx]: the
    result gathered by idx gives back grad_out, and a central finite
    difference of L(x) = sum(W * x[idx]) reproduces it."""
    rng = np.random.default_rng(3)
    rows, cols = 4, 9
    g = rng.standard_normal((rows, cols))
    idx = np.stack([rng.permutation(cols) for _ in range(rows)])
    out = oracle.permute_backward(g, idx)
    assert (np.take_along_axis(out, idx, axis=1) == g).all()
    x = rng.standard_normal((rows, cols))
    loss = lambda x: float((g * np.take_along_axis(x, idx, axis=1)).sum())
    h = 1e-6
    for r in range(rows):
        for i in range(cols):
            e = np.zeros_like(x)
            e[r, i] = h
            fd = (loss(x + e) - loss(x - e)) / (2 * h)
            assert abs(fd - out[r, i]) < 1e-6
    with pytest.raises(ValueError):
        oracle.permute_backward(g, np.zeros((rows, cols), dtype=np.int64))
