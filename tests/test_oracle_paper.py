"""Pins the oracle to the paper's worked examples and proofs.

* Figs. 1-3: every level of the traced recursion (stable flavour), and the
  final row for the paper's literal Lomuto partition (Algorithm 1).
* Section III's proof that one unsigned pass misorders mixed signs.
* Theorem 2's counterexamples [-2.0, 0.0, 0.5] and [0.75, 2.0].
* The mantissa-width switch of Algorithm 5 does not change the result.
"""
import os

import numpy as np
import pytest

import oracle
from numeric_order import from_signed, to_signed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_trace(name):
    meta, rows = {}, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                for tok in line[1:].split():
                    if "=" in tok:
                        k, v = tok.split("=", 1)
                        meta[k] = v
                continue
            r, vals = line.split(":", 1)
            rows[int(r)] = vals.split()
    w = int(meta["w"])
    mode = {"unsigned": oracle.UNSIGNED, "signed": oracle.SIGNED,
            "float": oracle.FLOAT}[meta["mode"]]
    if meta["encoding"] == "binary":
        conv = lambda s: int(s, 2)
    elif mode == oracle.SIGNED:
        conv = lambda s: from_signed(int(s), w)
    else:
        conv = lambda s: int(s)
    pats = {r: [conv(v) for v in vals] for r, vals in rows.items()}
    return (w, mode, bool(int(meta["asc"])), int(meta["mant_bits"]), pats)


TRACES = ["fig1_unsigned_trace.txt", "fig2_signed_desc_trace.txt",
          "fig3_toyfloat_trace.txt"]


@pytest.mark.parametrize("name", TRACES)
def test_trace_every_level_stable(name):
    w, mode, asc, mant, rows = load_trace(name)
    keys, idx, snap, snap_i = oracle.sort(rows[0], w, mode, asc=asc, mant_bits=mant,
                                          snapshots=True)
    for r, expect in rows.items():
        assert snap[r].tolist() == expect, f"{name}: row {r}"
    # the payload moved with the keys at every level
    inp = np.array(rows[0], dtype=np.uint64)
    for r in range(w + 1):
        assert (inp[snap_i[r]] == snap[r]).all()
    assert keys.tolist() == snap[w].tolist()


@pytest.mark.parametrize("name", TRACES)
def test_trace_final_row_lomuto(name):
    """The paper's own swap loop reaches the same final keys."""
    w, mode, asc, mant, rows = load_trace(name)
    keys, _ = oracle.sort(rows[0], w, mode, asc=asc, mant_bits=mant,
                          flavour=oracle.LOMUTO)
    last = max(rows)
    assert keys.tolist() == rows[last]


def test_fig1_lomuto_level1_differs_from_trace():
    """Fig. 1's level-1 row is a stable split; the literal swap loop
    permutes the second side (this is why indices follow the stable run)."""
    _, _, snap, _ = oracle.sort([5, 7, 1, 6, 3, 4, 0], 3, oracle.UNSIGNED,
                                flavour=oracle.LOMUTO, snapshots=True)
    assert snap[1].tolist() == [1, 3, 0, 6, 7, 4, 5]


def test_signed_msb_failure_proof():
    """Section III: a plain unsigned pass puts x < 0 after y >= 0."""
    w = 8
    x, y = from_signed(-3, w), from_signed(2, w)
    keys, _ = oracle.sort([x, y], w, oracle.UNSIGNED, asc=True)
    assert [to_signed(int(k), w) for k in keys] == [2, -3]
    keys, _ = oracle.sort([x, y], w, oracle.SIGNED, asc=True)
    assert [to_signed(int(k), w) for k in keys] == [-3, 2]


def f32_bits(vals):
    return np.array(vals, dtype=np.float32).view(np.uint32).astype(np.uint64)


@pytest.mark.parametrize("vals", [[-2.0, 0.0, 0.5], [0.75, 2.0], [0.5, 0.0, -2.0],
                                  [2.0, 0.75]])
def test_theorem2_counterexamples_sorted(vals):
    for asc in (True, False):
        keys, _ = oracle.sort(f32_bits(vals), 32, oracle.FLOAT, asc=asc, mant_bits=23)
        got = keys.astype(np.uint32).view(np.float32).tolist()
        assert got == sorted(vals, reverse=not asc)


def test_fig3_values():
    _, _, _, _, rows = load_trace("fig3_toyfloat_trace.txt")
    keys, _ = oracle.sort(rows[0], 6, oracle.FLOAT, asc=True, mant_bits=2)
    # -inf, -2.5, 1.25, 1.75 in the 1/3/2 layout with bias 3
    assert keys.tolist() == [0b111100, 0b110001, 0b001101, 0b001111]


@pytest.mark.parametrize("w,mant_list", [(6, range(0, 5)), (8, range(0, 7)),
                                         (16, [0, 2, 7, 10, 14])])
def test_mantissa_width_does_not_change_result(w, mant_list):
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 1 << w, size=300, dtype=np.uint64)
    for asc in (True, False):
        outs = [oracle.sort(keys, w, oracle.FLOAT, asc=asc, mant_bits=m) for m in mant_list]
        for k, i in outs[1:]:
            assert (k == outs[0][0]).all() and (i == outs[0][1]).all()


def test_argument_validation():
    with pytest.raises(ValueError):
        oracle.sort([1 << 8], 8, oracle.UNSIGNED)  # pattern wider than w
    with pytest.raises(ValueError):
        oracle.sort([1], 8, oracle.FLOAT, mant_bits=7)  # no exponent bit left
    with pytest.raises(ValueError):
        oracle.sort([1], 65, oracle.UNSIGNED)


@pytest.mark.parametrize("n", [0, 1])
def test_trivial_sizes(n):
    keys, idx = oracle.sort(list(range(n)), 8, oracle.SIGNED, asc=False)
    assert keys.tolist() == list(range(n)) and idx.tolist() == list(range(n))
