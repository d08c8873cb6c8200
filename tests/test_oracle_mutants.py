"""The pins catch plausible mistakes: each deliberately wrong build of the
oracle (compiled from the same source with -DBSO_MUTANT=k, on the CPU) must
fail at least one of the paper-derived checks that the real oracle passes.

  1  literal Algorithm 4: negative half sorted with asc
  2  no direction flip on the sign pass (treats signed keys as unsigned)
  3  float fields in the order sign, mantissa, exponent (Theorem 2 case 2)
  4  exponent before sign (Theorem 2 case 1)
  5  mantissa first (Theorem 2 case 1)
  8  recursion stops one bit early
  9  signed halves sorted in the inverse direction
"""
import numpy as np
import pytest

import oracle
from test_oracle_paper import load_trace, TRACES, f32_bits


def paper_checks(mutant):
    """Names of the paper-derived checks that the given build fails."""
    failed = []
    for name in TRACES:
        w, mode, asc, mant, rows = load_trace(name)
        keys, _ = oracle.sort(rows[0], w, mode, asc=asc, mant_bits=mant, mutant=mutant)
        if keys.tolist() != rows[max(rows)]:
            failed.append(name)
    for vals in ([-2.0, 0.0, 0.5], [0.75, 2.0]):
        for asc in (True, False):
            keys, _ = oracle.sort(f32_bits(vals), 32, oracle.FLOAT, asc=asc, mant_bits=23,
                                  mutant=mutant)
            if keys.astype(np.uint32).view(np.float32).tolist() != sorted(vals, reverse=not asc):
                failed.append(f"theorem2 {vals} asc={asc}")
    # exhaustive int8 / fp16 numeric order
    pats = np.arange(256, dtype=np.uint64)
    vals = pats.astype(np.uint8).view(np.int8)
    keys, _ = oracle.sort(pats, 8, oracle.SIGNED, asc=True, mutant=mutant)
    if not (keys == pats[np.argsort(vals, kind="stable")]).all():
        failed.append("exhaustive i8")
    pats = np.arange(1 << 16, dtype=np.uint64)
    keys, _ = oracle.sort(pats, 16, oracle.FLOAT, asc=True, mant_bits=10, mutant=mutant)
    v = keys.astype(np.uint16).view(np.float16).astype(np.float64)
    v = v[~np.isnan(v)]
    if not (v[1:] >= v[:-1]).all():
        failed.append("exhaustive f16")
    return failed


def test_real_oracle_passes_all():
    assert paper_checks(0) == []


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 8, 9])
def test_mutant_is_caught(mutant):
    failed = paper_checks(mutant)
    assert failed, f"mutant {mutant} slipped past every paper check"
