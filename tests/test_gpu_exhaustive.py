"""GPU parity on every bit pattern and on NaN-heavy floats (the special
values of Section III-C):

  - all 2^16 patterns of f16, bf16, i16 and u16 and all 2^8 patterns of the
    8-bit dtypes, each with a quarter more seeded repeats, shuffled, through
    the typed entry points, both directions, default and plain mode, with
    and without indices;
  - f32 and f64 patterns uniform over all bits with a further 10% NaNs
    (random payloads, both signs) at 200003 keys.

Each against the oracle element by element: keys bit-exact, stable indices
exact."""
import numpy as np
import pytest

from paper_2603_08929_amd import _lib
from paper_2603_08929_amd import workloads as W

pytestmark = pytest.mark.gpu

gpu_util = pytest.importorskip("gpu_util")


def _check(got_k, got_i, exp_k, exp_i, label):
    bad = np.nonzero(got_k != exp_k)[0]
    assert bad.size == 0, (f"{label}: {bad.size} key mismatches, first at {bad[:5]}: "
                           f"got {got_k[bad[:5]]} expected {exp_k[bad[:5]]}")
    if got_i is not None:
        bad = np.nonzero(got_i != exp_i)[0]
        assert bad.size == 0, (f"{label}: {bad.size} index mismatches, first at {bad[:5]}: "
                               f"got {got_i[bad[:5]]} expected {exp_i[bad[:5]]}")


@pytest.mark.parametrize("name", ["f16", "bf16", "i16", "u16", "u8", "i8", "e4m3", "e5m2"])
@pytest.mark.parametrize("asc", [True, False])
def test_every_pattern(name, asc):
    bits = W.all_patterns(name, 0.25, seed=len(name) + (0 if asc else 100))
    exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
    for flags in (0, _lib.PLAIN):
        for idx in ("u32", None):
            label = f"{name} all patterns n={bits.size} asc={asc} flags={flags} idx={idx}"
            print(label, flush=True)
            k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
            _check(k, i, exp_k, exp_i, label)


@pytest.mark.parametrize("name", ["f32", "f64"])
@pytest.mark.parametrize("asc", [True, False])
def test_nan_heavy_uniform(name, asc):
    n = 200003
    bits = W.plant_nans(W.uniform_bits(name, n, 61), name, 0.10, 62)
    exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
    for flags, idx in ((0, "u32"), (_lib.PLAIN, "i64"), (_lib.NO_SKIP, None)):
        label = f"{name} NaN-heavy n={n} asc={asc} flags={flags} idx={idx}"
        print(label, flush=True)
        k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
        _check(k, i, exp_k, exp_i, label)
