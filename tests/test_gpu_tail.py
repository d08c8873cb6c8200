"""GPU parity on inputs whose parts stay larger than the LDS finish for many
levels, so that live levels run in the tail launch (the levels past the
depth picked from n, walked by one kernel with grid barriers): log-uniform
integers and one-hot patterns peel one magnitude class off the big part per
level.  Against the oracle element by element, single and segmented, both
directions, 32- and 64-bit indices."""
import numpy as np
import pytest

from paper_2603_08929_amd import _lib

pytestmark = pytest.mark.gpu

gpu_util = pytest.importorskip("gpu_util")


def log_uniform(name, n, seed):
    """(1 << r) + random r low bits, r uniform over the key width: every
    magnitude class equally likely."""
    w = {"u32": 32, "i32": 32, "u64": 64, "f32": 32}[name]
    rng = np.random.default_rng(seed)
    r = rng.integers(0, w - 1, size=n, dtype=np.uint64)
    low = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    v = (np.uint64(1) << r) | (low & ((np.uint64(1) << r) - np.uint64(1)))
    raw = {32: np.uint32, 64: np.uint64}[w]
    return v.astype(raw)


def one_hot(name, n, seed):
    w = {"u32": 32, "u64": 64}[name]
    rng = np.random.default_rng(seed)
    r = rng.integers(0, w, size=n, dtype=np.uint64)
    return (np.uint64(1) << r).astype({32: np.uint32, 64: np.uint64}[w])


def _check(got_k, got_i, exp_k, exp_i, label):
    bad = np.nonzero(got_k != exp_k)[0]
    assert bad.size == 0, f"{label}: {bad.size} key mismatches, first at {bad[:5]}"
    if got_i is not None:
        bad = np.nonzero(got_i != exp_i)[0]
        assert bad.size == 0, f"{label}: {bad.size} index mismatches, first at {bad[:5]}"


@pytest.mark.parametrize("name,gen", [("u32", log_uniform), ("i32", log_uniform),
                                      ("f32", log_uniform), ("u64", log_uniform),
                                      ("u32", one_hot), ("u64", one_hot)])
@pytest.mark.parametrize("asc", [True, False])
def test_many_live_levels(name, gen, asc):
    for n in (200003, 1 << 20):
        bits = gen(name, n, seed=n % 1000 + 3)
        exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
        for flags, idx in ((0, "u32"), (_lib.NO_SKIP, "i64"), (0, None)):
            label = f"{gen.__name__} {name} n={n} asc={asc} flags={flags} idx={idx}"
            print(label, flush=True)
            k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
            _check(k, i, exp_k, exp_i, label)


@pytest.mark.parametrize("asc", [True, False])
def test_many_live_levels_segmented(asc):
    lengths = [150001, 3, 0, 70000, 1 << 18]
    n = sum(lengths)
    bits = log_uniform("u32", n, 77)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    label = f"segmented log-uniform u32 asc={asc}"
    print(label, flush=True)
    k, i, _ = gpu_util.gpu_segmented("u32", bits, lengths, asc, 0, "u32")
    for s in range(len(lengths)):
        a, b = offs[s], offs[s + 1]
        exp_k, exp_i = gpu_util.oracle_sort("u32", bits[a:b], asc)
        _check(k[a:b], i[a:b], exp_k, exp_i, f"{label} seg={s}")
