"""GPU parity: every typed entry point, both directions, every flag
combination, keys-only and with 32/64-bit indices, against the oracle
element by element (bit-exact keys, exact stable indices).  Sizes span the
empty, single and tiny cases, one tile (4096 keys for 8/16/32-bit keys, 2048
for 64-bit), the LDS-finish threshold (4096) and several tiles with ragged
tails."""
import numpy as np
import pytest

from paper_2603_08929_amd import _lib
from paper_2603_08929_amd.workloads import mixed_bits, presorted_u32, heavy_duplicates_u32

pytestmark = pytest.mark.gpu

gpu_util = pytest.importorskip("gpu_util")

NAMES = ["u8", "u16", "u32", "u64", "i8", "i16", "i32", "i64", "e4m3", "e5m2", "f16",
         "bf16", "f32", "f64"]
SMALL = [0, 1, 2, 3, 63, 64, 65, 2047, 2049, 4095, 4096, 4097, 8193, 30011]
FLAGS = [0, _lib.NO_SKIP, _lib.NO_FINISH, _lib.PLAIN]


def _check(name, bits, asc, got_k, got_i, exp_k, exp_i, label):
    assert got_k.dtype == exp_k.dtype
    bad = np.nonzero(got_k != exp_k)[0]
    assert bad.size == 0, (f"{label}: {bad.size} key mismatches, first at {bad[:5]}: "
                           f"got {got_k[bad[:5]]} expected {exp_k[bad[:5]]}")
    if got_i is not None:
        bad = np.nonzero(got_i != exp_i)[0]
        assert bad.size == 0, (f"{label}: {bad.size} index mismatches, first at {bad[:5]}: "
                               f"got {got_i[bad[:5]]} expected {exp_i[bad[:5]]}")


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("asc", [True, False])
def test_small_sizes_all_flags(name, asc):
    for n in SMALL:
        bits = mixed_bits(name, n, seed=n + 17)
        exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
        for flags in FLAGS:
            for idx in (None, "u32", "i64"):
                label = f"{name} n={n} asc={asc} flags={flags} idx={idx}"
                print(label, flush=True)
                k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
                _check(name, bits, asc, k, i, exp_k, exp_i, label)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("asc", [True, False])
def test_medium_sizes(name, asc):
    for n in (65536 + 7, 200003):
        bits = mixed_bits(name, n, seed=n)
        exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
        for flags, idx in ((0, "u32"), (0, None), (_lib.NO_SKIP, "i64")):
            label = f"{name} n={n} asc={asc} flags={flags} idx={idx}"
            print(label, flush=True)
            k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
            _check(name, bits, asc, k, i, exp_k, exp_i, label)


@pytest.mark.parametrize("case", ["dups16", "sorted", "reverse", "all_equal", "two_values"])
@pytest.mark.parametrize("asc", [True, False])
def test_structured_u32(case, asc):
    n = 150001
    if case == "dups16":
        bits = heavy_duplicates_u32(n, 5)
    elif case == "sorted":
        bits = presorted_u32(n, 6)
    elif case == "reverse":
        bits = presorted_u32(n, 6, reverse=True)
    elif case == "all_equal":
        bits = np.full(n, 0xDEADBEEF, dtype=np.uint32)
    else:
        bits = np.where(np.arange(n) % 3 == 0, 7, 0x80000000).astype(np.uint32)
    exp_k, exp_i = gpu_util.oracle_sort("u32", bits, asc)
    for name in ("u32", "i32", "f32"):
        exp_k, exp_i = gpu_util.oracle_sort(name, bits, asc)
        for flags in (0, _lib.NO_SKIP, _lib.NO_FINISH):
            for idx in ("u32", None, "i64"):
                label = f"{case} as {name} asc={asc} flags={flags} idx={idx}"
                print(label, flush=True)
                k, i = gpu_util.gpu_sort(name, bits, asc, flags, idx)
                _check(name, bits, asc, k, i, exp_k, exp_i, label)


def test_scratch_poison_and_determinism():
    """The result does not depend on what scratch held before the call, and
    two calls agree bit for bit."""
    bits = mixed_bits("f32", 123457, seed=9)
    outs = [gpu_util.gpu_sort("f32", bits, True, 0, "u32", poison=p) for p in (0x00, 0xFF, 0x5A)]
    for k, i in outs[1:]:
        assert (k == outs[0][0]).all() and (i == outs[0][1]).all()
    exp_k, exp_i = gpu_util.oracle_sort("f32", bits, True)
    assert (outs[0][0] == exp_k).all() and (outs[0][1] == exp_i).all()


def test_level_byte_accounting():
    """bsort_level_bytes: a split with an empty side moves nothing (keys in
    [0, 16) at the top bit) and keeps the identity indices; a split of
    uniform keys moves every key and makes the indices real."""
    import ctypes
    import torch
    n = 300007
    for bits, moved0, iota1 in ((heavy_duplicates_u32(n, 3), 0, n),
                                (np.random.default_rng(4).integers(0, 1 << 32, n, dtype=np.uint64)
                                 .astype(np.uint32), n, 0)):
        keys = gpu_util.to_device(bits, "u32")
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
        need = _lib.bsort_scratch_bytes(4, n, 1, 1, 0)
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        _lib.check(_lib.bsort_u32(keys.data_ptr(), n, 0, ind.data_ptr(), scratch.data_ptr(), need,
                                  gpu_util.stream()), "bsort_u32")
        live = np.zeros(66, dtype=np.uint64)
        iota = np.zeros(66, dtype=np.uint64)
        moved = np.zeros(66, dtype=np.uint64)
        _lib.bsort_level_stats(scratch.data_ptr(), gpu_util.stream(), live.ctypes.data, None, None,
                               66, None, None)
        assert _lib.bsort_level_bytes(scratch.data_ptr(), gpu_util.stream(), iota.ctypes.data,
                                      moved.ctypes.data, 66) == 66
        assert live[0] == n and iota[0] == n  # level 0: every index is the identity
        assert moved[0] == moved0
        assert iota[1] == iota1
        assert (moved <= live).all() and (iota <= live).all()
        exp_k, exp_i = gpu_util.oracle_sort("u32", bits, True)
        np.testing.assert_array_equal(gpu_util.from_device(keys, "u32"), exp_k)
