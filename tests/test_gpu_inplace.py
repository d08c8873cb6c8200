"""The in-place (small-scratch, keys-only) variant through the C ABI: the
sorted keys must equal the oracle's bit for bit, for every key width and
family, both directions, the skip and finish switches, segmented inputs
with empty, single-key and boundary-sized segments, and inputs whose
levels leave many misplaced keys (uniform) or few (nearly sorted, one hot
bit).  The scratch it asks for stays a small fraction of the keys."""
import numpy as np
import pytest
import torch

from paper_2603_08929_amd import _lib, api
from paper_2603_08929_amd import workloads as W
from paper_2603_08929_amd.workloads import DTYPES
from gpu_util import FAMILY, from_device, key_bytes, oracle_sort, stream, to_device

pytestmark = pytest.mark.gpu

NAMES = ["u8", "i8", "e4m3", "u16", "i16", "f16", "bf16", "u32", "i32", "f32", "u64", "i64",
         "f64"]


def gpu_inplace(name, bits, asc=True, flags=0, lengths=None, poison=None):
    n = bits.size
    keys = to_device(bits, name)
    fl = flags | (0 if asc else _lib.DESCENDING)
    B = len(lengths) if lengths is not None else 1
    need = _lib.bsort_inplace_scratch_bytes(key_bytes(name), n, B, fl)
    assert need > 0
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    if poison is not None:
        scratch.fill_(poison)
    kt = FAMILY[DTYPES[name][1]]
    if lengths is None:
        rc = _lib.bsort_sort_inplace(keys.data_ptr(), kt, key_bytes(name), n, fl,
                                     scratch.data_ptr(), scratch.numel(), stream())
    else:
        offs = np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))])
        offsets = torch.from_numpy(offs).cuda()
        rc = _lib.bsort_segmented_inplace(keys.data_ptr(), kt, key_bytes(name),
                                          offsets.data_ptr(), B, n, fl, scratch.data_ptr(),
                                          scratch.numel(), stream())
    _lib.check(rc, "bsort_sort_inplace")
    torch.cuda.synchronize()
    if n:
        assert _lib.bsort_device_status(scratch.data_ptr(), stream()) == 0
    return from_device(keys, name)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("n", [1, 2, 3000, 8193, 70001, 300007])
def test_inplace_matches_oracle(name, n):
    print(f"in-place {name} n={n}", flush=True)
    bits = W.mixed_bits(name, n, 500 + n)
    for asc in (True, False):
        np.testing.assert_array_equal(gpu_inplace(name, bits, asc=asc),
                                      oracle_sort(name, bits, asc=asc)[0],
                                      err_msg=f"{name} n={n} asc={asc}")


@pytest.mark.parametrize("name", ["u32", "f32", "i64", "u8"])
def test_inplace_switches(name):
    """BSORT_NO_SKIP (every bit split) and BSORT_NO_FINISH (no LDS finish:
    every level runs down to bit 0), on stale scratch."""
    n = 20011 if name != "i64" else 5003
    bits = W.mixed_bits(name, n, 510)
    for fl in (_lib.NO_SKIP, _lib.NO_FINISH, _lib.NO_SKIP | _lib.NO_FINISH):
        for asc in (True, False):
            np.testing.assert_array_equal(gpu_inplace(name, bits, asc=asc, flags=fl, poison=0xA5),
                                          oracle_sort(name, bits, asc=asc)[0],
                                          err_msg=f"flags={fl} asc={asc}")


@pytest.mark.parametrize("name", ["f32", "i16", "u64"])
def test_inplace_segmented(name):
    lengths = [0, 1, 2, 4095, 4096, 4097, 8192, 8193, 0, 30000, 1, 65537, 7]
    n = int(sum(lengths))
    bits = W.mixed_bits(name, n, 520)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for asc in (True, False):
        k = gpu_inplace(name, bits, asc=asc, lengths=lengths)
        for s in range(len(lengths)):
            a, b = offs[s], offs[s + 1]
            np.testing.assert_array_equal(k[a:b], oracle_sort(name, bits[a:b], asc=asc)[0],
                                          err_msg=f"segment {s} asc={asc}")


def test_inplace_skewed_levels():
    """Levels with few misplaced keys far apart (nearly sorted input, a
    single set bit in rare keys) and with all keys misplaced (reversed)."""
    n = 1 << 20
    rng = np.random.default_rng(530)
    cases = {
        "sorted": np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64)).astype(np.uint32),
        "reversed": np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64))[::-1]
        .astype(np.uint32),
        "rare_top": np.where(rng.random(n) < 0.001, np.uint32(1 << 31), np.uint32(0))
        | rng.integers(0, 1 << 20, size=n, dtype=np.uint64).astype(np.uint32),
        "constant": np.full(n, 7, dtype=np.uint32),
    }
    for label, bits in cases.items():
        bits = np.ascontiguousarray(bits)
        for asc in (True, False):
            np.testing.assert_array_equal(gpu_inplace("u32", bits, asc=asc),
                                          oracle_sort("u32", bits, asc=asc)[0],
                                          err_msg=f"{label} asc={asc}")


def test_inplace_full_size_against_stable_path():
    """2^26 f32 N(0,1) and 2^27 i64 uniform: the same keys as the stable
    path (itself checked against the oracle), and non-decreasing as numbers
    (no NaN in these inputs, so the float order is the numeric one)."""
    for name, n in (("f32", 1 << 26), ("i64", 1 << 27)):
        print(f"in-place full size {name} n={n}", flush=True)
        bits = W.normal_bits(name, n, 540) if name == "f32" else W.uniform_bits(name, n, 541)
        x = to_device(bits, name)
        if name == "f32":
            x = x.view(torch.float32)
        y = x.clone()
        api.sort_inplace_(x)
        api.sort_(y, return_indices=False)
        torch.cuda.synchronize()
        assert torch.equal(x, y)
        assert bool((x[1:] >= x[:-1]).all())
        del x, y
        torch.cuda.empty_cache()


def test_python_api_and_empty():
    x = torch.empty(0, dtype=torch.float32, device="cuda")
    api.sort_inplace_(x)
    bits = W.mixed_bits("f16", 100003, 550)
    t = to_device(bits, "f16").view(torch.float16)
    offsets = torch.tensor([0, 50000, 50001, 100003], dtype=torch.int64, device="cuda")
    api.sort_inplace_(t, offsets=offsets, descending=True)
    torch.cuda.synchronize()
    got = t.view(torch.int16).cpu().numpy().view(np.uint16)
    for a, b in ((0, 50000), (50000, 50001), (50001, 100003)):
        np.testing.assert_array_equal(got[a:b], oracle_sort("f16", bits[a:b], asc=False)[0])


def test_inplace_many_segments_and_no_finish():
    """2^14 segments of ragged small lengths (all finished straight from the
    seed, one list entry each), and a segmented NO_FINISH call in which every
    segment runs its global levels down to bit 0."""
    rng = np.random.default_rng(560)
    lengths = rng.integers(0, 200, size=1 << 14)
    n = int(lengths.sum())
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for name in ("f32", "u8"):
        bits = W.mixed_bits(name, n, 561)
        k = gpu_inplace(name, bits, asc=False, lengths=list(lengths))
        for s in range(0, lengths.size, 97):
            a, b = offs[s], offs[s + 1]
            np.testing.assert_array_equal(k[a:b], oracle_sort(name, bits[a:b], asc=False)[0])
    lengths = [3000, 1, 0, 12000, 257]
    offs = np.concatenate([[0], np.cumsum(lengths)])
    bits = W.mixed_bits("i32", int(sum(lengths)), 562)
    k = gpu_inplace("i32", bits, flags=_lib.NO_FINISH, lengths=lengths)
    for s in range(len(lengths)):
        a, b = offs[s], offs[s + 1]
        np.testing.assert_array_equal(k[a:b], oracle_sort("i32", bits[a:b])[0])
