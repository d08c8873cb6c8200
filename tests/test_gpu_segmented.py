"""Batched (segmented) sorts on the GPU through bsort_segmented: every
segment must equal the oracle's sort of that segment alone -- keys bit for
bit and the stable, segment-local permutation exactly -- and equal the
single-array call on the same keys."""
import numpy as np
import pytest
import torch

from paper_2603_08929_amd import _lib
from paper_2603_08929_amd import workloads as W
from gpu_util import gpu_segmented, gpu_sort, key_bytes, oracle_sort, stream, to_device, FAMILY
from paper_2603_08929_amd.workloads import DTYPES

pytestmark = pytest.mark.gpu

# The in-LDS finish takes parts of up to T keys (T = 8192 for 1-, 2- and
# 4-byte keys, 4096 for 8-byte keys); a level tile is 4096 (2048) keys.
T4, T8 = 8192, 4096


def mixed_lengths(name):
    T = T8 if key_bytes(name) == 8 else T4
    return [0, 1, 2, 0, 3, 63, 64, 65, T - 1, T, T + 1, 2 * T + 1, 0, 4096 * 3 + 17,
            1, 0, 40001, 5, 0]


def check_segments(name, bits, lengths, asc, keys, idx, offs):
    for s in range(len(lengths)):
        a, b = offs[s], offs[s + 1]
        rk, ri = oracle_sort(name, bits[a:b], asc=asc)
        np.testing.assert_array_equal(keys[a:b], rk, err_msg=f"keys, segment {s} len {b - a}")
        if idx is not None:
            np.testing.assert_array_equal(idx[a:b], ri, err_msg=f"idx, segment {s} len {b - a}")


@pytest.mark.parametrize("name", ["u8", "i8", "e4m3", "i16", "f16", "bf16", "u32", "i32",
                                  "f32", "u64", "i64", "f64"])
@pytest.mark.parametrize("asc", [True, False])
def test_mixed_lengths(name, asc):
    lengths = mixed_lengths(name)
    bits = W.mixed_bits(name, int(sum(lengths)), 11)
    print(f"segmented {name} asc={asc} n={bits.size}", flush=True)
    keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
    check_segments(name, bits, lengths, asc, keys, idx, offs)


@pytest.mark.parametrize("flags", [0, _lib.NO_SKIP, _lib.NO_FINISH, _lib.PLAIN])
@pytest.mark.parametrize("idx", [None, "u32", "i64"])
def test_flags_and_index_modes(flags, idx):
    name = "f32"
    lengths = mixed_lengths(name)
    bits = W.mixed_bits(name, int(sum(lengths)), 12)
    print(f"segmented f32 flags={flags} idx={idx}", flush=True)
    for asc in (True, False):
        keys, ind, offs = gpu_segmented(name, bits, lengths, asc=asc, flags=flags, idx=idx)
        check_segments(name, bits, lengths, asc, keys, ind, offs)


@pytest.mark.parametrize("name", ["f32", "i32"])
def test_log_uniform_batch(name):
    """A scaled-down version of the batched workload: 512 arrays with
    log-uniform lengths in [1, 2^16]."""
    lengths = W.batched_lengths(512, 1 << 16, 2)
    n = int(lengths.sum())
    bits = W.normal_bits("f32", n, 0) if name == "f32" else W.uniform_bits("i32", n, 0)
    print(f"log-uniform batch {name} n={n}", flush=True)
    keys, idx, offs = gpu_segmented(name, bits, lengths, asc=True)
    check_segments(name, bits, lengths, True, keys, idx, offs)


@pytest.mark.parametrize("name", ["u8", "i8", "i16", "f16", "i32", "f64", "u64"])
def test_plain_small_segments(name):
    """Plain mode over many small user segments (0 to 300 keys): most start in
    the tiny-segment pass at the top bit, where the sign rules of signed and
    float keys apply, some in its lane path, some in its batches."""
    rng = np.random.default_rng(21)
    lengths = rng.integers(0, 301, size=1500)
    lengths[rng.integers(0, lengths.size, size=200)] = rng.integers(0, 9, size=200)
    bits = W.mixed_bits(name, int(lengths.sum()), 21)
    print(f"segmented plain {name} n={bits.size}", flush=True)
    for asc in (True, False):
        for idx in ("u32", "i64", None):
            keys, ind, offs = gpu_segmented(name, bits, lengths, asc=asc, flags=_lib.PLAIN, idx=idx)
            check_segments(name, bits, lengths, asc, keys, ind, offs)


def test_equals_single_array_calls():
    name = "i32"
    lengths = [5000, 1, 9000, 70000, 0, 8192, 33]
    bits = W.mixed_bits(name, int(sum(lengths)), 13)
    for asc in (True, False):
        keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
        for s in range(len(lengths)):
            a, b = offs[s], offs[s + 1]
            k1, i1 = gpu_sort(name, bits[a:b], asc=asc)
            np.testing.assert_array_equal(keys[a:b], k1)
            np.testing.assert_array_equal(idx[a:b], i1)


def test_single_segment_equals_whole_array():
    name = "u32"
    bits = W.mixed_bits(name, 123457, 14)
    k0, i0, _ = gpu_segmented(name, bits, [bits.size])
    k1, i1 = gpu_sort(name, bits)
    np.testing.assert_array_equal(k0, k1)
    np.testing.assert_array_equal(i0, i1)


def test_many_tiny_segments():
    name = "u16"
    rng = np.random.default_rng(15)
    lengths = rng.integers(0, 4, size=200000)
    bits = W.mixed_bits(name, int(lengths.sum()), 15)
    for asc in (True, False):
        keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
        # compare with a stable numpy lexsort by (segment, order key)
        seg = np.repeat(np.arange(lengths.size), lengths)
        v = bits.astype(np.int64) if asc else -bits.astype(np.int64)
        perm = np.lexsort((v, seg))
        np.testing.assert_array_equal(keys, bits[perm])
        np.testing.assert_array_equal(idx, perm - offs[seg])


def test_constant_and_sorted_segments():
    name = "f32"
    lengths = [20000, 20000, 20000, 9000]
    one = np.float32(-1.5).view(np.uint32)
    parts = [np.full(20000, one, dtype=np.uint32),
             np.sort(W.uniform_bits("u32", 20000, 16)),
             np.sort(W.uniform_bits("u32", 20000, 17))[::-1].copy(),
             W.heavy_duplicates_u32(9000, 18)]
    bits = np.concatenate(parts)
    for asc in (True, False):
        keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
        check_segments(name, bits, lengths, asc, keys, idx, offs)


def test_bad_offsets_reported_and_nothing_sorted():
    """Offsets failing the device-side check: the status word says so and
    neither keys nor indices are written."""
    name = "u32"
    bits = W.uniform_bits(name, 10000, 19)
    for offs in ([0, 6000, 4000, 10000], [0, 5000, 9999], [1, 5000, 10000],
                 [0, -1, 10000], [0, 5000, 20000, 10000]):
        keys = to_device(bits, name)
        offsets = torch.tensor(offs, dtype=torch.int64, device="cuda")
        ind = torch.full((bits.size,), -7, dtype=torch.int32, device="cuda")
        B = len(offs) - 1
        need = _lib.bsort_scratch_bytes(4, bits.size, B, 1, 0)
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        rc = _lib.bsort_segmented(keys.data_ptr(), FAMILY["U"], 4, offsets.data_ptr(), B,
                                  bits.size, 0, ind.data_ptr(), scratch.data_ptr(), need,
                                  stream())
        _lib.check(rc, "bsort_segmented")
        torch.cuda.synchronize()
        assert _lib.bsort_device_status(scratch.data_ptr(), stream()) & 2
        np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint32), bits)
        assert (ind.cpu().numpy() == -7).all()


@pytest.mark.parametrize("name", ["f32", "u8", "i16", "f64"])
def test_many_small_segments(name):
    """20 000 segments of 0..600 keys: most take the one-wave finish (at most
    512 keys, 256 for 8-byte keys), the rest the full one."""
    rng = np.random.default_rng(160)
    lengths = rng.integers(0, 601, size=20000)
    lengths[rng.random(lengths.size) < 0.6] %= 40
    n = int(lengths.sum())
    bits = W.mixed_bits(name, n, 161)
    for asc in (True, False):
        keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
        for s in range(lengths.size):
            a, b = offs[s], offs[s + 1]
            if b - a == 0:
                continue
            rk, ri = oracle_sort(name, bits[a:b], asc=asc)
            np.testing.assert_array_equal(keys[a:b], rk, err_msg=f"segment {s} len {b - a}")
            np.testing.assert_array_equal(idx[a:b], ri, err_msg=f"segment {s} len {b - a}")
