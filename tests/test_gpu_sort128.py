"""128-bit keys through the C ABI against the oracle's 128-bit sort, bit for
bit: sorted keys and the stable permutation, for unsigned, two's-complement
and binary128 keys.  The inputs mix binary128 special values, random
patterns, and runs of equal high words both short and longer than the LDS
finish size, so the low-word sort takes its global levels too."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08929_amd import _lib, api
from gpu_util import stream

pytestmark = pytest.mark.gpu

FAM = {oracle.UNSIGNED: _lib.KEY_U, oracle.SIGNED: _lib.KEY_I, oracle.FLOAT: _lib.KEY_F}


def f128(sign, exp, frac):
    return (sign << 127) | (exp << 112) | frac


SPECIALS = [f128(0, 0, 0), f128(1, 0, 0), f128(0, 0, 1), f128(1, 0, 1), f128(0, 16383, 0),
            f128(1, 16383, 0), f128(0, 16383, 1 << 64), f128(1, 16383, 1 << 64),
            f128(0, 0x7FFF, 0), f128(1, 0x7FFF, 0), f128(0, 0x7FFF, 1), f128(1, 0x7FFF, 1),
            f128(1, 0x7FFF, (1 << 112) - 1), 1 << 127, (1 << 127) - 1, (1 << 128) - 1]


def make_keys(n, seed):
    """(lo, hi) uint64 arrays."""
    rng = np.random.default_rng(seed)
    lo = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    hi = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    if n >= 16:
        # a few high words repeated: runs longer than the finish size
        reps = np.array([0x3FFF000000000000, 0xBFFF000000000000, 5, 1 << 63], dtype=np.uint64)
        sel = rng.random(n) < 0.5
        hi[sel] = reps[rng.integers(0, reps.size, size=int(sel.sum()))]
        # duplicated whole keys
        d = rng.integers(0, n, size=n // 8)
        lo[d] = lo[0]
        hi[d] = hi[0]
        # special values
        k = min(len(SPECIALS), n)
        pos = rng.choice(n, size=k, replace=False)
        for p, v in zip(pos, SPECIALS[:k]):
            lo[p], hi[p] = v & ((1 << 64) - 1), v >> 64
    return lo, hi


def gpu_sort128(lo, hi, mode, asc=True, idx="u32", flags=0):
    n = lo.size
    keys = torch.from_numpy(np.stack([lo, hi], axis=1).view(np.int64).copy()).cuda()
    fl = flags | (0 if asc else _lib.DESCENDING)
    ind = None
    if idx == "u32":
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
    elif idx == "i64":
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        fl |= _lib.IDX64
    need = _lib.bsort_scratch_bytes128(n, int(ind is not None), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    rc = _lib.bsort_sort128(keys.data_ptr(), FAM[mode], n, fl,
                            ind.data_ptr() if ind is not None else None, scratch.data_ptr(),
                            scratch.numel(), stream())
    _lib.check(rc, "bsort_sort128")
    torch.cuda.synchronize()
    k = keys.cpu().numpy().view(np.uint64)
    i = None
    if ind is not None:
        i = ind.cpu().numpy()
        i = i.view(np.uint32).astype(np.int64) if idx == "u32" else i
    return k[:, 0].copy(), k[:, 1].copy(), i


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.SIGNED, oracle.FLOAT])
@pytest.mark.parametrize("n", [1, 2, 17, 3000, 70001])
def test_sort128_matches_oracle(mode, n):
    lo, hi = make_keys(n, 100 + n + mode)
    for asc in (True, False):
        rlo, rhi, ri = oracle.sort128(lo, hi, mode, asc=asc)
        for idx in ("u32", "i64", None):
            glo, ghi, gi = gpu_sort128(lo, hi, mode, asc=asc, idx=idx)
            np.testing.assert_array_equal(ghi, rhi, err_msg=f"hi asc={asc} idx={idx}")
            np.testing.assert_array_equal(glo, rlo, err_msg=f"lo asc={asc} idx={idx}")
            if gi is not None:
                np.testing.assert_array_equal(gi, ri)


@pytest.mark.parametrize("mode", [oracle.UNSIGNED, oracle.FLOAT])
def test_sort128_large_and_argsort(mode):
    n = (1 << 20) + 12345
    print(f"128-bit mode {mode} n={n}", flush=True)
    lo, hi = make_keys(n, 200 + mode)
    rlo, rhi, ri = oracle.sort128(lo, hi, mode, asc=True)
    glo, ghi, gi = gpu_sort128(lo, hi, mode)
    np.testing.assert_array_equal(ghi, rhi)
    np.testing.assert_array_equal(glo, rlo)
    np.testing.assert_array_equal(gi, ri)
    # argsort: keys untouched
    glo, ghi, gi = gpu_sort128(lo, hi, mode, flags=_lib.KEYS_UNCHANGED)
    np.testing.assert_array_equal(glo, lo)
    np.testing.assert_array_equal(ghi, hi)
    np.testing.assert_array_equal(gi, ri)


def test_sort128_empty_and_python_api():
    glo, ghi, gi = gpu_sort128(np.zeros(0, np.uint64), np.zeros(0, np.uint64), oracle.SIGNED)
    assert glo.size == 0 and gi.size == 0
    lo, hi = make_keys(50001, 300)
    t = torch.from_numpy(np.stack([lo, hi], axis=1).view(np.int64).copy()).cuda()
    idx = api.sort128_(t, family="i", descending=True, idx64=True)
    torch.cuda.synchronize()
    rlo, rhi, ri = oracle.sort128(lo, hi, oracle.SIGNED, asc=False)
    k = t.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(k[:, 0], rlo)
    np.testing.assert_array_equal(k[:, 1], rhi)
    np.testing.assert_array_equal(idx.cpu().numpy(), ri)
