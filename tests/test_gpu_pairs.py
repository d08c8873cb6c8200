"""Argsort (keys left unchanged), key-value sorts and the payload gather,
through the C ABI: the permutation must be the oracle's stable one, the
keys the oracle's sorted keys (or untouched), and every payload row must
come from the input row that the permutation names (numpy's take on the
oracle's indices: the plain definition of applying a permutation)."""
import numpy as np
import pytest
import torch

from paper_2603_08929_amd import _lib, api
from paper_2603_08929_amd import workloads as W
from paper_2603_08929_amd.workloads import DTYPES
from gpu_util import (FAMILY, from_device, gpu_segmented, gpu_sort, key_bytes, oracle_sort,
                      stream, to_device)

pytestmark = pytest.mark.gpu

# value width -> (torch dtype, columns): a row of that many bytes
VALUE_SHAPES = {1: (torch.uint8, 1), 2: (torch.int16, 1), 4: (torch.int32, 1),
                8: (torch.int64, 1), 16: (torch.int64, 2)}


def random_values(n, vb, seed):
    dt, cols = VALUE_SHAPES[vb]
    g = torch.Generator().manual_seed(seed)
    v = torch.randint(-(1 << 62), 1 << 62, (n, cols), generator=g, dtype=torch.int64)
    v = v.to(dt) if dt != torch.int64 else v
    return (v[:, 0] if cols == 1 else v).contiguous()


def pairs_call(name, bits, values, asc=True, flags=0, idx=None, lengths=None):
    """Key-value sort through the C ABI; idx in {None, 'u32', 'i64'}.
    Returns (keys as raw patterns, values on the host, indices or None)."""
    n = bits.size
    keys = to_device(bits, name)
    vals = values.cuda()
    vb = vals.element_size() * (vals[0].numel() if n else 1)
    fl = flags | (0 if asc else _lib.DESCENDING)
    ind = None
    if idx == "u32":
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
    elif idx == "i64":
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        fl |= _lib.IDX64
    B = len(lengths) if lengths is not None else 1
    need = _lib.bsort_pairs_scratch_bytes(key_bytes(name), n, B, vb, int(ind is not None), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    ip = ind.data_ptr() if ind is not None else None
    kt = FAMILY[DTYPES[name][1]]
    if lengths is None:
        rc = _lib.bsort_sort_pairs(keys.data_ptr(), kt, key_bytes(name), n, fl, vals.data_ptr(),
                                   vb, ip, scratch.data_ptr(), scratch.numel(), stream())
    else:
        offs = np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))])
        offsets = torch.from_numpy(offs).cuda()
        rc = _lib.bsort_segmented_pairs(keys.data_ptr(), kt, key_bytes(name), offsets.data_ptr(),
                                        B, n, fl, vals.data_ptr(), vb, ip, scratch.data_ptr(),
                                        scratch.numel(), stream())
    _lib.check(rc, "pairs")
    torch.cuda.synchronize()
    if n:
        assert _lib.bsort_device_status(scratch.data_ptr(), stream()) == 0
    out_i = None
    if ind is not None:
        out_i = ind.cpu().numpy()
        out_i = out_i.view(np.uint32).astype(np.int64) if idx == "u32" else out_i
    return from_device(keys, name), vals.cpu(), out_i


@pytest.mark.parametrize("name", ["u8", "i16", "f16", "f32", "i64", "f64"])
@pytest.mark.parametrize("n", [1, 2, 5000, 70001])
def test_argsort_leaves_keys(name, n):
    bits = W.mixed_bits(name, n, 41)
    for asc in (True, False):
        for idx in ("u32", "i64"):
            k, i = gpu_sort(name, bits, asc=asc, flags=_lib.KEYS_UNCHANGED, idx=idx)
            np.testing.assert_array_equal(k, bits.astype(DTYPES[name][2]))
            _, ri = oracle_sort(name, bits, asc=asc)
            np.testing.assert_array_equal(i, ri)


def test_argsort_segmented_and_python_api():
    lengths = [0, 1, 4095, 4096, 4097, 8193, 0, 30000, 2]
    for name in ("f32", "u16"):
        bits = W.mixed_bits(name, int(sum(lengths)), 42)
        for asc in (True, False):
            k, i, offs = gpu_segmented(name, bits, lengths, asc=asc, flags=_lib.KEYS_UNCHANGED)
            np.testing.assert_array_equal(k, bits.astype(DTYPES[name][2]))
            for s in range(len(lengths)):
                a, b = offs[s], offs[s + 1]
                np.testing.assert_array_equal(i[a:b], oracle_sort(name, bits[a:b], asc=asc)[1])
    # torch-facing call
    bits = W.normal_bits("f32", 100003, 43)
    x = to_device(bits, "f32").view(torch.float32)
    before = x.clone()
    idx = api.argsort(x, descending=True, idx64=True)
    assert torch.equal(x.view(torch.int32), before.view(torch.int32))
    np.testing.assert_array_equal(idx.cpu().numpy(), oracle_sort("f32", bits, asc=False)[1])


@pytest.mark.parametrize("vb", [1, 2, 4, 8, 16])
def test_sort_pairs_value_widths(vb):
    for name, n in (("f32", 100003), ("u16", 70001), ("i64", 5000), ("u8", 3)):
        bits = W.mixed_bits(name, n, 44 + vb)
        vals = random_values(n, vb, 45 + vb)
        for asc in (True, False):
            for idx in (None, "u32", "i64"):
                k, v, i = pairs_call(name, bits, vals, asc=asc, idx=idx)
                rk, ri = oracle_sort(name, bits, asc=asc)
                np.testing.assert_array_equal(k, rk)
                np.testing.assert_array_equal(v.numpy(), np.take(vals.numpy(), ri, axis=0))
                if i is not None:
                    np.testing.assert_array_equal(i, ri)


def test_sort_pairs_keys_unchanged_and_empty():
    name, n = "i32", 65543
    bits = W.mixed_bits(name, n, 46)
    vals = random_values(n, 8, 47)
    k, v, _ = pairs_call(name, bits, vals, flags=_lib.KEYS_UNCHANGED)
    np.testing.assert_array_equal(k, bits.astype(DTYPES[name][2]))
    np.testing.assert_array_equal(v.numpy(), np.take(vals.numpy(), oracle_sort(name, bits)[1],
                                                     axis=0))
    # n = 0: a no-op
    k, v, _ = pairs_call(name, bits[:0], vals[:0])
    assert k.size == 0 and v.numel() == 0


@pytest.mark.parametrize("vb", [4, 16])
def test_segmented_pairs(vb):
    lengths = [3, 0, 1, 2047, 2048, 2049, 8192, 8193, 0, 20000, 1]
    for name in ("f32", "i8"):
        n = int(sum(lengths))
        bits = W.mixed_bits(name, n, 48)
        vals = random_values(n, vb, 49)
        for asc in (True, False):
            k, v, i = pairs_call(name, bits, vals, asc=asc, idx="u32", lengths=lengths)
            offs = np.concatenate([[0], np.cumsum(lengths)])
            vn = vals.numpy()
            for s in range(len(lengths)):
                a, b = offs[s], offs[s + 1]
                rk, ri = oracle_sort(name, bits[a:b], asc=asc)
                np.testing.assert_array_equal(k[a:b], rk)
                np.testing.assert_array_equal(i[a:b], ri)
                np.testing.assert_array_equal(v.numpy()[a:b], np.take(vn[a:b], ri, axis=0))


def test_gather_segmented_and_skips():
    """Segment-local indices, several segments per 4096-position chunk and
    one segment spanning chunks; an index outside its segment leaves its
    output untouched."""
    rng = np.random.default_rng(50)
    lengths = [0, 5, 1, 0, 3000, 7000, 2, 0, 9000, 1]
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    n = int(offs[-1])
    idx = np.concatenate([rng.permutation(m) for m in lengths]).astype(np.int64)
    vals = random_values(n, 8, 51)
    base = np.repeat(offs[:-1], lengths)
    expect = vals.numpy()[base + idx]
    for i64 in (False, True):
        ind = torch.from_numpy(idx if i64 else idx.astype(np.int32)).cuda()
        out = api.gather(vals.cuda(), ind, torch.from_numpy(offs).cuda())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), expect)
    # skipped positions: index == segment length (just outside)
    bad = idx.copy()
    bad[offs[4] + 10] = lengths[4]
    bad[offs[8]] = lengths[8] + 123
    out = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    ind = torch.from_numpy(bad.astype(np.int32)).cuda()
    offsets = torch.from_numpy(offs).cuda()
    vd = vals.cuda()
    rc = _lib.bsort_gather(vd.data_ptr(), 8, ind.data_ptr(), offsets.data_ptr(), len(lengths), n,
                           0, out.data_ptr(), stream())
    _lib.check(rc, "bsort_gather")
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    skip = np.zeros(n, dtype=bool)
    skip[[offs[4] + 10, offs[8]]] = True
    assert (o[skip] == -7).all()
    np.testing.assert_array_equal(o[~skip], expect[~skip])
    # single array, no offsets
    perm = rng.permutation(n)
    out = api.gather(vd, torch.from_numpy(perm.astype(np.int32)).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), vals.numpy()[perm])


def test_python_sort_pairs():
    bits = W.uniform_bits("i16", 200003, 52)
    keys = to_device(bits, "i16")
    vals = random_values(bits.size, 16, 53).cuda()
    v0 = vals.cpu().numpy()
    idx = api.sort_pairs_(keys, vals, descending=True, return_indices=True)
    torch.cuda.synchronize()
    rk, ri = oracle_sort("i16", bits, asc=False)
    np.testing.assert_array_equal(from_device(keys, "i16"), rk)
    np.testing.assert_array_equal(idx.cpu().numpy().view(np.uint32).astype(np.int64), ri)
    np.testing.assert_array_equal(vals.cpu().numpy(), v0[ri])


@pytest.mark.parametrize("vb", [1, 2, 4, 8, 16])
def test_scatter_ragged_segments(vb):
    """bsort_scatter over ragged segments against numpy's assignment
    out[base + idx[j]] = values[j]; it undoes the gather; targets outside
    their segment keep the caller's bits."""
    rng = np.random.default_rng(60 + vb)
    lengths = [0, 5, 1, 0, 3000, 7000, 2, 0, 9000, 1, 4096, 4097]
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    n = int(offs[-1])
    idx = np.concatenate([rng.permutation(m) for m in lengths]).astype(np.int64)
    vals = random_values(n, vb, 61 + vb)
    vn = vals.numpy()
    base = np.repeat(offs[:-1], lengths)
    want = np.zeros_like(vn)
    want[base + idx] = vn
    offsets = torch.from_numpy(offs).cuda()
    for i64 in (False, True):
        ind = torch.from_numpy(idx if i64 else idx.astype(np.int32)).cuda()
        out = api.scatter(vals.cuda(), ind, offsets)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        # inverse of the gather
        back = api.scatter(api.gather(vals.cuda(), ind, offsets), ind, offsets)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(back.cpu().numpy(), vn)
    # skipped targets: index == segment length, and far outside
    bad = idx.copy()
    bad[offs[4] + 10] = lengths[4]
    bad[offs[8]] = lengths[8] + 123
    ok = np.ones(n, dtype=bool)
    ok[[offs[4] + 10, offs[8]]] = False
    fill = torch.full_like(vals, 7)
    out = fill.cuda()
    ind = torch.from_numpy(bad.astype(np.int32)).cuda()
    vd = vals.cuda()
    rc = _lib.bsort_scatter(vd.data_ptr(), vb, ind.data_ptr(), offsets.data_ptr(), len(lengths),
                            n, 0, out.data_ptr(), stream())
    _lib.check(rc, "bsort_scatter")
    torch.cuda.synchronize()
    exp = fill.numpy().copy()
    exp[(base + bad)[ok]] = vn[ok]
    np.testing.assert_array_equal(out.cpu().numpy(), exp)


def test_scatter_is_the_segmented_sort_backward():
    """Gradient of sum(W * sorted) through a segmented sort of ragged rows:
    W scattered back to each key's input position (numpy's autograd-free
    reference: grad[base + idx[j]] = W[j])."""
    rng = np.random.default_rng(62)
    lengths = [1, 17, 0, 5000, 8193, 3]
    name = "f32"
    n = int(sum(lengths))
    bits = W.normal_bits(name, n, 63)
    k, i, offs = gpu_segmented(name, bits, lengths, idx="i64")
    w = rng.standard_normal(n).astype(np.float32)
    g = api.scatter(torch.from_numpy(w).cuda(), torch.from_numpy(i).cuda(),
                    torch.from_numpy(offs).cuda())
    torch.cuda.synchronize()
    base = np.repeat(offs[:-1], lengths)
    want = np.zeros(n, dtype=np.float32)
    want[base + i] = w
    np.testing.assert_array_equal(g.cpu().numpy(), want)
