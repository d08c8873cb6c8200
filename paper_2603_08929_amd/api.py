"""PyTorch-facing calls: torch supplies device memory and the current HIP
stream; the sort itself is the library's kernels (see _lib.py)."""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _lib
from ._lib import (DESCENDING, IDX64, KEY_F, KEY_I, KEY_U, KEYS_UNCHANGED,  # noqa
                   NO_FINISH, NO_SKIP, PLAIN)

# torch dtype -> (key family, key bytes)
KEY_TYPES = {
    torch.uint8: (KEY_U, 1), torch.int8: (KEY_I, 1),
    torch.int16: (KEY_I, 2), torch.int32: (KEY_I, 4), torch.int64: (KEY_I, 8),
    torch.float16: (KEY_F, 2), torch.bfloat16: (KEY_F, 2),
    torch.float32: (KEY_F, 4), torch.float64: (KEY_F, 8),
}
for _name, _kt in (("uint16", (KEY_U, 2)), ("uint32", (KEY_U, 4)), ("uint64", (KEY_U, 8)),
                   ("float8_e4m3fn", (KEY_F, 1)), ("float8_e5m2", (KEY_F, 1)),
                   ("float8_e4m3fnuz", (KEY_F, 1)), ("float8_e5m2fnuz", (KEY_F, 1))):
    if hasattr(torch, _name):
        KEY_TYPES[getattr(torch, _name)] = _kt


def key_type(dtype: torch.dtype) -> Tuple[int, int]:
    try:
        return KEY_TYPES[dtype]
    except KeyError:
        raise TypeError(f"bsort: unsupported key dtype {dtype}") from None


def scratch_bytes(dtype: torch.dtype, n: int, num_segments: int = 1,
                  with_indices: bool = True, flags: int = 0) -> int:
    _, kb = key_type(dtype)
    return int(_lib.bsort_scratch_bytes(kb, n, num_segments, int(with_indices), flags))


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _flags(descending: bool, flags: int, idx64: bool) -> int:
    return flags | (DESCENDING if descending else 0) | (IDX64 if idx64 else 0)


def sort_(keys: torch.Tensor, descending: bool = False, return_indices: bool = True,
          idx64: bool = False, flags: int = 0, scratch: Optional[torch.Tensor] = None
          ) -> Optional[torch.Tensor]:
    """Sorts a contiguous 1-D device tensor in place; returns the stable
    permutation (uint32 as int32 storage, or int64 with idx64) or None."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("bsort.sort_: need a contiguous 1-D GPU tensor")
    kt, kb = key_type(keys.dtype)
    n = keys.numel()
    fl = _flags(descending, flags, idx64 and return_indices)
    idx = None
    if return_indices:
        idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_scratch_bytes(kb, n, 1, int(return_indices), fl)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    rc = _lib.bsort_sort(keys.data_ptr(), kt, kb, n, fl,
                         idx.data_ptr() if idx is not None else None,
                         scratch.data_ptr(), scratch.numel(), _stream(keys.device))
    _lib.check(rc, "bsort_sort")
    return idx


def sort(x: torch.Tensor, dim: int = -1, descending: bool = False, idx64: bool = True,
         flags: int = 0) -> Tuple[torch.Tensor, torch.Tensor]:
    """Like torch.sort(x, dim, descending, stable=True): (values, indices),
    x left unchanged.  Every slice along dim is one segment of a single
    segmented call.  Indices are int64 (torch's dtype), or uint32 in int32
    storage with idx64=False.  For gradients use sort_along."""
    if x.dim() == 0:
        raise ValueError("bsort.sort: need at least one dimension")
    if x.dim() == 1:
        v = x.contiguous().clone()
        idx = sort_(v, descending=descending, return_indices=True, idx64=idx64, flags=flags)
        return v, idx
    d = dim % x.dim()
    xm = x.movedim(d, -1).contiguous()
    cols = xm.shape[-1]
    rows = xm.numel() // cols if cols else 0
    v = xm.clone().reshape(-1)
    offsets = torch.arange(rows + 1, device=x.device, dtype=torch.int64) * cols
    # offsets made here are valid: no status read (the call stays asynchronous)
    idx = segmented_sort_(v, offsets, descending=descending, return_indices=True, idx64=idx64,
                          flags=flags, check=False)
    return v.reshape(xm.shape).movedim(-1, d), idx.reshape(xm.shape).movedim(-1, d)


def segmented_sort_(keys: torch.Tensor, offsets: torch.Tensor, descending: bool = False,
                    return_indices: bool = True, idx64: bool = False, flags: int = 0,
                    scratch: Optional[torch.Tensor] = None,
                    check: Optional[bool] = None) -> Optional[torch.Tensor]:
    """Sorts the segments [offsets[s], offsets[s+1]) of a 1-D tensor in place,
    all in one pass.  offsets: int64 device tensor of num_segments + 1.
    Offsets are validated on the device; check (default: on) reads the
    verdict back and raises RuntimeError if they were bad (nothing sorted,
    indices undefined) -- a host synchronisation; check=False leaves the
    call asynchronous (device_status(scratch) reads the word later)."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("bsort.segmented_sort_: need a contiguous 1-D GPU tensor")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("bsort.segmented_sort_: offsets must be a contiguous int64 GPU tensor")
    kt, kb = key_type(keys.dtype)
    n = keys.numel()
    B = offsets.numel() - 1
    fl = _flags(descending, flags, idx64 and return_indices)
    idx = None
    if return_indices:
        idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_scratch_bytes(kb, n, max(B, 1), int(return_indices), fl)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    rc = _lib.bsort_segmented(keys.data_ptr(), kt, kb, offsets.data_ptr(), B, n, fl,
                              idx.data_ptr() if idx is not None else None,
                              scratch.data_ptr(), scratch.numel(), _stream(keys.device))
    _lib.check(rc, "bsort_segmented")
    _raise_on_status(scratch, "segmented_sort_", True if check is None else check, offsets,
                     n)
    return idx


def backward_scatter(grad_sorted: torch.Tensor, indices: torch.Tensor,
                     zero_fill: bool = True) -> torch.Tensor:
    """grad_in[r, idx[r, j]] = grad_sorted[r, j] along the last dim.  With
    zero_fill=False the output is not cleared first: only for indices whose
    rows are permutations (as a sort returns them), which write every
    element exactly once."""
    g = grad_sorted.contiguous()
    ix = indices.contiguous()
    cols = g.shape[-1] if g.dim() else 1
    rows = g.numel() // cols if cols else 0
    out = torch.zeros_like(g) if zero_fill else torch.empty_like(g)
    if ix.dtype == torch.int64:
        fl = IDX64
    elif ix.dtype == torch.int32:
        fl = 0
    else:
        raise TypeError("indices must be int32 (uint32 payload) or int64")
    rc = _lib.bsort_backward_scatter(g.data_ptr(), ix.data_ptr(), rows, cols,
                                     g.element_size(), out.data_ptr(), fl, _stream(g.device))
    _lib.check(rc, "bsort_backward_scatter")
    return out


def argsort(keys: torch.Tensor, offsets: Optional[torch.Tensor] = None,
            descending: bool = False, idx64: bool = False, flags: int = 0,
            check: Optional[bool] = None) -> torch.Tensor:
    """The stable permutation that sorts a contiguous 1-D tensor (or each
    segment of it), keys left unchanged: int32 storage of uint32 indices, or
    int64 with idx64.  With offsets, the device's verdict on them is read
    back and bad offsets raise RuntimeError (check=False skips that host
    synchronisation; check=True reads the status without offsets too)."""
    kt, kb = key_type(keys.dtype)
    B, off = _segment_args(keys, offsets)
    n = keys.numel()
    fl = _flags(descending, flags | KEYS_UNCHANGED, idx64)
    idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_scratch_bytes(kb, n, max(B, 1), 1, fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    if offsets is None:
        rc = _lib.bsort_sort(keys.data_ptr(), kt, kb, n, fl, idx.data_ptr(), scratch.data_ptr(),
                             scratch.numel(), _stream(keys.device))
    else:
        rc = _lib.bsort_segmented(keys.data_ptr(), kt, kb, off, B, n, fl, idx.data_ptr(),
                                  scratch.data_ptr(), scratch.numel(), _stream(keys.device))
    _lib.check(rc, "argsort")
    _raise_on_status(scratch, "argsort", check, offsets, n)
    return idx


def _value_bytes(values: torch.Tensor, n: int) -> int:
    """Bytes of one element's payload: a 1-D tensor of n, or n rows of a
    contiguous tensor (the row moves as one word)."""
    if not values.is_cuda or not values.is_contiguous() or values.dim() < 1 \
            or values.shape[0] != n:
        raise ValueError("bsort: values must be a contiguous GPU tensor with one row per key")
    vb = values[0].numel() * values.element_size() if n else values.element_size()
    if vb not in (1, 2, 4, 8, 16):
        raise ValueError(f"bsort: a value row of {vb} bytes; 1, 2, 4, 8 or 16 are supported")
    return vb


def sort_pairs_(keys: torch.Tensor, values: torch.Tensor, offsets: Optional[torch.Tensor] = None,
                descending: bool = False, return_indices: bool = False, idx64: bool = False,
                flags: int = 0, check: Optional[bool] = None) -> Optional[torch.Tensor]:
    """Sorts keys (1-D, or each segment) in place and permutes values (one
    row of 1, 2, 4, 8 or 16 bytes per key) the same way; returns the
    permutation when asked.  check as for argsort."""
    kt, kb = key_type(keys.dtype)
    B, off = _segment_args(keys, offsets)
    n = keys.numel()
    vb = _value_bytes(values, n)
    fl = _flags(descending, flags, idx64 and return_indices)
    idx = None
    if return_indices:
        idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_pairs_scratch_bytes(kb, n, max(B, 1), vb, int(return_indices), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    ip = idx.data_ptr() if idx is not None else None
    if offsets is None:
        rc = _lib.bsort_sort_pairs(keys.data_ptr(), kt, kb, n, fl, values.data_ptr(), vb, ip,
                                   scratch.data_ptr(), scratch.numel(), _stream(keys.device))
    else:
        rc = _lib.bsort_segmented_pairs(keys.data_ptr(), kt, kb, off, B, n, fl,
                                        values.data_ptr(), vb, ip, scratch.data_ptr(),
                                        scratch.numel(), _stream(keys.device))
    _lib.check(rc, "sort_pairs")
    _raise_on_status(scratch, "sort_pairs_", check, offsets, n)
    return idx


def gather(values: torch.Tensor, indices: torch.Tensor,
           offsets: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[j] = values[base(j) + indices[j]] (base: the start of j's segment
    with offsets, else 0) -- applies a sort's permutation to another tensor
    with one row per key."""
    n = indices.numel()
    vb = _value_bytes(values, n)
    if not indices.is_cuda or indices.dim() != 1 or not indices.is_contiguous():
        raise ValueError("bsort.gather: indices must be a contiguous 1-D GPU tensor")
    if indices.dtype == torch.int64:
        fl = IDX64
    elif indices.dtype == torch.int32:
        fl = 0
    else:
        raise TypeError("indices must be int32 (uint32 payload) or int64")
    B, off = _segment_args(indices, offsets)
    out = torch.empty_like(values)
    rc = _lib.bsort_gather(values.data_ptr(), vb, indices.data_ptr(), off,
                           B if offsets is not None else 0, n, fl, out.data_ptr(),
                           _stream(values.device))
    _lib.check(rc, "bsort_gather")
    return out


def scatter(values: torch.Tensor, indices: torch.Tensor,
            offsets: Optional[torch.Tensor] = None, zero_fill: bool = True) -> torch.Tensor:
    """out[base(j) + indices[j]] = values[j] -- the inverse of gather: the
    backward of a (segmented) sort, ragged segments included.  zero_fill=False
    leaves the output uninitialised, for indices that are permutations."""
    n = indices.numel()
    vb = _value_bytes(values, n)
    if not indices.is_cuda or indices.dim() != 1 or not indices.is_contiguous():
        raise ValueError("bsort.scatter: indices must be a contiguous 1-D GPU tensor")
    if indices.dtype == torch.int64:
        fl = IDX64
    elif indices.dtype == torch.int32:
        fl = 0
    else:
        raise TypeError("indices must be int32 (uint32 payload) or int64")
    B, off = _segment_args(indices, offsets)
    out = torch.zeros_like(values) if zero_fill else torch.empty_like(values)
    rc = _lib.bsort_scatter(values.data_ptr(), vb, indices.data_ptr(), off,
                            B if offsets is not None else 0, n, fl, out.data_ptr(),
                            _stream(values.device))
    _lib.check(rc, "bsort_scatter")
    return out


def sort128_(keys: torch.Tensor, family: str = "u", descending: bool = False,
             return_indices: bool = True, idx64: bool = False, flags: int = 0
             ) -> Optional[torch.Tensor]:
    """Sorts 128-bit keys in place: a contiguous (n, 2) 64-bit tensor, row i
    being key i's low and high words.  family: 'u' unsigned, 'i' two's
    complement, 'f' sign | exponent | mantissa (IEEE binary128).  Returns
    the stable permutation or None."""
    if not keys.is_cuda or keys.dim() != 2 or keys.shape[1] != 2 or not keys.is_contiguous() \
            or keys.element_size() != 8:
        raise ValueError("bsort.sort128_: need a contiguous (n, 2) 64-bit GPU tensor")
    kt = {"u": KEY_U, "i": KEY_I, "f": KEY_F}[family]
    n = keys.shape[0]
    fl = _flags(descending, flags, idx64 and return_indices)
    idx = None
    if return_indices:
        idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_scratch_bytes128(n, int(return_indices), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    rc = _lib.bsort_sort128(keys.data_ptr(), kt, n, fl, idx.data_ptr() if idx is not None else None,
                            scratch.data_ptr(), scratch.numel(), _stream(keys.device))
    _lib.check(rc, "bsort_sort128")
    return idx


def sort_layout_(keys: torch.Tensor, bit_order, family: Optional[str] = None,
                 descending: bool = False, return_indices: bool = True, idx64: bool = False,
                 flags: int = 0) -> Optional[torch.Tensor]:
    """Sorts a contiguous 1-D tensor in place as keys whose order bits are
    stored in another layout: bit_order[i] is the stored bit of order bit
    w-1-i (a permutation of 0..w-1).  family: 'u', 'i' or 'f' (default: the
    dtype's).  Returns the stable permutation or None."""
    import ctypes
    kt, kb = key_type(keys.dtype)
    if family is not None:
        kt = {"u": KEY_U, "i": KEY_I, "f": KEY_F}[family]
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("bsort.sort_layout_: need a contiguous 1-D GPU tensor")
    order = (ctypes.c_uint8 * len(bit_order))(*[int(b) for b in bit_order])
    n = keys.numel()
    fl = _flags(descending, flags, idx64 and return_indices)
    idx = None
    if return_indices:
        idx = torch.empty(n, dtype=torch.int64 if idx64 else torch.int32, device=keys.device)
    need = _lib.bsort_scratch_bytes(kb, n, 1, int(return_indices), fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    rc = _lib.bsort_sort_layout(keys.data_ptr(), kt, kb, n, fl, order,
                                idx.data_ptr() if idx is not None else None, scratch.data_ptr(),
                                scratch.numel(), _stream(keys.device))
    _lib.check(rc, "bsort_sort_layout")
    return idx


def sort_inplace_(keys: torch.Tensor, offsets: Optional[torch.Tensor] = None,
                  descending: bool = False, flags: int = 0,
                  check: Optional[bool] = None) -> None:
    """Sorts a contiguous 1-D GPU tensor (or each segment of it) in place
    with the small-scratch in-place variant: keys only, the same sorted keys
    as sort_, no permutation.  check as for argsort."""
    kt, kb = key_type(keys.dtype)
    B, offp = _segment_args(keys, offsets)
    n = keys.numel()
    fl = _flags(descending, flags, False)
    need = _lib.bsort_inplace_scratch_bytes(kb, n, B, fl)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    if offsets is None:
        rc = _lib.bsort_sort_inplace(keys.data_ptr(), kt, kb, n, fl, scratch.data_ptr(),
                                     scratch.numel(), _stream(keys.device))
    else:
        rc = _lib.bsort_segmented_inplace(keys.data_ptr(), kt, kb, offp, B, n, fl,
                                          scratch.data_ptr(), scratch.numel(),
                                          _stream(keys.device))
    _lib.check(rc, "bsort_sort_inplace")
    _raise_on_status(scratch, "sort_inplace_", check, offsets, n)


def device_status(scratch: torch.Tensor) -> int:
    return int(_lib.bsort_device_status(scratch.data_ptr(), _stream(scratch.device)))


_STATUS_BITS = ((1, "a part exceeded the in-LDS finish capacity (internal error)"),
                (2, "the segment offsets failed the device-side check: nothing was sorted "
                    "and the indices are undefined"),
                (4, "a level tile's count prefix was inconsistent (internal error)"),
                (8, "a grid barrier of the tail launch timed out (the result is invalid)"))


def _raise_on_status(scratch: torch.Tensor, what: str, check: Optional[bool],
                     offsets: Optional[torch.Tensor], n: int) -> None:
    """Reads the device status word (a host synchronisation on the keys'
    stream) when check is True, or when check is None and the caller passed
    offsets, which only the device checks; raises if it is not 0."""
    if check is False or (check is None and offsets is None):
        return
    if n == 0:
        return  # no keys: the call enqueued nothing and wrote no status
    st = device_status(scratch)
    if st < 0:
        _lib.check(st, what)
    if st:
        why = "; ".join(text for bit, text in _STATUS_BITS if st & bit)
        raise RuntimeError(f"bsort.{what}: device status {st}: {why}")


def _segment_args(keys: torch.Tensor, offsets: Optional[torch.Tensor]):
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("bsort: need a contiguous 1-D GPU tensor")
    if offsets is not None and (offsets.dtype != torch.int64 or not offsets.is_cuda
                                or not offsets.is_contiguous()):
        raise ValueError("bsort: offsets must be a contiguous int64 GPU tensor")
    B = offsets.numel() - 1 if offsets is not None else 1
    return B, (offsets.data_ptr() if offsets is not None else None)


def autotune(keys: torch.Tensor, offsets: Optional[torch.Tensor] = None,
             descending: bool = False, indices: Optional[torch.Tensor] = None,
             flags: int = 0, reps: int = 2, scratch: Optional[torch.Tensor] = None) -> int:
    """Times every launch configuration on these keys (sorting them, like a
    normal call) and keeps the fastest for calls of this shape class.
    indices: None, or an int32 / int64 tensor of keys.numel() to fill.
    Returns the chosen configuration."""
    kt, kb = key_type(keys.dtype)
    B, off = _segment_args(keys, offsets)
    n = keys.numel()
    fl = _flags(descending, flags, indices is not None and indices.dtype == torch.int64)
    need = _lib.bsort_scratch_bytes(kb, n, max(B, 1), int(indices is not None), fl)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    rc = _lib.bsort_autotune(keys.data_ptr(), kt, kb, off, B, n, fl,
                             indices.data_ptr() if indices is not None else None,
                             scratch.data_ptr(), scratch.numel(), _stream(keys.device), reps)
    if rc < 0:
        _lib.check(rc, "bsort_autotune")
    return rc


class SortGraph:
    """One sort of fixed buffers recorded into a HIP graph; launch() replays
    it on the current stream (the buffers' contents at that time are
    sorted).  Keeps the buffers alive while it exists."""

    def __init__(self, keys: torch.Tensor, offsets: Optional[torch.Tensor] = None,
                 descending: bool = False, indices: Optional[torch.Tensor] = None,
                 flags: int = 0, scratch: Optional[torch.Tensor] = None):
        import ctypes
        kt, kb = key_type(keys.dtype)
        B, off = _segment_args(keys, offsets)
        n = keys.numel()
        fl = _flags(descending, flags, indices is not None and indices.dtype == torch.int64)
        need = _lib.bsort_scratch_bytes(kb, n, max(B, 1), int(indices is not None), fl)
        if scratch is None or scratch.numel() < need:
            scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
        self._bufs = (keys, offsets, indices, scratch)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(keys.device):
            rc = _lib.bsort_graph_create(ctypes.byref(self._h), keys.data_ptr(), kt, kb, off, B,
                                         n, fl, indices.data_ptr() if indices is not None else None,
                                         scratch.data_ptr(), scratch.numel())
        _lib.check(rc, "bsort_graph_create")
        self.device = keys.device
        self.scratch = scratch

    def launch(self) -> None:
        _lib.check(_lib.bsort_graph_launch(self._h, _stream(self.device)), "bsort_graph_launch")

    def close(self) -> None:
        if self._h:
            _lib.check(_lib.bsort_graph_destroy(self._h), "bsort_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
