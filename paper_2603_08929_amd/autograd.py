"""Differentiable sort: values = x.gather(dim, idx) with idx the stable
bsort permutation.  The backward of a gather by a permutation sends each
upstream gradient back to the position its value came from:
grad_x[..., idx[..., j]] = grad_values[..., j] (hand-written scatter kernel,
no atomics since idx is a permutation)."""
from __future__ import annotations

import torch

from . import api


def _rows_view(x: torch.Tensor, dim: int):
    d = dim % x.dim()
    xm = x.movedim(d, -1).contiguous()
    cols = xm.shape[-1]
    return d, xm, cols


class BSortFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, dim: int = -1, descending: bool = False):
        if x.dim() == 0:
            raise ValueError("BSortFunction: need at least one dimension")
        d, xm, cols = _rows_view(x, dim)
        rows = xm.numel() // cols if cols else 0
        values = xm.clone().reshape(-1)
        offsets = torch.arange(rows + 1, device=x.device, dtype=torch.int64) * cols
        idx = api.segmented_sort_(values, offsets, descending=descending,
                                  return_indices=True, idx64=True)
        values = values.reshape(xm.shape)
        idx = idx.reshape(xm.shape)
        ctx.save_for_backward(idx)
        ctx.dim = d
        ctx.mark_non_differentiable(idx)
        return values.movedim(-1, d), idx.movedim(-1, d)

    @staticmethod
    def backward(ctx, grad_values, grad_idx):
        (idx,) = ctx.saved_tensors
        d = ctx.dim
        g = grad_values.movedim(d, -1).contiguous()
        gx = api.backward_scatter(g, idx, zero_fill=False)  # idx rows are permutations
        return gx.movedim(-1, d), None, None


def sort_along(x: torch.Tensor, dim: int = -1, descending: bool = False):
    """(values, indices) like torch.sort, differentiable w.r.t. x."""
    return BSortFunction.apply(x, dim, descending)
