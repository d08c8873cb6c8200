"""The differentiable sort (BSortFunction / sort_along): forward values and
indices, and the backward scatter kernel, against finite differences on
tie-free inputs and against a gather-based reference gradient."""
import numpy as np
import pytest
import torch

from paper_2603_08929_amd import _lib, api
from paper_2603_08929_amd.autograd import BSortFunction, sort_along
from gpu_util import stream

pytestmark = pytest.mark.gpu


def tie_free(shape, dtype, seed):
    """Distinct values at least 1/16 apart: finite differences with a small
    step never change the order."""
    g = torch.Generator().manual_seed(seed)
    n = int(np.prod(shape))
    v = torch.randperm(n, generator=g).to(torch.float64) / 16.0 - n / 32.0
    return v.reshape(shape).to(dtype)


@pytest.mark.parametrize("dim", [-1, 0, 1])
@pytest.mark.parametrize("descending", [False, True])
def test_forward_matches_stable_torch_sort(dim, descending):
    x = torch.randn(6, 1000, 3, generator=torch.Generator().manual_seed(1))
    x[:, ::7] = 0.25  # ties: the permutation must be the stable one
    v, i = sort_along(x.cuda(), dim=dim, descending=descending)
    rv, ri = torch.sort(x, dim=dim, descending=descending, stable=True)
    assert torch.equal(v.cpu(), rv)
    assert torch.equal(i.cpu(), ri)


def test_gradcheck_float64():
    x = tie_free((3, 17), torch.float64, 2).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: sort_along(t, dim=-1)[0], (x,), eps=1e-6,
                                    atol=1e-9)
    x = tie_free((9, 4), torch.float64, 3).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: sort_along(t, dim=0, descending=True)[0], (x,),
                                    eps=1e-6, atol=1e-9)


def test_finite_differences_float32():
    """Central differences of loss = sum(W * sorted(x)) for every input."""
    x = tie_free((4, 33), torch.float32, 4)
    Wt = torch.randn(4, 33, generator=torch.Generator().manual_seed(3))
    xg = x.cuda().requires_grad_(True)
    v, _ = sort_along(xg)
    (Wt.cuda() * v).sum().backward()
    grad = xg.grad.cpu().double()
    h = 1e-2
    fd = torch.zeros_like(grad)
    for r in range(x.shape[0]):
        for c in range(x.shape[1]):
            xp = x.clone()
            xm = x.clone()
            xp[r, c] += h
            xm[r, c] -= h
            lp = (Wt * torch.sort(xp, dim=-1, stable=True)[0]).sum().double()
            lm = (Wt * torch.sort(xm, dim=-1, stable=True)[0]).sum().double()
            fd[r, c] = (lp - lm) / (2 * h)
    torch.testing.assert_close(grad, fd, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16,
                                   torch.float64])
@pytest.mark.parametrize("descending", [False, True])
def test_backward_equals_gather_reference(dtype, descending):
    g = torch.Generator().manual_seed(5)
    x = torch.randn(37, 5003, generator=g).to(dtype)
    Wt = torch.randn(37, 5003, generator=g).to(dtype)
    xg = x.cuda().requires_grad_(True)
    v, idx = sort_along(xg, descending=descending)
    (Wt.cuda() * v).sum().backward()
    # reference: values = x.gather(idx), autograd of the gather, on the CPU
    xr = x.clone().float().requires_grad_(True)
    vr = xr.gather(-1, idx.cpu())
    (Wt.float() * vr).sum().backward()
    assert torch.equal(xg.grad.cpu().float(), xr.grad)
    assert torch.equal(v.cpu(), x.gather(-1, idx.cpu()))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_backward_scatter_kernel_direct(dtype):
    """grad_in[r, idx[r, j]] = grad_sorted[r, j], uint32 and int64 indices."""
    g = torch.Generator().manual_seed(6)
    rows, cols = 19, 7777
    idx = torch.stack([torch.randperm(cols, generator=g) for _ in range(rows)])
    gs = torch.randn(rows, cols, generator=g).to(dtype)
    ref = torch.zeros_like(gs).scatter_(-1, idx, gs)
    out64 = api.backward_scatter(gs.cuda(), idx.cuda())
    out32 = api.backward_scatter(gs.cuda(), idx.to(torch.int32).cuda())
    assert torch.equal(out64.cpu(), ref)
    assert torch.equal(out32.cpu(), ref)


# (rows, cols, element bytes): whole rows packed into one LDS run (tiny,
# odd and just-fitting rows), one row per 128 KB run, rows cut into 2..8
# slices with ragged last slices, and rows too wide for the staged kernel
# (the direct kernel).
SCATTER_SHAPES = [(5000, 64, 4), (333, 7, 2), (9, 1, 8), (3, 16384, 4), (5, 32768, 2),
                  (4, 65536, 4), (3, 16385, 8), (2, 98309, 4), (3, 131072 * 2 - 1, 4),
                  (2, 524288, 2), (2, 600001, 2), (1, 1 << 17, 8), (6, 20000, 4), (3, 65536, 2)]


@pytest.mark.parametrize("rows,cols,eb", SCATTER_SHAPES)
def test_backward_scatter_shapes_and_skips(rows, cols, eb):
    """Every staging shape against numpy's scatter: random permutations per
    row with some entries replaced by indices outside [0, cols) (negative
    ones for int64), whose output positions must keep the caller's bits."""
    rng = np.random.default_rng(rows * 7 + cols + eb)
    idx = np.stack([rng.permutation(cols) for _ in range(rows)]).astype(np.int64)
    bad = rng.random(idx.shape) < 0.01
    bad.flat[0] = True
    vdt = {2: np.uint16, 4: np.uint32, 8: np.uint64}[eb]
    sdt = {2: np.int16, 4: np.int32, 8: np.int64}[eb]  # same bits, a torch dtype
    g = rng.integers(0, 1 << (8 * eb - 1), size=idx.shape, dtype=np.uint64).astype(vdt)
    fill = vdt(0x5A5A5A5A5A5A5A5A & ((1 << (8 * eb)) - 1))
    gd = torch.from_numpy(g.view(sdt)).cuda()
    for i64 in (False, True):
        ix = idx.copy()
        ix[bad] = np.where(rng.random(int(bad.sum())) < 0.5, cols, -1 if i64 else cols + 9)
        ok = (ix >= 0) & (ix < cols)
        want = np.full(idx.shape, fill, dtype=vdt)
        want[np.nonzero(ok)[0], ix[ok]] = g[ok]
        out = torch.from_numpy(np.full(idx.shape, fill, dtype=vdt).view(sdt)).cuda()
        ind = torch.from_numpy(ix if i64 else ix.astype(np.uint32).view(np.int32)).cuda()
        rc = _lib.bsort_backward_scatter(gd.data_ptr(), ind.data_ptr(), rows, cols, eb,
                                         out.data_ptr(), _lib.IDX64 if i64 else 0, stream())
        _lib.check(rc, "bsort_backward_scatter")
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().view(vdt), want,
                                      err_msg=f"{rows}x{cols} eb={eb} i64={i64}")


def test_edge_shapes():
    for shape in [(0, 5), (5, 0), (1, 1), (3, 1), (1, 70000)]:
        x = torch.randn(*shape).cuda().requires_grad_(True)
        v, i = sort_along(x)
        rv, ri = torch.sort(x.detach().cpu(), dim=-1, stable=True)
        assert torch.equal(v.detach().cpu(), rv) and torch.equal(i.cpu(), ri)
        v.sum().backward()
        assert torch.equal(x.grad.cpu(), torch.ones(shape))
    with pytest.raises(ValueError):
        BSortFunction.apply(torch.tensor(1.0, device="cuda"), -1, False)
