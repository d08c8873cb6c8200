"""The torch-facing sort: bsort.sort(x, dim, descending) against
torch.sort(..., stable=True) on the CPU, for several dtypes, dims and
shapes (empty and single-element slices included); x is left unchanged."""
import pytest
import torch

import paper_2603_08929_amd as bsort

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16, torch.float64,
                                   torch.int32, torch.int16, torch.int64, torch.uint8])
@pytest.mark.parametrize("shape,dim", [((5000,), 0), ((7, 3001), -1), ((7, 3001), 0),
                                       ((4, 5, 6), 1), ((3, 0), -1), ((2, 1), -1)])
def test_sort_matches_torch(dtype, shape, dim):
    g = torch.Generator().manual_seed(7)
    if dtype.is_floating_point:
        x = torch.randn(*shape, generator=g).to(dtype)
        if x.numel() > 10:
            x.view(-1)[::11] = 0.5  # ties
            x.view(-1)[1::13] = -0.0
    elif dtype == torch.uint8:
        x = torch.randint(0, 256, shape, generator=g, dtype=torch.int64).to(dtype)
    else:
        x = torch.randint(-1000, 1000, shape, generator=g, dtype=torch.int64).to(dtype)
    xd = x.cuda()
    before = xd.clone()
    for desc in (False, True):
        v, i = bsort.sort(xd, dim=dim, descending=desc)
        rv, ri = torch.sort(x, dim=dim, descending=desc, stable=True)
        assert torch.equal(v.cpu(), rv)
        assert torch.equal(i.cpu(), ri)
    assert torch.equal(xd, before)


def test_bad_offsets_raise_in_the_torch_api():
    """Offsets the device rejects: segmented_sort_, argsort, sort_pairs_ and
    sort_inplace_ read the status word and raise; with check=False the call
    returns and the keys are left as they were."""
    from paper_2603_08929_amd import api
    keys = torch.arange(100, 0, -1, dtype=torch.int32, device="cuda")
    vals = torch.arange(100, dtype=torch.float32, device="cuda")
    bad = torch.tensor([0, 60, 40, 100], dtype=torch.int64, device="cuda")  # decreasing
    orig = keys.clone()
    for call in (lambda: api.segmented_sort_(keys, bad),
                 lambda: api.argsort(keys, bad),
                 lambda: api.sort_pairs_(keys, vals, bad),
                 lambda: api.sort_inplace_(keys, bad)):
        with pytest.raises(RuntimeError, match="offsets failed"):
            call()
        assert torch.equal(keys, orig)
        assert torch.equal(vals, torch.arange(100, dtype=torch.float32, device="cuda"))
    api.segmented_sort_(keys, bad, check=False)
    torch.cuda.synchronize()
    assert torch.equal(keys, orig)
    good = torch.tensor([0, 40, 60, 100], dtype=torch.int64, device="cuda")
    api.segmented_sort_(keys, good)
    ref = torch.cat([torch.sort(orig[a:b].cpu(), stable=True)[0]
                     for a, b in ((0, 40), (40, 60), (60, 100))])
    assert torch.equal(keys.cpu(), ref)
