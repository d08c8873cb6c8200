"""bsort on MI355X: MSB-first stable bit-partition sort (arXiv 2603.08929)
as HIP kernels for gfx950 behind a C ABI (include/bsort.h).

    import paper_2603_08929_amd as bsort
    values, indices = bsort.sort(x, dim=-1)       # like torch.sort(..., stable=True)
    idx = bsort.sort_(x, descending=True)         # in place
    idx = bsort.segmented_sort_(x, offsets)       # many arrays, one pass
    idx = bsort.argsort(x)                        # keys left unchanged
    bsort.sort_pairs_(keys, values)               # values follow the keys
    y = bsort.BSortFunction.apply(x, -1, False)   # differentiable
"""
from ._lib import (DESCENDING, IDX64, NO_FINISH, NO_SKIP, PLAIN, KEY_F, KEY_I,  # noqa: F401
                   KEY_U, lib, strerror)
from .api import (argsort, backward_scatter, device_status, gather, scatter, scratch_bytes,  # noqa: F401
                  segmented_sort_, sort, sort128_, sort_, sort_inplace_, sort_layout_,
                  sort_pairs_,
                  key_type)
from .autograd import BSortFunction, sort_along  # noqa: F401
