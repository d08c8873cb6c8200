"""The C ABI without a GPU: the library loads, exports every function that
include/bsort.h declares, sizes its scratch, and rejects bad arguments
before it would touch a device (no compute call is made here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsort.h")

_lib = pytest.importorskip("paper_2603_08929_amd._lib")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bsort_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for t in ("u8", "u16", "u32", "u64", "i8", "i16", "i32", "i64", "f8", "f16", "f32", "f64"):
        assert f"bsort_{t}" in names
    for n in ("bsort_scratch_bytes", "bsort_segmented", "bsort_backward_scatter",
              "bsort_strerror", "bsort_device_status", "bsort_sort"):
        assert n in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_declared_symbol(name):
    assert hasattr(_lib.lib, name), f"{name} declared in bsort.h but not exported"
    assert name in _lib.SYMBOLS


def test_scratch_bytes():
    sb = _lib.bsort_scratch_bytes
    assert sb(3, 100, 1, 1, 0) == 0            # bad key width
    assert sb(4, 100, 1, 1, 1 << 20) == 0      # unknown flag
    base = sb(4, 1 << 20, 1, 0, 0)
    with_idx = sb(4, 1 << 20, 1, 1, 0)
    idx64 = sb(4, 1 << 20, 1, 1, _lib.IDX64)
    assert base >= 4 * (1 << 20)               # the second key buffer
    assert with_idx - base >= 4 * (1 << 20)    # a second index buffer
    assert idx64 - with_idx >= 4 * (1 << 20)   # both uint32 halves in scratch
    assert sb(4, 1 << 21, 1, 1, 0) > with_idx  # grows with n
    assert sb(8, 1 << 20, 1, 1, 0) > with_idx  # and with the key width
    # the no-finish mode needs work lists for many small segments
    assert sb(4, 1 << 20, 1, 1, _lib.NO_FINISH) > with_idx
    for kb in (1, 2, 4, 8):
        assert sb(kb, 0, 1, 1, 0) > 0 and sb(kb, 1, 1, 1, 0) > 0


def test_strerror():
    assert _lib.strerror(_lib.OK) == "ok"
    assert "scratch" in _lib.strerror(_lib.ESCRATCH)
    assert "invalid" in _lib.strerror(_lib.EINVAL)
    assert "gfx950" in _lib.strerror(_lib.ENODEV)
    assert _lib.strerror(12345) == "unknown status"


def test_validation_before_any_device_work():
    """Every case below returns before the library queries a device."""
    f = _lib.bsort_u32
    fake = 1 << 40  # never dereferenced: validation fails first
    # n = 0 is a no-op that succeeds, even with null pointers
    assert f(None, 0, 0, None, None, 0, None) == _lib.OK
    # unknown flag bits
    assert f(fake, 10, 1 << 7, None, fake, 1 << 30, None) == _lib.EINVAL
    # null keys or scratch with n > 0
    assert f(None, 10, 0, None, fake, 1 << 30, None) == _lib.EINVAL
    assert f(fake, 10, 0, None, None, 1 << 30, None) == _lib.EINVAL
    # scratch too small
    need = _lib.bsort_scratch_bytes(4, 1000, 1, 1, 0)
    assert f(fake, 1000, 0, fake, fake, need - 1, None) == _lib.ESCRATCH
    # 2^32 keys or more: refused with and without indices
    assert f(fake, 1 << 32, 0, fake, fake, 1 << 62, None) == _lib.ETOOBIG
    assert f(fake, 1 << 32, 0, None, fake, 1 << 62, None) == _lib.ETOOBIG
    assert _lib.bsort_u8(fake, (1 << 32) + 12345, 0, None, fake, 1 << 62, None) == _lib.ETOOBIG
    # misaligned scratch
    assert f(fake, 1000, 0, None, fake + 4, 1 << 30, None) == _lib.EINVAL
    # generic entry point: bad key family or width
    assert _lib.bsort_sort(fake, 7, 4, 10, 0, None, fake, 1 << 30, None) == _lib.EINVAL
    assert _lib.bsort_sort(fake, 0, 3, 10, 0, None, fake, 1 << 30, None) == _lib.EINVAL
    # segmented: offsets required; zero segments only with zero keys
    seg = _lib.bsort_segmented
    assert seg(fake, 0, 4, None, 3, 10, 0, None, fake, 1 << 30, None) == _lib.EINVAL
    assert seg(fake, 0, 4, fake, 0, 10, 0, None, fake, 1 << 30, None) == _lib.EINVAL
    assert seg(fake, 0, 4, fake, 0, 0, 0, None, fake, 1 << 30, None) == _lib.OK
    # backward scatter: element width and flags
    bs = _lib.bsort_backward_scatter
    assert bs(fake, fake, 2, 3, 3, fake, 0, None) == _lib.EINVAL
    assert bs(fake, fake, 2, 3, 4, fake, 1, None) == _lib.EINVAL
    assert bs(None, None, 0, 3, 4, None, 0, None) == _lib.OK
    assert bs(None, fake, 2, 3, 4, fake, 0, None) == _lib.EINVAL
    # status read needs a scratch pointer
    assert _lib.bsort_device_status(None, None) == _lib.EINVAL


def test_pairs_argsort_gather_validation():
    """Argsort, key-value and gather arguments are refused before any device
    work; scratch sizes grow by what each mode adds."""
    fake = 1 << 40
    sb, psb = _lib.bsort_scratch_bytes, _lib.bsort_pairs_scratch_bytes
    n = 1 << 20
    # argsort keeps a copy of the keys in scratch
    assert sb(4, n, 1, 1, _lib.KEYS_UNCHANGED) - sb(4, n, 1, 1, 0) >= 4 * n
    # ... and needs the index output
    assert _lib.bsort_u32(fake, 10, _lib.KEYS_UNCHANGED, None, fake, 1 << 30, None) == _lib.EINVAL
    # key-value scratch: the sort's, the permutation when the caller keeps
    # none, and the gathered values
    assert psb(4, n, 1, 3, 0, 0) == 0                       # value width
    assert psb(3, n, 1, 8, 0, 0) == 0                       # key width
    with_idx = psb(4, n, 1, 8, 1, 0)
    assert with_idx - sb(4, n, 1, 1, 0) >= 8 * n
    assert psb(4, n, 1, 8, 0, 0) - with_idx >= 4 * n
    assert psb(4, n, 1, 16, 1, 0) - with_idx >= 8 * n
    sp = _lib.bsort_sort_pairs
    assert sp(None, 0, 4, 0, 0, None, 8, None, None, 0, None) == _lib.OK   # n = 0
    assert sp(fake, 0, 4, 10, 0, fake, 3, None, fake, 1 << 30, None) == _lib.EINVAL
    assert sp(fake, 0, 4, 10, 1 << 7, fake, 8, None, fake, 1 << 30, None) == _lib.EINVAL
    assert sp(fake, 0, 4, 10, 0, None, 8, None, fake, 1 << 30, None) == _lib.EINVAL
    assert sp(fake, 0, 4, 10, 0, fake + 4, 8, None, fake, 1 << 30, None) == _lib.EINVAL
    need = psb(4, 1000, 1, 8, 0, 0)
    assert sp(fake, 0, 4, 1000, 0, fake, 8, None, fake, need - 1, None) == _lib.ESCRATCH
    assert sp(fake, 0, 4, 1 << 32, 0, fake, 8, None, fake, 1 << 62, None) == _lib.ETOOBIG
    spg = _lib.bsort_segmented_pairs
    assert spg(fake, 0, 4, None, 3, 10, 0, fake, 8, None, fake, 1 << 30, None) == _lib.EINVAL
    assert spg(fake, 0, 4, fake, 0, 10, 0, fake, 8, None, fake, 1 << 30, None) == _lib.EINVAL
    g = _lib.bsort_gather
    assert g(None, 8, None, None, 0, 0, 0, None, None) == _lib.OK          # n = 0
    assert g(fake, 8, fake, None, 0, 10, 1, fake, None) == _lib.EINVAL      # flag
    assert g(fake, 12, fake, None, 0, 10, 0, fake, None) == _lib.EINVAL     # width
    assert g(fake, 8, fake, None, 0, 10, 0, fake + 2, None) == _lib.EINVAL  # alignment
    assert g(fake, 8, None, None, 0, 10, 0, fake, None) == _lib.EINVAL      # no indices
    assert g(fake, 8, fake, fake, 0, 10, 0, fake, None) == _lib.EINVAL      # offsets, no segments


def test_torch_dtype_mapping():
    import torch
    from paper_2603_08929_amd import api
    assert api.key_type(torch.float32) == (_lib.KEY_F, 4)
    assert api.key_type(torch.bfloat16) == (_lib.KEY_F, 2)
    assert api.key_type(torch.int8) == (_lib.KEY_I, 1)
    assert api.key_type(torch.uint8) == (_lib.KEY_U, 1)
    with pytest.raises(TypeError):
        api.key_type(torch.complex64)


def test_configurations_and_graph_without_device():
    import ctypes
    n = _lib.bsort_config_count()
    assert n == 12
    names = {_lib.bsort_config_name(i).decode() for i in range(n)}
    assert len(names) == n
    assert _lib.bsort_config_name(n) == b"invalid configuration"
    assert _lib.bsort_config_override(n) == _lib.EINVAL
    assert _lib.bsort_config_override(-2) == _lib.EINVAL
    assert _lib.bsort_config_override(3) == _lib.OK
    assert _lib.bsort_config_override(-1) == _lib.OK
    assert _lib.bsort_tuned_config(3, 1, 100, 1) == _lib.EINVAL
    # graph of an empty sort: no HIP call at all
    h = ctypes.c_void_p()
    assert _lib.bsort_graph_create(None, None, 0, 4, None, 1, 0, 0, None, None, 0) == _lib.EINVAL
    assert _lib.bsort_graph_create(ctypes.byref(h), None, 0, 4, None, 1, 0, 0, None, None,
                                   0) == _lib.OK
    assert h.value
    assert _lib.bsort_graph_launch(h, None) == _lib.OK
    assert _lib.bsort_graph_destroy(h) == _lib.OK
    assert _lib.bsort_graph_launch(None, None) == _lib.EINVAL
    # invalid arguments are refused before any capture
    fake = 1 << 40
    assert _lib.bsort_graph_create(ctypes.byref(h), fake, 7, 4, None, 1, 10, 0, None, fake,
                                   1 << 30) == _lib.EINVAL
    assert _lib.bsort_autotune(fake, 0, 4, None, 1, 10, 1 << 9, None, fake, 1 << 30, None,
                               1) == _lib.EINVAL


def test_sort128_validation():
    fake = 1 << 40
    sb = _lib.bsort_scratch_bytes128
    n = 1 << 20
    assert sb(n, 1, 1 << 7) == 0                       # unknown flag
    base = sb(n, 1, 0)
    assert base >= 16 * n + 8 * n                      # words, permutations, offsets
    assert sb(n, 1, _lib.IDX64) - base >= 8 * n        # wider permutations
    f = _lib.bsort_sort128
    assert f(None, 0, 0, 0, None, None, 0, None) == _lib.OK                        # n = 0
    assert f(fake, 3, 10, 0, fake, fake, 1 << 30, None) == _lib.EINVAL              # key type
    assert f(fake, 0, 10, 1 << 7, fake, fake, 1 << 30, None) == _lib.EINVAL         # flag
    assert f(fake + 8, 0, 10, 0, fake, fake, 1 << 30, None) == _lib.EINVAL          # alignment
    assert f(fake, 0, 10, 0, fake + 2, fake, 1 << 30, None) == _lib.EINVAL          # idx alignment
    assert f(fake, 0, 10, _lib.KEYS_UNCHANGED, None, fake, 1 << 30, None) == _lib.EINVAL
    assert f(fake, 0, 1000, 0, fake, fake, sb(1000, 1, 0) - 1, None) == _lib.ESCRATCH
    assert f(fake, 0, 1 << 32, 0, fake, fake, 1 << 62, None) == _lib.ETOOBIG


def test_layout_validation():
    import ctypes
    fake = 1 << 40
    f = _lib.bsort_sort_layout
    order = (ctypes.c_uint8 * 32)(*range(31, -1, -1))
    bad = (ctypes.c_uint8 * 32)(*([0] * 32))          # not a permutation
    big = (ctypes.c_uint8 * 32)(*([40] + list(range(30, -1, -1))))
    need = _lib.bsort_scratch_bytes(4, 100, 1, 1, 0)
    assert f(None, 0, 4, 0, 0, None, None, None, 0, None) == _lib.OK        # n = 0
    assert f(fake, 0, 4, 100, 0, None, fake, fake, need, None) == _lib.EINVAL
    assert f(fake, 0, 4, 100, 0, bad, fake, fake, need, None) == _lib.EINVAL
    assert f(fake, 0, 4, 100, 0, big, fake, fake, need, None) == _lib.EINVAL
    assert f(fake, 0, 3, 100, 0, order, fake, fake, need, None) == _lib.EINVAL
    assert f(fake + 2, 0, 4, 100, 0, order, fake, fake, need, None) == _lib.EINVAL
    assert f(fake, 0, 4, 100, 0, order, fake, fake, need - 1, None) == _lib.ESCRATCH



def test_inplace_validation_and_scratch():
    """The in-place variant's scratch is a small fraction of the keys, and
    bad arguments are refused before any device work."""
    fake = 1 << 40
    sb = _lib.bsort_inplace_scratch_bytes
    for kb in (1, 2, 4, 8):
        n = 1 << 26
        need = sb(kb, n, 1, 0)
        # per-tile words only: under a quarter of 1-byte keys, 1/16 of 4- and 8-byte keys
        assert 0 < need < n * kb // (4 if kb == 1 else 8 if kb == 2 else 16), (kb, need)
        # far below what the stable path asks for
        assert need * 8 < _lib.bsort_scratch_bytes(kb, n, 1, 0, 0)
    assert sb(3, 100, 1, 0) == 0                                  # width
    assert sb(4, 100, 1, _lib.IDX64) == 0                         # no permutation output
    assert sb(4, 100, 1, _lib.KEYS_UNCHANGED) == 0
    assert sb(4, 1 << 20, 1, _lib.NO_FINISH) > sb(4, 1 << 20, 1, 0)
    assert sb(4, 1 << 20, 5000, 0) > sb(4, 1 << 20, 1, 0)        # per-segment entries
    f = _lib.bsort_sort_inplace
    need = sb(4, 1000, 1, 0)
    assert f(None, 0, 4, 0, 0, None, 0, None) == _lib.OK                       # n = 0
    assert f(fake, 7, 4, 1000, 0, fake, need, None) == _lib.EINVAL             # family
    assert f(fake, 0, 3, 1000, 0, fake, need, None) == _lib.EINVAL             # width
    assert f(fake, 0, 4, 1000, _lib.IDX64, fake, need, None) == _lib.EINVAL    # flag
    assert f(fake, 0, 4, 1000, 1 << 7, fake, need, None) == _lib.EINVAL
    assert f(None, 0, 4, 1000, 0, fake, need, None) == _lib.EINVAL             # null keys
    assert f(fake, 0, 4, 1000, 0, None, need, None) == _lib.EINVAL             # null scratch
    assert f(fake, 0, 4, 1000, 0, fake, need - 1, None) == _lib.ESCRATCH
    assert f(fake, 0, 4, 1000, 0, fake + 4, need, None) == _lib.EINVAL         # alignment
    assert f(fake, 0, 4, 1 << 32, 0, fake, 1 << 62, None) == _lib.ETOOBIG
    seg = _lib.bsort_segmented_inplace
    assert seg(fake, 0, 4, None, 3, 10, 0, fake, 1 << 30, None) == _lib.EINVAL
    assert seg(fake, 0, 4, fake, 0, 10, 0, fake, 1 << 30, None) == _lib.EINVAL
    assert seg(fake, 0, 4, fake, 0, 0, 0, fake, 1 << 30, None) == _lib.OK


def test_scatter_validation():
    fake = 1 << 40
    f = _lib.bsort_scatter
    assert f(None, 4, None, None, 0, 0, 0, None, None) == _lib.OK                 # n = 0
    assert f(fake, 4, fake, None, 0, 10, 1 << 7, fake, None) == _lib.EINVAL       # flag
    assert f(fake, 3, fake, None, 0, 10, 0, fake, None) == _lib.EINVAL            # width
    assert f(fake + 2, 4, fake, None, 0, 10, 0, fake, None) == _lib.EINVAL        # alignment
    assert f(None, 4, fake, None, 0, 10, 0, fake, None) == _lib.EINVAL            # null values
    assert f(fake, 4, fake, fake, 0, 10, 0, fake, None) == _lib.EINVAL            # 0 segments
    assert f(fake, 4, fake, None, 0, 1 << 32, 0, fake, None) == _lib.ETOOBIG


def test_autotune_cache_files(tmp_path):
    """Without tuned choices the cache is just its header, and loads back
    without touching a device; unreadable or malformed files are refused
    and change nothing."""
    _lib.bsort_autotune_reset()
    path = tmp_path / "t.txt"
    assert _lib.bsort_autotune_save(str(path).encode()) == _lib.OK
    assert path.read_text() == "bsort-autotune 1\n"
    assert _lib.bsort_autotune_load(str(path).encode()) == _lib.OK
    assert _lib.bsort_autotune_load(str(tmp_path / "missing.txt").encode()) == _lib.EINVAL
    assert _lib.bsort_autotune_save(str(tmp_path / "no" / "dir.txt").encode()) == _lib.EINVAL
    assert _lib.bsort_autotune_load(None) == _lib.EINVAL
    for text in ("bsort-autotune 2\n", "bsort-autotune 1\ngfx950 256 3 0 10 1\n",
                 "bsort-autotune 1\ngfx950 256 4 2 10 1\n",
                 "bsort-autotune 1\ngfx950 256 4 0 48 1\n",
                 "bsort-autotune 1\ngfx950 256 4 0 10 99\n",
                 "bsort-autotune 1\ngfx950 256 4 0 10 1 extra\n",
                 "bsort-autotune 1\ngfx950 256 4 0\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        assert _lib.bsort_autotune_load(str(bad).encode()) == _lib.EINVAL, text


def test_noalloc_validation_before_any_device_work():
    """The allocation-free entry point: n = 0 succeeds with null pointers,
    bad arguments are refused, and a call needing more scratch than the
    built-in buffer holds returns ENOSPACE -- all before a device is queried."""
    f = _lib.bsort_segmented_noalloc
    fake = 1 << 40
    assert f(None, _lib.KEY_U, 4, None, 0, 0, 0, None, None) == _lib.OK
    assert f(fake, _lib.KEY_U, 3, fake, 1, 10, 0, None, None) == _lib.EINVAL   # key width
    assert f(fake, _lib.KEY_U, 4, fake, 1, 10, 1 << 7, None, None) == _lib.EINVAL  # flag
    cap = _lib.NOALLOC_SCRATCH_BYTES
    n = 1 << 24  # u32 keys with indices: 64 MiB of ping-pong buffers alone
    assert _lib.bsort_scratch_bytes(4, n, 1, 1, 0) > cap
    assert f(fake, _lib.KEY_U, 4, fake, 1, n, 0, fake, None) == _lib.ENOSPACE
    assert "allocation-free" in _lib.strerror(_lib.ENOSPACE)


def test_levels_validation_before_any_device_work():
    """bsort_levels: a level count outside [0, w] is refused, n = 0 succeeds
    with null pointers -- before a device is queried."""
    f = _lib.bsort_levels
    fake = 1 << 40
    assert f(None, _lib.KEY_U, 4, None, 1, 0, 0, 3, None, None, 0, None) == _lib.OK
    for kb, bad in ((1, 9), (2, 17), (4, 33), (8, 65), (4, -1)):
        assert f(fake, _lib.KEY_U, kb, None, 1, 10, 0, bad, None, fake, 1 << 30,
                 None) == _lib.EINVAL, (kb, bad)
    assert f(fake, _lib.KEY_U, 3, None, 1, 10, 0, 1, None, fake, 1 << 30, None) == _lib.EINVAL
