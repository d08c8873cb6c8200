"""Launch configurations, the autotuner and HIP-graph replay: every
configuration must give the oracle's result bit for bit, the autotuner's
choice must be used afterwards, and a recorded graph must sort exactly as
an eager call does, replay after replay."""
import numpy as np
import pytest
import torch

from paper_2603_08929_amd import _lib, api
from paper_2603_08929_amd import workloads as W
from gpu_util import FAMILY, gpu_segmented, gpu_sort, key_bytes, oracle_sort, stream, to_device
from paper_2603_08929_amd.workloads import DTYPES

pytestmark = pytest.mark.gpu

NCFG = 12


@pytest.fixture
def override():
    yield lambda c: _lib.check(_lib.bsort_config_override(c), "override")
    _lib.check(_lib.bsort_config_override(-1), "override")


@pytest.mark.parametrize("config", range(NCFG))
def test_every_configuration_single(config, override):
    override(config)
    print(f"configuration {config}: {_lib.bsort_config_name(config).decode()}", flush=True)
    for name, n in [("u8", 70001), ("i16", 9000), ("f32", 2047), ("f32", 4097), ("f32", 8193),
                    ("i32", 65543), ("f64", 30011), ("u64", 4097)]:
        bits = W.mixed_bits(name, n, 21)
        for asc in (True, False):
            rk, ri = oracle_sort(name, bits, asc=asc)
            for idx in ("u32", "i64"):
                k, i = gpu_sort(name, bits, asc=asc, idx=idx)
                np.testing.assert_array_equal(k, rk, err_msg=f"{name} n={n} asc={asc}")
                np.testing.assert_array_equal(i, ri, err_msg=f"{name} n={n} asc={asc}")
    bits = W.mixed_bits("f32", 300007, 22)
    rk, ri = oracle_sort("f32", bits)
    k, i = gpu_sort("f32", bits, flags=_lib.NO_SKIP)
    np.testing.assert_array_equal(k, rk)
    np.testing.assert_array_equal(i, ri)


@pytest.mark.parametrize("config", range(NCFG))
def test_every_configuration_segmented(config, override):
    override(config)
    lengths = [0, 1, 2, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 0, 20000, 3, 1]
    for name in ("f32", "u16", "i64"):
        bits = W.mixed_bits(name, int(sum(lengths)), 23)
        for asc in (True, False):
            keys, idx, offs = gpu_segmented(name, bits, lengths, asc=asc)
            for s in range(len(lengths)):
                a, b = offs[s], offs[s + 1]
                rk, ri = oracle_sort(name, bits[a:b], asc=asc)
                np.testing.assert_array_equal(keys[a:b], rk)
                np.testing.assert_array_equal(idx[a:b], ri)


def test_autotune_single_array():
    _lib.bsort_autotune_reset()
    try:
        name, n = "i32", 1 << 20
        bits = W.uniform_bits(name, n, 24)
        keys = to_device(bits, name)
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
        best = api.autotune(keys, indices=ind, reps=1)
        assert 0 <= best < NCFG
        assert _lib.bsort_tuned_config(4, 1, n, 1) == best
        assert _lib.bsort_tuned_config(4, 0, n, 1) == 0  # other index mode: untouched
        rk, ri = oracle_sort(name, bits)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(keys.cpu().numpy().view(np.int32).view(np.uint32), rk)
        np.testing.assert_array_equal(ind.cpu().numpy().view(np.uint32).astype(np.int64), ri)
        # a later normal call uses the tuned configuration and still agrees
        k, i = gpu_sort(name, bits)
        np.testing.assert_array_equal(k, rk)
        np.testing.assert_array_equal(i, ri)
    finally:
        _lib.bsort_autotune_reset()


def test_autotune_segmented():
    _lib.bsort_autotune_reset()
    try:
        lengths = W.batched_lengths(256, 1 << 14, 2)
        n = int(lengths.sum())
        bits = W.normal_bits("f32", n, 25)
        keys = to_device(bits, "f32")
        offs = np.concatenate([[0], np.cumsum(lengths)])
        offsets = torch.from_numpy(offs).cuda()
        ind = torch.empty(n, dtype=torch.int64, device="cuda")
        best = api.autotune(keys.view(torch.float32), offsets=offsets, indices=ind,
                            descending=True, reps=1)
        assert 0 <= best < NCFG
        assert _lib.bsort_tuned_config(4, 1, n, lengths.size) == best
        torch.cuda.synchronize()
        kn = keys.cpu().numpy().view(np.uint32)
        inn = ind.cpu().numpy()
        for s in range(lengths.size):
            a, b = offs[s], offs[s + 1]
            rk, ri = oracle_sort("f32", bits[a:b], asc=False)
            np.testing.assert_array_equal(kn[a:b], rk)
            np.testing.assert_array_equal(inn[a:b], ri)
    finally:
        _lib.bsort_autotune_reset()


def test_autotune_cache_round_trip(tmp_path):
    """A tuned choice survives save, reset and load; a hand-written file for
    this device type sets a choice; a file for another type changes
    nothing."""
    _lib.bsort_autotune_reset()
    try:
        name, n = "u32", 1 << 18
        bits = W.uniform_bits(name, n, 26)
        keys = to_device(bits, name)
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
        best = api.autotune(keys, indices=ind, reps=1)
        path = str(tmp_path / "tune.txt")
        assert _lib.bsort_autotune_save(path.encode()) == _lib.OK
        _lib.bsort_autotune_reset()
        assert _lib.bsort_tuned_config(4, 1, n, 1) == 0
        assert _lib.bsort_autotune_load(path.encode()) == _lib.OK
        assert _lib.bsort_tuned_config(4, 1, n, 1) == best
        # hand-written entries: this device type, and another one
        props = torch.cuda.get_device_properties(0)
        arch = props.gcnArchName.replace(" ", "_")
        cls = n.bit_length() - 1
        other = tmp_path / "other.txt"
        other.write_text(f"bsort-autotune 1\ngfx000 7 4 0 {cls} 9\n")
        _lib.bsort_autotune_reset()
        assert _lib.bsort_autotune_load(str(other).encode()) == _lib.OK
        assert _lib.bsort_tuned_config(4, 0, n, 1) == 0
        mine = tmp_path / "mine.txt"
        mine.write_text(f"bsort-autotune 1\n{arch} {props.multi_processor_count} 4 0 {cls} 9\n")
        assert _lib.bsort_autotune_load(str(mine).encode()) == _lib.OK
        assert _lib.bsort_tuned_config(4, 0, n, 1) == 9
        # and a sort with the loaded configuration still agrees with the oracle
        k, i = gpu_sort(name, bits, idx=None)
        np.testing.assert_array_equal(k, oracle_sort(name, bits)[0])
    finally:
        _lib.bsort_autotune_reset()


def _graph_replays(make_eager, graph, keys, pristine, reps=3):
    """Replays the graph several times, with eager work and synchronisation
    between the replays, and compares every replay with the eager result."""
    ek, ei = make_eager()
    for r in range(reps):
        keys.copy_(pristine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        i = graph._bufs[2]
        assert torch.equal(keys, ek), f"replay {r}: keys"  # integer carriers: NaN-safe
        assert torch.equal(i, ei), f"replay {r}: indices"
        _ = (pristine.float() * 2).sum().item()  # unrelated eager work


def test_graph_single_array():
    for name, n, flags in [("u32", 1 << 18, 0), ("f16", 100003, _lib.DESCENDING),
                           ("u64", 5000, 0), ("i8", 1 << 20, _lib.NO_SKIP)]:
        bits = W.mixed_bits(name, n, 26)
        pristine = to_device(bits, name)
        keys = pristine.clone()
        ind = torch.empty(n, dtype=torch.int32, device="cuda")
        g = api.SortGraph(keys.view(_view_dtype(name)), indices=ind, flags=flags)

        def eager():
            k = pristine.clone()
            i = torch.empty(n, dtype=torch.int32, device="cuda")
            kb = key_bytes(name)
            need = _lib.bsort_scratch_bytes(kb, n, 1, 1, flags)
            scr = torch.empty(need, dtype=torch.uint8, device="cuda")
            _lib.check(_lib.bsort_sort(k.data_ptr(), FAMILY[DTYPES[name][1]], kb, n, flags,
                                       i.data_ptr(), scr.data_ptr(), need, stream()), "eager")
            torch.cuda.synchronize()
            return k, i

        _graph_replays(eager, g, keys, pristine)
        ek, ei = eager()
        rk, ri = oracle_sort(name, bits, asc=not (flags & _lib.DESCENDING))
        np.testing.assert_array_equal(ek.cpu().numpy().view(DTYPES[name][2]), rk)
        np.testing.assert_array_equal(ei.cpu().numpy().view(np.uint32).astype(np.int64), ri)
        g.close()


def test_graph_segmented():
    lengths = W.batched_lengths(300, 1 << 15, 2)
    n = int(lengths.sum())
    bits = W.normal_bits("f32", n, 27)
    pristine = to_device(bits, "f32")
    keys = pristine.clone()
    offs = np.concatenate([[0], np.cumsum(lengths)])
    offsets = torch.from_numpy(offs).cuda()
    ind = torch.empty(n, dtype=torch.int32, device="cuda")
    g = api.SortGraph(keys.view(torch.float32), offsets=offsets, indices=ind)

    def eager():
        k, i, _ = gpu_segmented("f32", bits, lengths)
        return (torch.from_numpy(k.view(np.int32).copy()).cuda(),
                torch.from_numpy(i.astype(np.uint32).view(np.int32)).cuda())

    _graph_replays(eager, g, keys, pristine)
    g.close()


def test_graph_of_empty_sort():
    keys = torch.empty(0, dtype=torch.float32, device="cuda")
    g = api.SortGraph(keys)
    g.launch()
    torch.cuda.synchronize()
    g.close()


def _view_dtype(name):
    """The torch dtype whose key family matches the dtype name."""
    return {"u8": torch.uint8, "i8": torch.int8, "i16": torch.int16, "u16": torch.uint16,
            "f16": torch.float16, "bf16": torch.bfloat16, "u32": torch.uint32,
            "i32": torch.int32, "f32": torch.float32, "u64": torch.uint64,
            "i64": torch.int64, "f64": torch.float64}[name]
