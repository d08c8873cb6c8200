#!/usr/bin/env python3
"""Throughput of the bsort bit-partition sort on one MI355X.

One step sorts, in place and with the stable uint32 permutation, each of
the seven 2^26-key single arrays of the benchmark workload:
  int32 uniform over the full range;
  float32 N(0,1) with 0.1% each of signed zeros, subnormals and infinities;
  uint32 uniform in [0, 16) (heavy duplicates);
  uint32 presorted, sorted ascending and descending;
  uint32 reverse-sorted, sorted ascending and descending.
Inputs are resident in HBM before the timed region (one fresh copy per
step and array, cloned beforehand).  value = keys sorted / wall time of the
timed steps (Gkeys/s).

`roofline` covers the dominant kernel, the global-level pass: during the
first timed step (--event-steps) its launches carry hipEvents on the
library's stream that take the kernel's own start and end times from the
dispatch (events add a few microseconds between dependent launches, so the
other timed steps run without them);
algorithmic bytes per launch = the level's live keys read (4 bytes each,
plus 4 for the index where it is not still the identity) and the keys of
segments whose split moved them written with their indices (4 + 4 bytes); a
split with an empty side moves nothing.
`traffic` is the HBM bytes per level launch that the FETCH_SIZE and
WRITE_SIZE counters measured for this kernel (committed summary under
profiles/, scaled by the same counters' reading of a plain 1 GiB copy), or
null if the kernel sources changed since.
`cpu_baseline` times the oracle on the host: the stable flavour on the seven
whole arrays on one pinned core (the value), the Lomuto flavour beside it on
another, and a pinned thread pool over the 4096-array batch and the rows
of the differentiable sort; host CPU model and core count included.

The other workloads are reported beside the headline (`extras`, skipped
with --no-extras): the word-size sweep (8-, 16- and 64-bit keys at 2^28 /
2^27, default and plain w-pass mode), the 4096-array batch in one segmented
call vs one call per array (outputs compared bit for bit), and the backward
scatter of the differentiable sort.

`--summarize-pmc FETCH_CSV WRITE_CSV` turns the counter files of two
rocprofv3 --pmc runs of this script into the traffic summary.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gkeys/s and achieved HBM GB/s per dtype; batched vs per-array, bit-exact"
HBM_PEAK_GBS = 8000.0
N = 1 << 26
MAX_LEVELS = 66
LEVEL_KERNEL = "level_kernel<unsigned int, true"
CALIB_KERNEL = "bitwise_not"
CALIB_ELEMS = 1 << 28  # int32: 1 GiB read + 1 GiB written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "level_kernel_u32_idx_2p26_traffic.txt")
SOURCES = [os.path.join(ROOT, "paper_2603_08929_amd", "csrc", "bsort_kernels.hpp")]  # device code
# The level kernel and everything it is built from come first in that file;
# the hash covers the text up to this line, which follows the kernel.
LEVEL_END = "// ------------------------------------------------------------- LDS finish"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_hash(texts) -> str:
    """Hash of the kernel sources with comments and blank space removed, so
    that only a change of the code itself invalidates a measurement."""
    import re
    h = hashlib.sha256()
    for t in texts:
        t = re.sub(r"/\*.*?\*/", "", t, flags=re.S)
        t = re.sub(r"//[^\n]*", "", t)
        h.update("".join(t.split()).encode())
    return h.hexdigest()[:16]


def source_hash() -> str:
    """Hash of the level kernel's code: the device source up to the end of
    the level kernel."""
    text = open(SOURCES[0]).read()
    cut = text.find(LEVEL_END)
    if cut < 0:
        raise RuntimeError("level kernel end marker not found in the device source")
    return code_hash([text[:cut]])


def workload_arrays():
    """(label, dtype name, raw uint32 bits, descending) for one step."""
    from paper_2603_08929_amd import workloads as W
    i32 = W.uniform_bits("i32", N, 0)
    f32 = W.plant_specials(W.normal_bits("f32", N, 0), "f32", 0.001, 1)
    dup = W.heavy_duplicates_u32(N, 0)
    srt = W.presorted_u32(N, 0)
    rev = srt[::-1].copy()
    return [("i32_uniform", "i32", i32, False),
            ("f32_normal_specials", "f32", f32, False),
            ("u32_dups16", "u32", dup, False),
            ("u32_sorted_asc", "u32", srt, False),
            ("u32_sorted_desc", "u32", srt, True),
            ("u32_reverse_asc", "u32", rev, False),
            ("u32_reverse_desc", "u32", rev, True)]


# ----------------------------------------------------------- counter summary

def summarize_pmc(fetch_csv: str, write_csv: str) -> str:
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the level kernel and of
    the calibration copy -> HBM bytes per level launch."""
    import csv

    def load(path, counter):
        per = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            key = ("level" if LEVEL_KERNEL in name else
                   "calib" if CALIB_KERNEL in name else None)
            if key is None:
                continue
            per.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)
        return per

    fe = load(fetch_csv, "FETCH_SIZE")
    wr = load(write_csv, "WRITE_SIZE")
    true_bytes = 4.0 * CALIB_ELEMS
    f_scale = true_bytes / (sum(fe["calib"]) / len(fe["calib"]))
    w_scale = true_bytes / (sum(wr["calib"]) / len(wr["calib"]))
    nl = len(fe["level"])
    assert nl == len(wr["level"]), "level launches differ between the passes"
    fetch = sum(fe["level"]) / nl * f_scale
    write = sum(wr["level"]) / nl * w_scale
    lines = [
        f"source_sha256_16: {source_hash()}",
        f"level_launches: {nl}",
        f"calibration: {CALIB_KERNEL} over {CALIB_ELEMS} int32 "
        f"({true_bytes / 2**30:.0f} GiB read + {true_bytes / 2**30:.0f} GiB written)",
        f"calib_fetch_counter_bytes: {sum(fe['calib']) / len(fe['calib']):.0f}",
        f"calib_write_counter_bytes: {sum(wr['calib']) / len(wr['calib']):.0f}",
        f"fetch_scale: {f_scale:.4f}",
        f"write_scale: {w_scale:.4f}",
        f"level_fetch_counter_bytes_per_launch: {sum(fe['level']) / nl:.0f}",
        f"level_write_counter_bytes_per_launch: {sum(wr['level']) / nl:.0f}",
        f"level_fetch_bytes_per_launch: {fetch:.0f}",
        f"level_write_bytes_per_launch: {write:.0f}",
        f"level_traffic_bytes_per_launch: {fetch + write:.0f}",
    ]
    return "\n".join(lines) + "\n"


def load_traffic():
    """HBM bytes per level launch from the committed counter summary, or
    None if it is missing or was taken on other kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith(("#", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("source_sha256_16") != source_hash():
            return None
        return float(kv["level_traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# ------------------------------------------------------------------ helpers

def level_stats(lib, scratch, stream):
    """Per level of the last call on this scratch: (live keys, live keys whose
    indices are still the identity, keys of segments whose split moved them),
    then the keys of the LDS finish and of the copy-back."""
    import ctypes
    import numpy as np
    live = np.zeros(MAX_LEVELS, dtype=np.uint64)
    iota = np.zeros(MAX_LEVELS, dtype=np.uint64)
    moved = np.zeros(MAX_LEVELS, dtype=np.uint64)
    fk = ctypes.c_uint64(0)
    ck = ctypes.c_uint64(0)
    lib.bsort_level_stats(scratch.data_ptr(), stream, live.ctypes.data, None, None, MAX_LEVELS,
                          ctypes.byref(fk), ctypes.byref(ck))
    lib.bsort_level_bytes(scratch.data_ptr(), stream, iota.ctypes.data, moved.ctypes.data,
                          MAX_LEVELS)
    return (live, iota, moved), int(fk.value), int(ck.value)


def level_alg_bytes(stats, lvl, K, I):
    """Algorithmic HBM bytes of one level: its live keys are read (with their
    indices where those are not the identity) and the keys of segments whose
    split moved them are written with their indices."""
    live, iota, moved = (float(x[lvl]) for x in stats)
    return live * K + (live - iota) * I + moved * (K + I)


def alg_bytes(stats, finish_keys, K, I):
    """Algorithmic HBM bytes of one sort: every executed level (above); the
    LDS finish reads and writes its keys once for all remaining bits."""
    tot = sum(level_alg_bytes(stats, lvl, K, I) for lvl in range(MAX_LEVELS))
    return tot + finish_keys * 2.0 * (K + I)


def timed(fn, reps, torch):
    """Median milliseconds of fn() over reps runs, hipEvents on the current
    stream (the one the library is given)."""
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


# ------------------------------------------------------------------- extras

SWEEP_DTYPES = None  # word-size sweep cases to run (names), None for all of them


def extras_word_size(lib, torch, np, dev, stream):
    from paper_2603_08929_amd import workloads as W
    entry = {"u8": lib.bsort_u8, "i8": lib.bsort_i8, "i16": lib.bsort_i16, "f16": lib.bsort_f16,
             "bf16": lib.bsort_f16, "i32": lib.bsort_i32, "f32": lib.bsort_f32,
             "u64": lib.bsort_u64, "i64": lib.bsort_i64, "f64": lib.bsort_f64}
    sint = {1: np.int8, 2: np.int16, 4: np.int32, 8: np.int64}
    N28, N27 = 1 << 28, 1 << 27
    cases = [("u8", N28, "uniform"), ("i8", N28, "uniform"), ("i16", N28, "uniform"),
             ("f16", N28, "normal"), ("bf16", N28, "normal"), ("i32", N27, "uniform"),
             ("f32", N27, "normal"), ("u64", N27, "uniform"), ("i64", N27, "uniform"),
             ("f64", N27, "normal")]
    if SWEEP_DTYPES is not None:
        cases = [c for c in cases if c[0] in SWEEP_DTYPES]
    out = []
    for name, n, dist in cases:
        log(f"word-size sweep {name} n={n}")
        w = W.DTYPES[name][0]
        K, I = w // 8, 4
        bits = W.uniform_bits(name, n, 0) if dist == "uniform" else W.normal_bits(name, n, 0)
        src = torch.from_numpy(bits.view(sint[K])).to(dev)
        del bits
        work = torch.empty_like(src)
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        need = max(lib.bsort_scratch_bytes(K, n, 1, 1, fl) for fl in (0, lib.PLAIN))
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)

        def run(flags):
            lib.check(entry[name](work.data_ptr(), n, flags, idx.data_ptr(), scratch.data_ptr(),
                                  need, stream), name)

        def once(flags):
            work.copy_(src)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            run(flags)
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1)

        once(0)
        ms = sorted(once(0) for _ in range(3))[1]
        stats, fk, _ = level_stats(lib, scratch, stream)
        live = stats[0]
        ab = alg_bytes(stats, fk, K, I)
        # plain mode: exactly w global levels (no LDS finish); the fraction
        # over all of them is the whole sort's algorithmic bytes over its
        # time; the per-pass figure is the median level-kernel launch among
        # those that hold most keys in tiles (late levels move their small
        # segments in the tiny-segment pass instead)
        lib.check(lib.bsort_timing_arm(w), "arm")
        ms_plain = once(lib.PLAIN)
        lv_ms = np.zeros(w, dtype=np.float32)
        lv = np.zeros(w, dtype=np.int32)
        got = lib.bsort_timing_read(lv_ms.ctypes.data, lv.ctypes.data, w)
        lib.bsort_timing_disarm()
        pstats, pfk, _ = level_stats(lib, scratch, stream)
        ab_plain = alg_bytes(pstats, pfk, K, I)
        full = [i for i in range(1, got) if float(pstats[2][lv[i]]) >= 0.5 * n]
        per_pass = float(np.median(lv_ms[full])) if full else float("nan")
        pass_bytes = 2.0 * n * (K + I)
        out.append({
            "dtype": name, "n": n, "ms": round(ms, 3), "gkeys_s": round(n / ms / 1e6, 3),
            "levels_executed": int((live > 0).sum()), "finish_keys": fk,
            "alg_GBps": round(ab / ms / 1e6, 1), "alg_frac": round(ab / ms / 1e6 / HBM_PEAK_GBS, 4),
            "plain_ms": round(ms_plain, 3), "plain_levels": int(got),
            "plain_alg_frac": round(ab_plain / ms_plain / 1e6 / HBM_PEAK_GBS, 4),
            "plain_pass_us": round(per_pass * 1e3, 1),
            "plain_pass_frac": round(pass_bytes / (per_pass / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        })
        del src, work, idx, scratch
        torch.cuda.empty_cache()
    return out


def extras_batched(lib, torch, np, dev, stream):
    from paper_2603_08929_amd import api
    from paper_2603_08929_amd import workloads as W
    lengths = W.batched_lengths()
    n = int(lengths.sum())
    B = lengths.size
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    offsets = torch.from_numpy(offs).to(dev)
    out = []
    for name in ("f32", "i32"):
        log(f"batched {name} n={n} arrays={B}")
        lib.bsort_autotune_reset()
        kt = lib.KEY_F if name == "f32" else lib.KEY_I
        typed = lib.bsort_f32 if name == "f32" else lib.bsort_i32
        tdt = torch.float32 if name == "f32" else torch.int32
        bits = W.normal_bits("f32", n, 0) if name == "f32" else W.uniform_bits("i32", n, 0)
        src = torch.from_numpy(bits.view(np.int32)).to(dev)
        del bits
        work = torch.empty_like(src)
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        need = lib.bsort_scratch_bytes(4, n, B, 1, 0)
        need1 = lib.bsort_scratch_bytes(4, int(lengths.max()), 1, 1, 0)
        scratch = torch.empty(max(need, need1), dtype=torch.uint8, device=dev)
        kp, ip, sp = work.data_ptr(), idx.data_ptr(), scratch.data_ptr()

        def batched():
            lib.check(lib.bsort_segmented(kp, kt, 4, offsets.data_ptr(), B, n, 0, ip, sp,
                                          scratch.numel(), stream), "segmented")

        def per_array():
            for s in range(B):
                a = int(offs[s])
                lib.check(typed(kp + 4 * a, int(lengths[s]), 0, ip + 4 * a, sp, need1, stream),
                          "per-array")

        def once(fn):
            work.copy_(src)
            return timed(fn, 1, torch)

        once(batched)
        t_b = sorted(once(batched) for _ in range(3))[1]
        stats, fk, _ = level_stats(lib, scratch, stream)
        live = stats[0]
        ab = alg_bytes(stats, fk, 4, 4)
        kb, ib = work.clone(), idx.clone()
        once(per_array)
        t_p = once(per_array)
        same = bool(torch.equal(kb, work) and torch.equal(ib, idx))
        # autotuned, then the tuned call recorded into a HIP graph
        work.copy_(src)
        best = api.autotune(work.view(tdt), offsets=offsets, indices=idx, reps=2,
                            scratch=scratch)
        t_t = sorted(once(batched) for _ in range(3))[1]
        same_t = bool(torch.equal(kb, work) and torch.equal(ib, idx))
        g = api.SortGraph(work.view(tdt), offsets=offsets, indices=idx, scratch=scratch)
        t_g = sorted(once(g.launch) for _ in range(3))[1]
        same_g = bool(torch.equal(kb, work) and torch.equal(ib, idx))
        g.close()
        lib.bsort_autotune_reset()
        out.append({"dtype": name, "arrays": B, "keys": n,
                    "batched_ms": round(t_b, 3), "batched_gkeys_s": round(n / t_b / 1e6, 3),
                    "batched_alg_GBps": round(ab / t_b / 1e6, 1),
                    "per_array_ms": round(t_p, 3), "per_array_gkeys_s": round(n / t_p / 1e6, 3),
                    "speedup": round(t_p / t_b, 2), "bit_exact_equal": same,
                    "autotuned_config": lib.bsort_config_name(best).decode(),
                    "autotuned_ms": round(t_t, 3), "autotuned_gkeys_s": round(n / t_t / 1e6, 3),
                    "graph_ms": round(t_g, 3), "graph_gkeys_s": round(n / t_g / 1e6, 3),
                    "tuned_and_graph_bit_exact_equal": same_t and same_g,
                    "levels_executed": int((live > 0).sum()), "finish_keys": fk})
        del src, work, idx, scratch, kb, ib
        torch.cuda.empty_cache()
    return out


def extras_small(lib, torch, np, dev, stream):
    """64 Ki uint32 keys (seed 0), ascending, with indices: a latency-bound
    size, one eager call vs one graph launch."""
    from paper_2603_08929_amd import api
    from paper_2603_08929_amd import workloads as W
    log("small array, eager vs graph")
    n = 1 << 16
    src = torch.from_numpy(W.uniform_bits("u32", n, 0).view(np.int32)).to(dev)
    work = torch.empty_like(src)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    need = lib.bsort_scratch_bytes(4, n, 1, 1, 0)
    scratch = torch.empty(need, dtype=torch.uint8, device=dev)

    def eager():
        lib.check(lib.bsort_u32(work.data_ptr(), n, 0, idx.data_ptr(), scratch.data_ptr(), need,
                                stream), "u32")

    def once(fn):
        work.copy_(src)
        return timed(fn, 1, torch)

    for _ in range(3):
        once(eager)
    t_e = sorted(once(eager) for _ in range(21))[10]
    ke, ie = work.clone(), idx.clone()
    g = api.SortGraph(work.view(torch.uint32), indices=idx, scratch=scratch)
    for _ in range(3):
        once(g.launch)
    t_g = sorted(once(g.launch) for _ in range(21))[10]
    same = bool(torch.equal(ke, work) and torch.equal(ie, idx))
    g.close()
    return {"n": n, "eager_us": round(t_e * 1e3, 1), "eager_gkeys_s": round(n / t_e / 1e6, 3),
            "graph_us": round(t_g * 1e3, 1), "graph_gkeys_s": round(n / t_g / 1e6, 3),
            "bit_exact_equal": same}


def extras_pairs(lib, torch, np, dev, stream):
    """Argsort and key-value modes on the f32 N(0,1) 2^26-key array (the
    indexed sort beside them, outputs compared bit for bit), the payload
    gather alone, and a small-key-width workload: 2^24 tokens routed by an
    8-bit id (256 ids) and a 16-bit id (4096 ids) with 8-byte payloads,
    checked against torch's stable sort."""
    from paper_2603_08929_amd import workloads as W
    log("argsort and key-value modes")
    n = 1 << 26
    src = torch.from_numpy(W.normal_bits("f32", n, 0).view(np.int32)).to(dev)
    keys = torch.empty_like(src)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    idx2 = torch.empty_like(idx)
    vals0 = torch.arange(n, dtype=torch.int64, device=dev) * 2654435761
    vals = torch.empty_like(vals0)
    out = torch.empty_like(vals0)
    need = max(lib.bsort_scratch_bytes(4, n, 1, 1, 0),
               lib.bsort_scratch_bytes(4, n, 1, 1, lib.KEYS_UNCHANGED),
               lib.bsort_pairs_scratch_bytes(4, n, 1, 8, 0, 0))
    scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    sp, sn = scratch.data_ptr(), scratch.numel()

    def med(prep, fn, reps=5):
        ts = []
        for _ in range(reps + 1):
            prep()
            torch.cuda.synchronize()
            ts.append(timed(fn, 1, torch))
        return sorted(ts[1:])[reps // 2]

    def cp_keys():
        keys.copy_(src)

    def cp_both():
        keys.copy_(src)
        vals.copy_(vals0)

    t_idx = med(cp_keys, lambda: lib.check(lib.bsort_f32(keys.data_ptr(), n, 0, idx.data_ptr(),
                                                          sp, sn, stream), "f32"))
    ref_keys = keys.clone()
    t_arg = med(cp_keys, lambda: lib.check(lib.bsort_f32(keys.data_ptr(), n, lib.KEYS_UNCHANGED,
                                                          idx2.data_ptr(), sp, sn, stream), "arg"))
    arg_ok = bool(torch.equal(keys, src) and torch.equal(idx2, idx))
    t_pair = med(cp_both, lambda: lib.check(lib.bsort_sort_pairs(
        keys.data_ptr(), lib.KEY_F, 4, n, 0, vals.data_ptr(), 8, None, sp, sn, stream), "pairs"))
    pair_ok = bool(torch.equal(keys, ref_keys) and torch.equal(vals, vals0[idx.long()]))
    t_g = med(lambda: None, lambda: lib.check(lib.bsort_gather(
        vals0.data_ptr(), 8, idx.data_ptr(), None, 0, n, 0, out.data_ptr(), stream), "gather"))
    gather_ok = bool(torch.equal(out, vals0[idx.long()]))
    res = {"f32_normal_2p26": {
        "indexed_sort_ms": round(t_idx, 3), "argsort_ms": round(t_arg, 3),
        "pairs_8B_ms": round(t_pair, 3), "pairs_8B_gkeys_s": round(n / t_pair / 1e6, 3),
        "gather_8B_ms": round(t_g, 3),
        "gather_alg_GBps": round(20.0 * n / t_g / 1e6, 1),  # 4 B index + 8 B read + 8 B write
        "bit_exact_equal": arg_ok and pair_ok and gather_ok}}
    del keys, idx, idx2, vals0, vals, out, scratch
    torch.cuda.empty_cache()
    routing = []
    m = 1 << 24
    rng = np.random.default_rng(0)
    for kname, kb, kt, hi, tdt in (("u8", 1, lib.KEY_U, 256, torch.uint8),
                                   ("i16", 2, lib.KEY_I, 4096, torch.int16)):
        ids = torch.from_numpy(rng.integers(0, hi, size=m).astype(np.int64)).to(dev).to(tdt)
        tok0 = torch.arange(m, dtype=torch.int64, device=dev)
        k = torch.empty_like(ids)
        v = torch.empty_like(tok0)
        need = lib.bsort_pairs_scratch_bytes(kb, m, 1, 8, 0, 0)
        scr = torch.empty(need, dtype=torch.uint8, device=dev)

        def prep():
            k.copy_(ids)
            v.copy_(tok0)

        t = med(prep, lambda: lib.check(lib.bsort_sort_pairs(
            k.data_ptr(), kt, kb, m, 0, v.data_ptr(), 8, None, scr.data_ptr(), scr.numel(),
            stream), "routing"))
        rv, ri = torch.sort(ids.to(torch.int32), stable=True)
        ok = bool(torch.equal(k.to(torch.int32), rv) and torch.equal(v, ri))
        routing.append({"key": f"{kname} ids in [0, {hi})", "tokens": m, "value_bytes": 8,
                        "ms": round(t, 3), "gkeys_s": round(m / t / 1e6, 3),
                        "equal_torch_stable_sort": ok})
        del ids, tok0, k, v, scr, rv, ri
    res["token_routing"] = routing
    return res


def extras_wide(lib, torch, np, dev, stream):
    """128-bit keys, 2^26 of them with u32 indices: uniform patterns (every
    high word distinct, so the low-word pass has nothing to do), and high
    words drawn from 1024 values (runs of ~2^16 keys that the low-word pass
    sorts)."""
    log("128-bit keys")
    n = 1 << 26
    rng = np.random.default_rng(0)
    out = []
    for name, nhi in (("u128 uniform", 0), ("u128, 1024 distinct high words", 1024)):
        lo = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
        if nhi:
            hi = rng.integers(0, 1 << 64, size=nhi, dtype=np.uint64)[rng.integers(0, nhi, size=n)]
        else:
            hi = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
        src = torch.from_numpy(np.stack([lo, hi], axis=1).view(np.int64)).to(dev)
        del lo, hi
        keys = torch.empty_like(src)
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        need = lib.bsort_scratch_bytes128(n, 1, 0)
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
        ts = []
        for _ in range(4):
            keys.copy_(src)
            torch.cuda.synchronize()
            ts.append(timed(lambda: lib.check(lib.bsort_sort128(
                keys.data_ptr(), lib.KEY_U, n, 0, idx.data_ptr(), scratch.data_ptr(), need,
                stream), "sort128"), 1, torch))
        t = sorted(ts[1:])[1]
        # ordered as 128-bit unsigned (words compared as signed after flipping
        # their top bits), and the output is the input gathered by idx
        flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
        h, lw = keys[:, 1] ^ flip, keys[:, 0] ^ flip
        ordered = bool(((h[1:] > h[:-1]) | ((h[1:] == h[:-1]) & (lw[1:] >= lw[:-1]))).all())
        il = idx.long()
        same = bool(torch.equal(src[:, 0].contiguous()[il], keys[:, 0].contiguous())
                    and torch.equal(src[:, 1].contiguous()[il], keys[:, 1].contiguous()))
        out.append({"keys": name, "n": n, "ms": round(t, 3), "gkeys_s": round(n / t / 1e6, 3),
                    "ordered": ordered, "gather_of_input_equals_output": same})
        del src, keys, idx, scratch
        torch.cuda.empty_cache()
    return out


def extras_small_segments(lib, torch, np, dev, stream):
    """Segmented sorts of many equal small segments (f32 N(0,1), u32
    indices), checked against torch's stable sort of the rows."""
    log("many small segments")
    out = []
    for segs, seglen in ((1 << 20, 32), (1 << 18, 128), (1 << 16, 512), (1 << 13, 8192)):
        n = segs * seglen
        g = torch.Generator(device=dev).manual_seed(0)
        src = torch.randn(n, generator=g, device=dev)
        offs = torch.arange(0, n + 1, seglen, dtype=torch.int64, device=dev)
        k = torch.empty_like(src)
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        need = lib.bsort_scratch_bytes(4, n, segs, 1, 0)
        scr = torch.empty(need, dtype=torch.uint8, device=dev)
        ts = []
        for _ in range(4):
            k.copy_(src)
            torch.cuda.synchronize()
            ts.append(timed(lambda: lib.check(lib.bsort_segmented(
                k.data_ptr(), lib.KEY_F, 4, offs.data_ptr(), segs, n, 0, idx.data_ptr(),
                scr.data_ptr(), need, stream), "segmented"), 1, torch))
        t = sorted(ts[1:])[1]
        ref = torch.sort(src.view(segs, seglen), dim=1, stable=True)
        ok = bool(torch.equal(ref.values.view(-1), k)
                  and torch.equal(ref.indices.view(-1).to(torch.int32), idx))
        out.append({"segments": segs, "keys_per_segment": seglen, "ms": round(t, 3),
                    "gkeys_s": round(n / t / 1e6, 2), "equal_torch_stable_sort": ok})
        del src, offs, k, idx, scr, ref
    return out


def extras_inplace(lib, torch, np, dev, stream):
    """The in-place keys-only variant beside the stable keys-only sort on the
    same arrays: time (keys restored outside the timed region), scratch each
    asks for, and the sorted keys compared bit for bit."""
    from paper_2603_08929_amd import workloads as W
    out = []
    fam = {"f32": lib.KEY_F, "u32": lib.KEY_U, "u64": lib.KEY_U, "u8": lib.KEY_U}
    carrier = {4: torch.int32, 8: torch.int64, 1: torch.int8}
    for name, n in (("f32", 1 << 26), ("u32", 1 << 26), ("u64", 1 << 27), ("u8", 1 << 26)):
        log(f"in-place {name} n={n}")
        kb = W.DTYPES[name][0] // 8
        bits = W.normal_bits(name, n, 0) if name == "f32" else W.uniform_bits(name, n, 1)
        npc = {1: np.int8, 4: np.int32, 8: np.int64}[kb]
        src = torch.from_numpy(np.ascontiguousarray(bits.astype(W.DTYPES[name][2])).view(npc))
        src = src.to(dev)
        assert src.dtype == carrier[kb]
        a = torch.empty_like(src)
        b = torch.empty_like(src)
        need_ip = lib.bsort_inplace_scratch_bytes(kb, n, 1, 0)
        need_st = lib.bsort_scratch_bytes(kb, n, 1, 0, 0)
        s_ip = torch.empty(need_ip, dtype=torch.uint8, device=dev)
        s_st = torch.empty(need_st, dtype=torch.uint8, device=dev)

        def run_ip():
            lib.check(lib.bsort_sort_inplace(a.data_ptr(), fam[name], kb, n, 0, s_ip.data_ptr(),
                                             need_ip, stream), "inplace")

        def run_st():
            lib.check(lib.bsort_sort(b.data_ptr(), fam[name], kb, n, 0, None, s_st.data_ptr(),
                                     need_st, stream), "stable")

        def med(buf, fn, reps=5):
            ts = []
            for _ in range(reps + 1):
                buf.copy_(src)
                torch.cuda.synchronize()
                ts.append(timed(fn, 1, torch))
            return sorted(ts[1:])[reps // 2]

        t_ip = med(a, run_ip)
        t_st = med(b, run_st)
        ok = bool(torch.equal(a, b)) and lib.bsort_device_status(s_ip.data_ptr(), stream) == 0
        out.append({"dtype": name, "n": n, "inplace_ms": round(t_ip, 3),
                    "inplace_gkeys_s": round(n / t_ip / 1e6, 3), "stable_ms": round(t_st, 3),
                    "inplace_scratch_bytes": int(need_ip), "stable_scratch_bytes": int(need_st),
                    "scratch_ratio_of_keys": round(need_ip / (n * kb), 4), "keys_equal": ok})
        del src, a, b, s_ip, s_st
        torch.cuda.empty_cache()
    return out


def extras_backward(lib, torch, np, dev, stream):
    from paper_2603_08929_amd.autograd import sort_along
    out = []
    for shape, dt in (((1024, 65536), torch.float32), ((4096, 16384), torch.float16)):
        log(f"differentiable sort {tuple(shape)} {dt}")
        g = torch.Generator(device=dev).manual_seed(0)
        x = torch.randn(*shape, generator=g, device=dev, dtype=torch.float32).to(dt)
        g3 = torch.Generator(device=dev).manual_seed(3)
        Wt = torch.randn(*shape, generator=g3, device=dev, dtype=torch.float32).to(dt)
        xg = x.clone().requires_grad_(True)

        def fwd():
            return sort_along(xg)

        v, idx = fwd()
        t_f = timed(fwd, 3, torch)
        gin = torch.empty_like(x)
        rows, cols = shape
        eb = x.element_size()

        def bwd():
            lib.check(lib.bsort_backward_scatter(Wt.data_ptr(), idx.data_ptr(), rows, cols, eb,
                                                 gin.data_ptr(), lib.IDX64, stream), "bwd")

        bwd()
        t_b = timed(bwd, 5, torch)
        loss = (Wt * v).sum()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize(dev)
        t_ab = (time.perf_counter() - t0) * 1e3
        ok = bool(torch.equal(xg.grad, gin))
        bb = (2 * eb + 8) * rows * cols
        out.append({"shape": list(shape), "dtype": str(dt).replace("torch.", ""),
                    "forward_ms": round(t_f, 3),
                    "forward_gkeys_s": round(rows * cols / t_f / 1e6, 3),
                    "backward_scatter_ms": round(t_b, 4),
                    "backward_GBps": round(bb / t_b / 1e6, 1),
                    "backward_frac": round(bb / t_b / 1e6 / HBM_PEAK_GBS, 4),
                    "autograd_backward_wall_ms": round(t_ab, 3), "grad_equal": ok})
        del x, Wt, xg, v, idx, gin
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- CPU baseline

def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def pinned_thread(core, body):
    """Start body() on a thread pinned to one host core (sched_setaffinity
    with pid 0 applies to the calling thread only)."""
    import threading

    def run():
        os.sched_setaffinity(0, {core})
        body()

    t = threading.Thread(target=run)
    t.start()
    return t


def oracle_pool(jobs, cores):
    """Sort every (bits, dtype name, ascending) job with the stable oracle on
    one thread per core, each pinned, largest jobs first; wall seconds."""
    import queue
    import oracle
    q = queue.Queue()
    for j in sorted(jobs, key=lambda j: -j[0].size):
        q.put(j)

    def worker():
        while True:
            try:
                bits, name, asc = q.get_nowait()
            except queue.Empty:
                return
            oracle.sort_dtype(bits, name, asc=asc)

    t0 = time.perf_counter()
    ts = [pinned_thread(c, worker) for c in cores]
    for t in ts:
        t.join()
    return time.perf_counter() - t0


def cpu_baseline(arrays, pool: bool, batch=None, rows=None):
    """The oracle as it stands, on the host's cores, beside the GPU figure.
      - value: the stable flavour (keys + stable indices: the GPU's work) on
        every whole array of the headline workload, one after the other on
        one thread pinned to one core;
      - lomuto: the in-place keys-only flavour (Algorithm 1's exchange) on
        the same whole arrays, at the same time on a second pinned core;
      - pool (the batch of 4096 arrays and the rows of the differentiable
        sort): the stable flavour over all arrays or rows at once, one
        pinned thread per available core (at most 16).
    arrays: (label, dtype name, raw bits, descending)."""
    import numpy as np
    import oracle
    from paper_2603_08929_amd import workloads as W
    avail = sorted(os.sched_getaffinity(0))
    keys = sum(int(a[2].size) for a in arrays)
    log(f"oracle: {len(arrays)} whole arrays, stable and Lomuto, pinned to cores "
        f"{avail[0]} and {avail[-1]}")
    times = {"stable": [], "lomuto": []}

    def flavour(kind):
        def body():
            for (label, name, bits, desc) in arrays:
                w, mode, mant = oracle.DTYPES[name]
                u = bits.astype(np.uint64)
                t = time.perf_counter()
                if kind == "stable":
                    oracle.sort(u, w, mode, asc=not desc, mant_bits=mant, flavour=oracle.STABLE)
                else:
                    oracle.sort(u, w, mode, asc=not desc, mant_bits=mant, flavour=oracle.LOMUTO,
                                with_idx=False)
                times[kind].append(time.perf_counter() - t)
        return body

    ts = [pinned_thread(avail[0], flavour("stable")),
          pinned_thread(avail[-1], flavour("lomuto"))]
    for t in ts:
        t.join()
    st, lo = sum(times["stable"]), sum(times["lomuto"])
    same = len(avail) == 1
    out = {"value": round(keys / st / 1e9, 6), "unit": "Gkeys/s", "cores": 1,
           "kind": "oracle",
           "sample": f"the {len(arrays)} whole arrays of {arrays[0][2].size} keys, keys + "
                     f"stable indices, stable oracle on one pinned core, {st:.1f} s"
                     + (" (sharing its core with the Lomuto run)" if same else
                        " (the Lomuto run beside it on another core)"),
           "host": {"cpu_model": cpu_model(), "cores_available": len(avail),
                    "os_cpu_count": os.cpu_count()},
           "per_array_s": {a[0]: [round(times["stable"][i], 3), round(times["lomuto"][i], 3)]
                           for i, a in enumerate(arrays)},
           "lomuto": {"value": round(keys / lo / 1e9, 6), "unit": "Gkeys/s", "cores": 1,
                      "sample": "same arrays, keys only, in-place exchange flavour, "
                                f"{lo:.1f} s"}}
    if pool:
        cores = avail[:16]
        res = {"threads": len(cores)}
        if batch is None:
            lengths = W.batched_lengths()
            offs = np.concatenate([[0], np.cumsum(lengths)])
            bits = W.normal_bits("f32", int(offs[-1]), 0)
            batch = [bits[offs[s]:offs[s + 1]] for s in range(lengths.size)]
        nb = sum(b.size for b in batch)
        log(f"oracle pool: {len(batch)} arrays, {nb} keys, {len(cores)} threads")
        t = oracle_pool([(b, "f32", True) for b in batch], cores)
        res["batched_f32"] = {"arrays": len(batch), "keys": int(nb), "s": round(t, 3),
                              "gkeys_s": round(nb / t / 1e9, 6)}
        if rows is None:
            rows = [("f32", 1024, 65536), ("f16", 4096, 16384)]
        for (name, r, c) in rows:
            x = W.normal_bits(name, r * c, 5).reshape(r, c)
            log(f"oracle pool: {name} {r}x{c} rows")
            t = oracle_pool([(x[i], name, True) for i in range(r)], cores)
            res[f"rows_{name}_{r}x{c}"] = {"keys": r * c, "s": round(t, 3),
                                          "gkeys_s": round(r * c / t / 1e9, 6)}
        out["pool"] = res
    return out


# --------------------------------------------------------------------- main

EXTRAS_GROUPS = ("word_size_sweep", "batched_vs_per_array", "small_u32_64k",
                 "differentiable_sort", "argsort_and_pairs", "keys_128_bit", "small_segments",
                 "in_place")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extras groups to run (default: all of them)")
    ap.add_argument("--event-steps", type=int, default=1,
                    help="timed steps whose level launches carry hipEvents (the first ones)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--sweep-dtypes", default=None,
                    help="comma-separated dtypes of the word-size sweep (default: all ten)")
    args = ap.parse_args()
    global SWEEP_DTYPES
    if args.sweep_dtypes:
        SWEEP_DTYPES = set(args.sweep_dtypes.split(","))
    if args.summarize_pmc:
        sys.stdout.write(summarize_pmc(*args.summarize_pmc))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the sort of one "
                          "array is a single-GPU workload here (--gpus 1)"}))
        return 2
    if args.extras != "all":
        unknown = [g for g in args.extras.split(",") if g not in EXTRAS_GROUPS]
        if unknown:
            print(f"unknown extras group(s) {unknown}; known: {list(EXTRAS_GROUPS)}",
                  file=sys.stderr)
            return 2

    import numpy as np
    import torch

    from paper_2603_08929_amd import _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    log("generating inputs")
    arrays = workload_arrays()
    entry = {"i32": _lib.bsort_i32, "f32": _lib.bsort_f32, "u32": _lib.bsort_u32}

    # counter calibration: one plain elementwise pass of known size
    a = torch.zeros(CALIB_ELEMS, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.bitwise_not(a, out=b)
    torch.cuda.synchronize(dev)
    del a, b

    pristine = [torch.from_numpy(a[2].view(np.int32)).to(dev) for a in arrays]
    idx = [torch.empty(N, dtype=torch.int32, device=dev) for _ in arrays]
    need = max(_lib.bsort_scratch_bytes(4, N, 1, 1, _lib.DESCENDING if a[3] else 0)
               for a in arrays)
    scratch = torch.empty(need, dtype=torch.uint8, device=dev)

    def sort_one(j, keys):
        fl = _lib.DESCENDING if arrays[j][3] else 0
        rc = entry[arrays[j][1]](keys.data_ptr(), N, fl, idx[j].data_ptr(),
                                 scratch.data_ptr(), need, stream)
        _lib.check(rc, "bsort")

    # work statistics per array (deterministic: identical in every step)
    log("characterising the arrays")
    stats = []  # per array: per-level (live, identity-index, moved) keys
    per_array = []
    launches = []  # level-kernel launches per sort of each array
    for j in range(len(arrays)):
        k = pristine[j].clone()
        _lib.check(_lib.bsort_timing_arm(64), "bsort_timing_arm")
        sort_one(j, k)
        torch.cuda.synchronize(dev)
        t_ms = np.zeros(64, dtype=np.float32)
        t_lv = np.zeros(64, dtype=np.int32)
        launches.append(int(_lib.bsort_timing_read(t_ms.ctypes.data, t_lv.ctypes.data, 64)))
        _lib.bsort_timing_disarm()
        st3, fk, ck = level_stats(_lib, scratch, stream)
        st = _lib.bsort_device_status(scratch.data_ptr(), stream)
        if st != 0:
            raise RuntimeError(f"device status {st} on {arrays[j][0]}")
        stats.append(st3)
        per_array.append({"array": arrays[j][0], "global_levels": int((st3[0] > 0).sum()),
                          "levels_moving_keys": int((st3[2] > 0).sum()),
                          "level_launches": launches[j], "finish_keys": fk, "copy_keys": ck})
        del k

    steps, warm = args.steps, args.warmup
    work = [[p.clone() for p in pristine] for _ in range(steps + warm)]
    torch.cuda.synchronize(dev)
    log("warmup")
    for s in range(warm):
        for j in range(len(arrays)):
            sort_one(j, work[s][j])
    torch.cuda.synchronize(dev)

    # The level launches of the first `ev_steps` timed steps carry the
    # events (the library times the first `cap` level launches after arming);
    # the events add a few microseconds between launches, so the later steps
    # run without them.
    ev_steps = max(1, min(args.event_steps, steps))
    cap = ev_steps * sum(launches)
    _lib.check(_lib.bsort_timing_arm(cap), "bsort_timing_arm")
    log("timed steps")
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for s in range(warm, warm + steps):
        for j in range(len(arrays)):
            sort_one(j, work[s][j])
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    ms = np.zeros(cap, dtype=np.float32)
    lv = np.zeros(cap, dtype=np.int32)
    got = _lib.bsort_timing_read(ms.ctypes.data, lv.ctypes.data, cap)
    _lib.bsort_timing_disarm()
    # the level-kernel launches of the first ev_steps steps, in launch order
    # (step, array, level); levels past the tail depth run in the tail
    # launch, which is not a level-kernel launch
    starts = [i for i in range(got) if lv[i] == 0]
    if got != cap or len(starts) != ev_steps * len(arrays):
        raise RuntimeError(f"timing: {got} of {cap} level launches recorded in "
                           f"{len(starts)} sorts")
    del work

    # algorithmic bytes of each timed level launch
    K, I = 4, 4
    alg = np.zeros(got, dtype=np.float64)
    for q, i0 in enumerate(starts):
        j = q % len(arrays)
        i1 = starts[q + 1] if q + 1 < len(starts) else got
        for i in range(i0, i1):
            lvl = int(lv[i])
            alg[i] = level_alg_bytes(stats[j], lvl, K, I)
    ms = ms[:got]
    cap = got
    level_time_s = float(ms.astype(np.float64).sum()) / 1e3
    achieved = alg.sum() / level_time_s / 1e9
    elapsed = t1 - t0
    keys_total = steps * len(arrays) * N
    value = keys_total / elapsed / 1e9
    traffic = load_traffic()

    extras = None
    if not args.no_extras:
        del pristine, idx, scratch
        torch.cuda.empty_cache()
        groups = {"word_size_sweep": extras_word_size,
                  "batched_vs_per_array": extras_batched,
                  "small_u32_64k": extras_small,
                  "differentiable_sort": extras_backward,
                  "argsort_and_pairs": extras_pairs,
                  "keys_128_bit": extras_wide,
                  "small_segments": extras_small_segments,
                  "in_place": extras_inplace}
        assert tuple(groups) == EXTRAS_GROUPS
        want = list(groups) if args.extras == "all" else args.extras.split(",")
        extras = {g: groups[g](_lib, torch, np, dev, stream) for g in want}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline([(a[0], a[1], a[2], a[3]) for a in arrays], pool=True)
        cpu["gpu_over_oracle"] = round(value / cpu["value"], 1)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(elapsed / steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded numpy PCG64), resident in HBM",
        "config": {"workload": "single arrays of 2^26 keys, keys + stable uint32 indices: "
                               "int32 uniform, float32 N(0,1)+0.1% specials, uint32 in [0,16), "
                               "uint32 presorted and reverse-sorted, each asc and desc",
                   "keys_per_array": N, "arrays_per_step": len(arrays)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "HBM bytes per level launch",
                     "alg_bytes_per_launch": round(float(alg.mean())),
                     "kernel": "level_kernel<u32, idx>",
                     "launches": int(cap), "event_steps": ev_steps,
                     "avg_launch_us": round(level_time_s / cap * 1e6, 3),
                     "level_time_share": round(level_time_s / (elapsed * ev_steps / steps), 4)},
        "cpu_baseline": cpu,
        "per_array": per_array,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
