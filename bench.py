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

`roofline` covers the dominant kernel, the global-level pass: its launches
are bracketed by hipEvents on the library's stream during the timed region;
algorithmic bytes per launch = live keys of that level x (read + write of
key and index: 2 * (4 + 4) bytes; level 0 reads no index: 4 + 4 + 4).
`cpu_baseline` times the oracle (single thread) on a prefix sample.
"""
from __future__ import annotations

import argparse
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23,
                    help="keys per array in the oracle's timed sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the sort of one "
                          "array is a single-GPU workload here (--gpus 1)"}))
        return 2

    import ctypes

    import numpy as np
    import torch

    from paper_2603_08929_amd import _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    arrays = workload_arrays()
    entry = {"i32": _lib.bsort_i32, "f32": _lib.bsort_f32, "u32": _lib.bsort_u32}

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
    live = np.zeros((len(arrays), MAX_LEVELS), dtype=np.uint64)
    per_array = []
    for j in range(len(arrays)):
        k = pristine[j].clone()
        sort_one(j, k)
        fk = ctypes.c_uint64(0)
        ck = ctypes.c_uint64(0)
        buf = np.zeros(MAX_LEVELS, dtype=np.uint64)
        _lib.bsort_level_stats(scratch.data_ptr(), stream, buf.ctypes.data, None, None,
                               MAX_LEVELS, ctypes.byref(fk), ctypes.byref(ck))
        st = _lib.bsort_device_status(scratch.data_ptr(), stream)
        if st != 0:
            raise RuntimeError(f"device status {st} on {arrays[j][0]}")
        live[j] = buf
        per_array.append({"array": arrays[j][0],
                          "global_levels": int((buf > 0).sum()),
                          "finish_keys": int(fk.value), "copy_keys": int(ck.value)})
        del k

    steps, warm = args.steps, args.warmup
    work = [[p.clone() for p in pristine] for _ in range(steps + warm)]
    torch.cuda.synchronize(dev)
    for s in range(warm):
        for j in range(len(arrays)):
            sort_one(j, work[s][j])
    torch.cuda.synchronize(dev)

    cap = steps * len(arrays) * 32
    _lib.check(_lib.bsort_timing_arm(cap), "bsort_timing_arm")
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
    if got != cap:
        raise RuntimeError(f"timing: {got} of {cap} level launches recorded")

    # algorithmic bytes of each timed level launch (launch order: step, array, level)
    K, I = 4, 4
    alg = np.zeros(cap, dtype=np.float64)
    p = 0
    for s in range(steps):
        for j in range(len(arrays)):
            for lvl in range(32):
                nl = float(live[j][lvl])
                alg[p] = nl * ((2 * K + I) if lvl == 0 else 2 * (K + I))
                p += 1
    level_time_s = float(ms.astype(np.float64).sum()) / 1e3
    achieved = alg.sum() / level_time_s / 1e9
    elapsed = t1 - t0
    keys_total = steps * len(arrays) * N
    value = keys_total / elapsed / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = min(args.cpu_sample, N)
        tot = 0.0
        for (label, name, bits, desc) in arrays:
            sample = bits[:m].astype(np.uint64)
            t = time.perf_counter()
            oracle.sort_dtype(sample, name, asc=not desc)
            tot += time.perf_counter() - t
        cpu = {"value": round(len(arrays) * m / tot / 1e9, 6), "unit": "Gkeys/s", "cores": 1,
               "kind": "oracle",
               "sample": f"first {m} keys of each of the {len(arrays)} arrays, keys + stable "
                         f"indices, single-threaded stable oracle, {tot:.1f} s"}

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
                     "traffic": None,
                     "kernel": "level_kernel<u32, idx>",
                     "launches": int(cap), "avg_launch_us": round(level_time_s / cap * 1e6, 3),
                     "level_time_share": round(level_time_s / elapsed, 4)},
        "cpu_baseline": cpu,
        "per_array": per_array,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
