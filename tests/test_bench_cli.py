"""bench.py's host-side contract without a GPU: more than one GPU is
refused with a message, unknown extras groups are refused before any work,
the source hash that guards the committed traffic figure is stable, and the
counter summariser turns two counter files into the traffic lines."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_unknown_extras_group_is_refused():
    r = run("--extras", "in_place,nope")
    assert r.returncode == 2
    assert "nope" in r.stderr


def test_source_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.source_hash()
    assert h == bench.source_hash() and len(h) == 16


def test_counter_summary(tmp_path):
    """Two minimal counter CSVs (a calibration dispatch and two level
    launches) give per-launch bytes scaled by the calibration."""
    sys.path.insert(0, ROOT)
    import bench
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    calib_bytes = bench.CALIB_ELEMS * 4
    lvl = '"void bsort::level_kernel<unsigned int, true, 512, 8>(x)"'
    cal = '"void at::native::elementwise_kernel<bitwise_not>"'
    rows_f = [f"1,{cal},FETCH_SIZE,{calib_bytes / 2 / 1024}",
              f"2,{lvl},FETCH_SIZE,1000", f"3,{lvl},FETCH_SIZE,3000"]
    rows_w = [f"1,{cal},WRITE_SIZE,{calib_bytes / 1024}",
              f"2,{lvl},WRITE_SIZE,500", f"3,{lvl},WRITE_SIZE,1500"]
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    f.write_text(head + "\n".join(rows_f) + "\n")
    w.write_text(head + "\n".join(rows_w) + "\n")
    out = bench.summarize_pmc(str(f), str(w))
    vals = dict(line.split(": ", 1) for line in out.strip().splitlines())
    assert vals["level_launches"] == "2"
    assert abs(float(vals["fetch_scale"]) - 2.0) < 1e-3
    assert abs(float(vals["write_scale"]) - 1.0) < 1e-3
    # (1000 + 3000) KiB fetched x 2, (500 + 1500) KiB written, over 2 launches
    assert int(float(vals["level_fetch_bytes_per_launch"])) == 4000 * 1024
    assert int(float(vals["level_write_bytes_per_launch"])) == 1000 * 1024


def test_cpu_baseline_leg_small():
    """The CPU-baseline leg on small arrays: whole arrays timed with both
    oracle flavours on pinned threads, the pool over a batch and rows, and
    the host description.  The process's own affinity is left alone."""
    import numpy as np
    import bench
    from paper_2603_08929_amd import workloads as W
    before = os.sched_getaffinity(0)
    arrays = [("i32_uniform", "i32", W.uniform_bits("i32", 4096, 0), False),
              ("u32_reverse_desc", "u32", W.presorted_u32(4096, 0, reverse=True), True)]
    r = bench.cpu_baseline(arrays, pool=True,
                           batch=[W.normal_bits("f32", 100 + i, i) for i in range(20)],
                           rows=[("f16", 8, 256)])
    assert os.sched_getaffinity(0) == before
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert r["lomuto"]["value"] > 0
    assert set(r["per_array_s"]) == {"i32_uniform", "u32_reverse_desc"}
    assert r["host"]["cores_available"] == len(before) and r["host"]["cpu_model"]
    assert r["pool"]["threads"] == min(16, len(before))
    assert r["pool"]["batched_f32"]["arrays"] == 20
    assert r["pool"]["rows_f16_8x256"]["keys"] == 8 * 256
