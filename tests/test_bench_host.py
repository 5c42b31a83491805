"""Host logic of the benchmark script (CPU): the one-GPU guard, the per-kernel
summary of rocprofv3 CSVs that the committed profile summaries are made
with, and the overlap measure of a kernel trace.  The CSVs are small
synthetic files with rocprofv3's column names."""
from __future__ import annotations

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)
    return str(path)


TRACE_FIELDS = ["Dispatch_Id", "Kernel_Name", "Queue_Id", "Start_Timestamp", "End_Timestamp"]


def _trace_row(d, name, q, t0, t1):
    return {"Dispatch_Id": d, "Kernel_Name": name, "Queue_Id": q, "Start_Timestamp": t0, "End_Timestamp": t1}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    line = [x for x in r.stdout.splitlines() if x.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]


def test_counter_summary_of_a_kernel_trace(tmp_path):
    rows = [
        _trace_row(1, "hp::assemble_kernel<float>(int, ...)", 1, 0, 1000),
        _trace_row(2, "hp::gemm_direct_kernel<false, 1, 16, 2, false>(int, ...)", 1, 1000, 3000),
        _trace_row(3, "hp::panel_kernel<float>(int, ...)", 2, 1500, 2500),
        _trace_row(4, "hp::gemm_direct_kernel<false, 1, 16, 2, false>(int, ...)", 1, 3000, 7000),
        _trace_row(5, "hp::residual_local_kernel(int, ...)", 1, 7000, 7500),
        _trace_row(6, "hp::gemm_direct_kernel<false, 1, 16, 2, false>(int, ...)", 1, 8000, 8100),
    ]
    p = _write(tmp_path / "k.csv", TRACE_FIELDS, rows)
    g = "hp::gemm_direct_kernel<false, 1, 16, 2, false>"
    allk = bench.counter_summary(p)
    assert allk[g]["dispatches"] == 3 and allk[g]["counters"]["DurationNs"] == 2000 + 4000 + 100
    assert allk["hp::panel_kernel<float>"]["counters"]["DurationNs"] == 1000
    # a name filter, and a window from the assembly to the first residual
    only = bench.counter_summary(p, kernel="gemm_direct")
    assert set(only) == {g}
    win = bench.counter_summary(p, kernel="gemm_direct", window=("assemble_kernel", "residual_local_kernel"))
    assert win[g]["dispatches"] == 2 and win[g]["counters"]["DurationNs"] == 6000


def test_counter_summary_of_pmc_rows(tmp_path):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = []
    for d, kb in ((1, 100.0), (2, 300.0)):
        # one row per dispatch and counter instance: values of a dispatch add up
        rows.append({"Dispatch_Id": d, "Kernel_Name": "hp::copy_rows_kernel<float>(x)",
                     "Counter_Name": "FETCH_SIZE", "Counter_Value": kb / 2})
        rows.append({"Dispatch_Id": d, "Kernel_Name": "hp::copy_rows_kernel<float>(x)",
                     "Counter_Name": "FETCH_SIZE", "Counter_Value": kb / 2})
    p = _write(tmp_path / "c.csv", fields, rows)
    s = bench.counter_summary(p)
    e = s["hp::copy_rows_kernel<float>"]
    assert e["dispatches"] == 2 and e["counters"]["FETCH_SIZE"] == pytest.approx(400.0)


def test_trace_overlap_counts_concurrent_queues(tmp_path):
    rows = [
        # single-system panels on queue 1: [0, 10) and [20, 30)
        _trace_row(1, "hp::panel_kernel<float>(int)", 1, 0, 10),
        _trace_row(2, "hp::panel_finish_kernel<float>(int)", 1, 20, 30),
        # a batched trailing update on queue 2: [5, 25) overlaps both
        _trace_row(3, "hp::batch_trail_kernel<float>(int)", 2, 5, 25),
        # another batched step on queue 3, alone: [40, 50)
        _trace_row(4, "hp::batch_panel_kernel<float>(int)", 3, 40, 50),
        # not a factorization kernel: ignored
        _trace_row(5, "hp::assemble_kernel<float>(int)", 4, 0, 100),
    ]
    p = _write(tmp_path / "t.csv", TRACE_FIELDS, rows)
    o = bench.trace_overlap(p)
    assert o["ms_any_running"] == pytest.approx(40 / 1e6)
    assert o["ms_two_or_more_queues"] == pytest.approx(10 / 1e6)
    assert o["ms_batched_and_single_system"] == pytest.approx(10 / 1e6)
    assert o["factorization_kernels"] == {"batched queue 2": 1, "batched queue 3": 1, "single queue 1": 2}
