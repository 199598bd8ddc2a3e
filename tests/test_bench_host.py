"""Host side of the benchmark (no GPU): the oracle timings it reports.

* The single-core figure on the plain workload and the multi-process figure
  on the batch both run the oracle as it stands and report what they ran.
* `bench.py --gpus 2` refuses: the benchmark measures one GPU.
"""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_reports_the_plain_sample():
    r = bench.cpu_baseline(0.5)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "site-updates/s"
    assert r["value"] > 0 and "1024x1024" in r["sample"]


def test_cpu_batched_runs_one_process_per_core():
    r = bench.cpu_batched(0.5, cores=2)
    assert r["kind"] == "oracle" and r["cores"] == 2 and r["unit"] == "site-updates/s"
    assert r["value"] > 0 and "2 processes" in r["sample"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr) or "1 GPU" in (p.stdout + p.stderr)
