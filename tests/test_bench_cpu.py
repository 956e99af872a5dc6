"""bench.py's contract that holds without a GPU: more than one GPU is refused
with a message and a non-zero status, and the committed HBM counter summary
it reports `roofline.traffic` from belongs to the current stage-kernel source
(a stale one would be silently ignored and report null)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_stored_traffic_matches_the_stage_kernel_source():
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["kernel_source_sha"] == bench.kernel_source_hash()
    tuned = {"nfast": 4, "threads": 192, "xblock": 0, "pipe": 0, "wgs_per_cu": 5, "walk_block": 3}
    traffic = bench.stored_traffic(tuned)
    assert traffic is not None and traffic > t["algorithmic_bytes_per_launch"]
    assert bench.stored_traffic(dict(tuned, threads=128)) is None  # a shape without counter runs
    assert bench.stored_traffic(tuned, real=False) is None  # the complex form has counters of its own
