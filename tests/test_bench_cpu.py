"""Host-side checks of the benchmark script: the committed hardware byte counts belong to the
current select-and-sum source, and multi-GPU runs are refused with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_record_matches_kernel_source():
    import bench
    digest = bench.select_sum_source_digest()
    assert len(digest) == 64
    rec = bench.traffic_record("select_sum")
    assert rec is not None, "profiles/select_sum_traffic.json was taken on another kernel source"
    assert 0.9 < rec["traffic_over_algorithmic"] < 1.5
    assert rec["bytes_per_launch"] > rec["algorithmic_bytes_per_launch"] * 0.9


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
