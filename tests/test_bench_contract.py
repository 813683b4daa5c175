"""The bench's command-line contract and its committed counter record (CPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_record_matches_the_kernel_source():
    """profiles/gram_traffic.json was taken on the current matvec-pair source
    (so the bench reports its traffic rather than null) and its bytes follow
    from its own counters and copy-scaled factors."""
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "gram_traffic.json")))
    got = bench.traffic_record(rec["n"], rec["d"])
    assert got == rec["bytes_per_launch"]
    b = (rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_factor"] +
         rec["write_kib_per_dispatch"] * 1024 * rec["write_factor"])
    assert abs(b - rec["bytes_per_launch"]) <= 1e-3 * b
    assert rec["bytes_per_launch"] >= rec["algorithmic_bytes_per_launch"]
