"""bench.py's contract on the host: one GPU only (a request for more exits
with a message before touching a device), and the committed HBM-traffic
summary of the packed local apply belongs to the current kernel source, so
the bench line carries its `traffic` figure."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_profile_matches_kernel_source():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.pop(0)
    t = bench.measured_traffic("C4", "fp32", "inverse")
    # a kernel edit makes the summary stale (bench.py then reports traffic null): re-take it
    assert t is not None, "profiles/k_symv_C4_fp32_hbm_traffic.md was taken on another kern_symv.hip: re-take it"
    # at least the algorithmic bytes of one C4 FP32 apply (2.43 GB), at most 10% above them
    assert 2.43e9 <= t <= 1.1 * 2.432e9
