"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message before anything touches a device, and the kernel-source hash
that guards the committed HBM-traffic counters is stable and content-based."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.kernel_source_hash()
    b = bench.kernel_source_hash()
    assert a == b and len(a) == 64
