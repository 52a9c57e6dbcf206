"""CPU checks of the benchmark's contract that need no GPU: more than one
GPU is refused with a message before anything touches a device, and the
algorithmic byte counts per pixel are those the passes move (Eq. 5 and
Eq. 4a fused between the transforms)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_pixel():
    sys.path.insert(0, ROOT)
    import bench
    # column pass: complex64 iterate in and out (8 + 8) and the float target
    assert bench.COL_BYTES_PER_PX == 8 + 8 + 4
    # row pass: complex64 iterate in and out
    assert bench.ROW_BYTES_PER_PX == 8 + 8
    assert bench.HBM_PEAK_GBS == 8000.0
