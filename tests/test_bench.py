"""CPU checks of bench.py's contract: one GPU only, and the committed HBM
traffic summary belongs to the current level-kernel source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""                    # no JSON line


def test_traffic_summary_matches_kernel_source():
    """A committed counter summary must belong to the current level-kernel
    source (else bench.py reports traffic as null); when it does, the
    measured bytes are at least a fraction of the algorithmic bytes."""
    sys.path.insert(0, ROOT)
    import bench
    if not os.path.exists(bench.TRAFFIC_FILE):
        assert bench.measured_traffic() is None
        return
    t = bench.measured_traffic()
    assert t is not None, f"{bench.TRAFFIC_FILE} was taken on another kernel source"
    assert t > 0
