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


def test_union_frontier_totals_brute_force():
    """The batch's union-frontier totals against a per-level enumeration."""
    import numpy as np
    import bench
    rng = np.random.default_rng(0)
    for q, n in ((1, 30), (7, 50), (64, 40)):
        L = rng.integers(-1, 6, size=(q, n)).astype(np.int32)
        deg = rng.integers(0, 10, size=n).astype(np.int64)
        f, d = bench.union_frontier_totals(L, deg)
        want_f = want_d = 0
        for k in range(6):
            F = [v for v in range(n) if any(L[i, v] == k for i in range(q))]
            want_f += len(F)
            want_d += int(sum(deg[v] for v in F))
        assert (f, d) == (want_f, want_d)
    # the bytes: 4 B per column entry + 8 B per 64-source mask word per entry,
    # 8 B of pointers per union-frontier vertex, 8 B per (vertex, source) output
    assert bench.batch_bytes(64, 10, 3, 5) == 12 * 5 + 8 * 3 + 8 * 64 * 10
    assert bench.batch_bytes(65, 10, 3, 5) == 20 * 5 + 8 * 3 + 8 * 65 * 10
