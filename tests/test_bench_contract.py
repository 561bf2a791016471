"""Host-side checks of bench.py's contract (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_bytes_of_the_large_workload():
    # the method's own bytes per row (band read + LU written for the factor
    # kernel); the design's G operator is reported apart as overhead
    n, k, m, r = 1 << 22, 32, 16, 8
    assert bench.algorithmic_bytes("factor_pass1", n, k, m, r, 8) == (8 * 65 + 8 * 65) * n
    assert bench.algorithmic_bytes("factor_pass1", n, k, m, r, 4) == (8 * 65 + 4 * 65) * n
    assert bench.algorithmic_bytes("factor_pass1", n, k, m, r, 8) == 1040 * n  # 4.36 GB at n = 2^22
    assert bench.design_overhead_bytes("factor_pass1", n, k, 8) == 8 * 32 * n
    # solve sweeps: factor words of the sweep pair plus the right-hand sides
    assert bench.algorithmic_bytes("dstage_kernel", n, k, m, r, 8) == (8 * 65 + 8 * m) * n
    assert bench.algorithmic_bytes("retrieve_kernel", n, k, m, r, 8) == (8 * 65 + 16 * m) * n
    # the W forward intermediate is written only when the spikes are truncated
    assert bench.algorithmic_bytes("spike_fwd", n, k, m, k, 8) == 8 * k * n
    assert bench.algorithmic_bytes("spike_fwd", n, k, m, r, 8) == 2 * 8 * k * n
    assert bench.algorithmic_bytes("no_such_kernel", n, k, m, r, 8) is None


def test_phase_bytes_of_the_large_workload():
    # factor 7.62 GB and solve 5.97 GB at n = 2^22, k = 32, 16 right-hand sides, FP64
    pb = bench.phase_bytes(1 << 22, 32, 16, 8)
    assert round(pb["factor"] / 1e9, 2) == 7.62
    assert round(pb["solve"] / 1e9, 2) == 5.97
