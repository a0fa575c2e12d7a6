"""The benchmark's host-side pieces (no GPU): algorithmic byte counts, the
hash-gated reading of committed counter summaries, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_update():
    # population read + write, plus E read + write per cell (and a per-cell
    # weight field read)
    assert bench.bytes_per_update(64) == 8.125
    assert bench.bytes_per_update(16) == 8.5
    assert bench.bytes_per_update(64, per_cell_w=True) == 8.1875
    # reverse step: 12 B per update, 84 B (+4 with a weight field) per cell
    assert bench.adjoint_bytes_per_update(64) == 12.0 + 84.0 / 64
    assert bench.adjoint_bytes_per_update(64, per_cell_w=True) == 12.0 + 88.0 / 64


def test_committed_counter_summaries_match_the_kernel_sources():
    """Every traffic summary was taken on the kernel sources as committed (so
    the bench line reports it), and a summary read against other sources is
    ignored."""
    assert bench.recorded_traffic() is not None
    assert bench.recorded_traffic(bench.ADJOINT_TRAFFIC_FILE, bench.ADJOINT_SOURCES) is not None
    for path in bench.FUSED_TRAFFIC_FILES.values():
        assert bench.recorded_traffic(path, bench.FUSED_SOURCES) is not None
    assert bench.recorded_traffic(bench.TRAFFIC_FILE, bench.ADJOINT_SOURCES) is None
    assert bench.recorded_traffic(os.path.join(ROOT, "profiles", "missing.md")) is None


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
