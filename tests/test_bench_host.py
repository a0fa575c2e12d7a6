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


def test_counter_summaries_are_hash_gated(tmp_path):
    """A traffic summary is read only if it was taken on the kernel sources
    as they are now (its recorded hash matches); otherwise the bench line
    reports no traffic."""
    good = tmp_path / "good.md"
    good.write_text("# summary\n"
                    f"- kernel_sha256_16: `{bench.kernel_hash()}`\n"
                    "- hbm_bytes_per_launch: `123456.0`\n")
    assert bench.recorded_traffic(str(good)) == 123456.0
    assert bench.recorded_traffic(str(good), bench.ADJOINT_SOURCES) is None
    stale = tmp_path / "stale.md"
    stale.write_text("- kernel_sha256_16: `0000000000000000`\n"
                     "- hbm_bytes_per_launch: `123456.0`\n")
    assert bench.recorded_traffic(str(stale)) is None
    assert bench.recorded_traffic(os.path.join(ROOT, "profiles", "missing.md")) is None


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
