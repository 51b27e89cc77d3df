"""Host-side checks of bench.py: the one-GPU contract, the traffic lookup
that only trusts counter summaries taken on the current kernel source, and
the algorithmic-bytes formula."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_read_only_for_the_current_source(tmp_path, monkeypatch):
    import hashlib
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "paper_1511_06441_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "csp.hip").write_bytes(b"// kernel source\n")
    good = hashlib.sha256(b"// kernel source\n").hexdigest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # a summary recorded for this source is used
    (prof / "k_ranges3_cube128_traffic.md").write_text(
        "traffic_bytes_per_launch: 1.5e9\ncsp_hip_sha256: " + good + "\n")
    assert bench.measured_traffic("cube128") == 1.5e9
    # one recorded for another source is ignored
    (prof / "k_ranges3_cube128_traffic.md").write_text(
        "traffic_bytes_per_launch: 1.5e9\ncsp_hip_sha256: " + "0" * 64 + "\n")
    assert bench.measured_traffic("cube128") is None
    assert bench.measured_traffic("square64") is None           # no summary at all


@pytest.mark.parametrize("N,c,expect", [
    (10, dict(U=0, D=0, E=0, R=0), 40),
    (1, dict(U=1, D=1, E=1, R=1), 4 + 4 + 6 + 8 + 16),
])
def test_algorithmic_bytes(N, c, expect):
    assert bench.algorithmic_bytes(N, c) == expect
