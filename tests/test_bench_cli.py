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


@pytest.mark.parametrize("N,c,L,expect", [
    (10, dict(U=0, D=0, E=0, R=0), 4, 40),
    (1, dict(U=1, D=1, E=1, R=1), 4, 4 + 4 + 6 + 8 + 16),
    (1, dict(U=1, D=1, E=1, R=1), 2, 2 + 2 + 4 + 8 + 12),
])
def test_algorithmic_bytes(N, c, L, expect):
    assert bench.algorithmic_bytes(N, c, L) == expect


def test_label_width_follows_the_workload():
    """Configurations with 16-bit labels count 2-byte label traffic; the
    256^3 cubes count 4 bytes."""
    assert bench.WORKLOADS["square64"]["label_bytes"] == 2
    assert bench.WORKLOADS["cube128"]["label_bytes"] == 2
    assert bench.WORKLOADS["cube256"]["label_bytes"] == 4
    assert bench.WORKLOADS["cube256stress"]["label_bytes"] == 4


def test_cpu_window_sample_is_bounded():
    """The 256^3 CPU sample is a window of cycles (two prefix runs), not a
    whole solve."""
    k1, k2 = bench.WORKLOADS["cube256"]["sample_cycles"]
    assert 0 < k1 < k2 <= 2000


def test_batch_cpu_sample_is_bounded():
    """The batch's CPU sample is every 64th problem (16 of 1,024), a few
    million vertices in all, and the default bench line takes it."""
    import inspect
    from paper_1511_06441_amd import inputs as gen
    step = inspect.signature(bench.cpu_baseline_batch).parameters["step"].default
    js = range(0, 1024, step)
    assert len(js) == 16
    verts = sum(n ** d for (_, d, n, _, _) in (gen.mixed_params(41, j) for j in js))
    assert verts < 6_000_000
