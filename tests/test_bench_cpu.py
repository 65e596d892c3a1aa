"""Host-side logic of bench.py: the one-GPU guard and the counter-traffic
lookup (no GPU, no torch import)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line for a configuration that was not measured


def _profile(tmp_path, sha, fetch_kib, write_kib, cal_fetch_kib, cal_write_kib):
    d = {
        "kernel_source_sha": sha,
        "fetch_kib": fetch_kib,
        "write_kib": write_kib,
        "copy_calibration": {"bytes_each_way": 1 << 30, "fetch_kib": cal_fetch_kib,
                             "write_kib": cal_write_kib},
    }
    (tmp_path / "lut_apply_w_pmc.json").write_text(json.dumps(d))


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    # A 1 GiB copy that reads as half its bytes on FETCH_SIZE and exactly its
    # bytes on WRITE_SIZE: fetch counts double, writes count once.
    _profile(tmp_path, bench.kernel_source_hash(), 1000.0, 3000.0, 524288.0, 1048576.0)
    assert bench.load_traffic("w") == round(1000.0 * 1024 * 2 + 3000.0 * 1024)


def test_traffic_is_dropped_once_the_kernel_source_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    _profile(tmp_path, "0" * 16, 1000.0, 3000.0, 524288.0, 1048576.0)
    assert bench.load_traffic("w") is None
    assert bench.load_traffic("missing") is None


def test_committed_counters_match_the_algorithmic_bytes():
    # The committed workload-1 counters, if taken on the current source, must
    # describe a correction launch: within a few per cent of its 4 B per pixel
    # plus the LUT read once.
    t = bench.load_traffic("4x12000x12000_L1024_quadratic")
    if t is None:
        pytest.skip("counters were taken on another kernel source")
    algorithmic = 4 * 12000 * 12000 * 4 + 4 * 12000 * 1024 * 2
    assert 1.0 <= t / algorithmic < 1.05
