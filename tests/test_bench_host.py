"""Host-side checks of bench.py (no GPU): the one-GPU contract and the rule
that profiled HBM traffic is reported only for the launch it was taken on."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _profile(tmp_path, tag, khash, alg, measured):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    (d / f"conv_traffic_{tag}.json").write_text(json.dumps(
        {"kernel_sha256_16": khash, "algorithmic_bytes_per_launch": alg,
         "bytes_per_launch": measured}))


def test_traffic_only_for_the_profiled_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "abc")
    _profile(tmp_path, "seamount-N8192", "abc", 48777184.0, 50680115)
    assert bench.traffic_from_profiles("seamount-N8192", False, 48777184.0) == 50680115
    # another form, other bytes, another kernel source, no profile: null
    assert bench.traffic_from_profiles("seamount-N8192", True, 48777184.0) is None
    assert bench.traffic_from_profiles("seamount-N8192", False, 12345.0) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "def")
    assert bench.traffic_from_profiles("seamount-N8192", False, 48777184.0) is None
    assert bench.traffic_from_profiles("rough-N65536", False, 1.0) is None
    # a closure profile is looked up under its own name
    monkeypatch.setattr(bench, "kernel_hash", lambda: "abc")
    _profile(tmp_path, "rough-N65536-closure", "abc", 132453280.0, 140000000)
    assert bench.traffic_from_profiles("rough-N65536", True, 132453280.0) == 140000000
    # counters taken on one conv tile do not stand for a run on another
    (tmp_path / "profiles" / "conv_traffic_rough-N65536.json").write_text(json.dumps(
        {"kernel_sha256_16": "abc", "algorithmic_bytes_per_launch": 5.0,
         "bytes_per_launch": 6, "conv_tile": 512}))
    assert bench.traffic_from_profiles("rough-N65536", False, 5.0, 512) == 6
    assert bench.traffic_from_profiles("rough-N65536", False, 5.0, 1024) is None
    # counters of another tile sit in a file of their own
    (tmp_path / "profiles" / "conv_traffic_rough-N65536_tile1024.json").write_text(json.dumps(
        {"kernel_sha256_16": "abc", "algorithmic_bytes_per_launch": 5.0,
         "bytes_per_launch": 7, "conv_tile": 1024}))
    assert bench.traffic_from_profiles("rough-N65536", False, 5.0, 1024) == 7
    assert bench.traffic_from_profiles("rough-N65536", False, 5.0, 512) == 6
    assert bench.traffic_from_profiles("rough-N65536", True, 5.0, 1024) is None
    # the variable-step conv's counters sit under their own prefix
    (tmp_path / "profiles" / "var_traffic_sine-cycle-N4096.json").write_text(json.dumps(
        {"kernel_sha256_16": "abc", "algorithmic_bytes_per_launch": 43415915.9,
         "bytes_per_launch": 61878122}))
    assert bench.traffic_from_profiles("sine-cycle-N4096", False, 43415915.9,
                                       prefix="var_traffic_") == 61878122
    assert bench.traffic_from_profiles("sine-cycle-N4096", False, 43415915.9) is None
    assert bench.traffic_from_profiles("sine-cycle-N4096", False, 43415916.9,
                                       prefix="var_traffic_") is None


def test_committed_traffic_profiles_match_their_algorithmic_bytes():
    """The committed counter summaries carry the launch's algorithmic bytes
    and a measured traffic within a few percent of them (no re-reads)."""
    d = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(d) if f.startswith("conv_traffic_") and f.endswith(".json")]
    assert files
    for f in files:
        with open(os.path.join(d, f)) as fh:
            z = json.load(fh)
        ratio = z["bytes_per_launch"] / z["algorithmic_bytes_per_launch"]
        assert 1.0 <= ratio < 1.1, (f, ratio)
        assert len(z["kernel_sha256_16"]) == 16


def test_committed_variable_step_traffic():
    """The variable-step conv's counter summary: its algorithmic bytes are
    the records inside the windows only; the kernel also fetches the records
    of a live tile's slots past the window (requested before the window test,
    weighed zero), so its traffic is above them, but within 1.5 times."""
    with open(os.path.join(ROOT, "profiles", "var_traffic_sine-cycle-N4096.json")) as fh:
        z = json.load(fh)
    ratio = z["bytes_per_launch"] / z["algorithmic_bytes_per_launch"]
    assert 1.0 <= ratio < 1.5, ratio
    assert z["dispatches"][0] == z["dispatches"][1] > 0
    assert len(z["kernel_sha256_16"]) == 16
