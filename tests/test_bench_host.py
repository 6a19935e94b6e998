"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic of
the dominant kernel, and the rule that recorded counter traffic is reported only
while the kernel source still hashes to the value recorded with it."""
import hashlib
import json
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
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_ksg_roofline_arithmetic():
    V, N, ms = 1_760_000, 1000, 48.0
    r = bench._roofline_of("ksg_field", {}, {"ksg_field": ms}, N, V)
    pairs = V * N * (N - 1)
    assert r["bound"] == "alu" and r["kernel"] == "ksg_field"
    assert r["achieved"] == pytest.approx(pairs / (ms * 1e-3) / 1e12)
    assert r["peak"] == pytest.approx(256 * 4 * 16 * 2.4e9 / 1e12 / 8)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "p.txt"
    prof.write_text(f"k.hip sha256 prefix at measurement: {sha[:16]}.\n"
                    "  traffic_bytes_per_launch: 1.5e+09   (algorithmic ...)\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_PMC_TRAFFIC", {"k": ("p.txt", "k.hip")})
    assert bench._measured_traffic("k") == pytest.approx(1.5e9)
    assert bench._measured_traffic("other") is None
    src.write_text("kernel v2\n")                       # source changed since the counters
    assert bench._measured_traffic("k") is None
    sha2 = hashlib.sha256(src.read_bytes()).hexdigest()
    prof.write_text(prof.read_text() +
                    f"k.hip sha256 prefix after a comment-only edit: {sha2[:16]}\n")
    assert bench._measured_traffic("k") == pytest.approx(1.5e9)


def test_recorded_ksg_traffic_matches_the_current_source():
    """The committed counter profile belongs to the committed KSG source."""
    t = bench._measured_traffic("ksg_field")
    assert t is not None and 1.0e10 < t < 1.3e10


def test_recorded_ksg_issue_rates():
    """The dominant kernel's measured VALU issue and lane occupancy come from the
    same hash-checked counter profile."""
    issue, lanes = bench._measured_issue("ksg_field")
    assert 0.5 < issue <= 1.0 and 0.5 < lanes <= 1.0
    r = bench._roofline_of("ksg_field", {}, {"ksg_field": 48.0}, 1000, 1_760_000)
    assert r["valu_issue_frac"] == issue and r["valu_lanes_active_frac"] == lanes
