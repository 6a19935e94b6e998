"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic of
the learned-field kernel behind `value` and of the KSG field kernel, the
percentile summary, the coarse-grid interpolation of the equal-time baseline,
and the rule that recorded counter figures are reported only while the kernel
sources still hash to the values recorded with them."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_value_roofline_is_the_learned_field_kernel():
    r = bench._value_roofline({"ndf_field": 0.25})
    flops = 2.0 * 69760 * 1_760_000
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 2500.0
    assert r["achieved"] == pytest.approx(flops / 0.25e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 2500.0) and 0 < r["frac"] < 1


def test_ksg_roofline_is_a_lane_op_fraction():
    V, N, ms = 1_760_000, 1000, 48.0
    r = bench._ksg_roofline(ms, N, V)
    assert r["bound"] == "alu" and r["unit"] == "T lane-ops/s"
    assert r["peak"] == pytest.approx(256 * 4 * 16 * 2.4e9 / 1e12)
    assert r["brute_force_equivalent_pair_evals_per_s"] == pytest.approx(V * N * (N - 1) / 48e-3)
    # the lane operations come from the hash-checked counter profile
    assert r["achieved"] is not None and 0 < r["frac"] <= 1
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert 0 < r["lds_bank_conflict_frac"] < 1


def test_stats_and_coarse_upsampling():
    st = bench._stats(list(range(1, 101)))
    assert st["median"] == 50.5 and st["p10"] == pytest.approx(10.9) and st["n"] == 100
    # trilinear upsampling reproduces a field affine in (i, j, k) exactly
    import gen
    cfg = gen.CONFIGS["mid"]
    axes = [bench._coarse_axis(cfg.nx, 5), bench._coarse_axis(cfg.ny, 5),
            bench._coarse_axis(cfg.nz, 5)]
    assert axes[0][0] == 0 and axes[0][-1] == cfg.nx - 1
    iz, iy, ix = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    f = (0.5 * ix - 2.0 * iy + 3.0 * iz + 1.0).reshape(-1)
    v = np.arange(cfg.n_vertices)
    i, j, k = v % cfg.nx, (v // cfg.nx) % cfg.ny, v // (cfg.nx * cfg.ny)
    np.testing.assert_allclose(bench._upsample(f, axes, v, cfg),
                               0.5 * i - 2.0 * j + 3.0 * k + 1.0, atol=1e-12)


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "p.txt"
    prof.write_text(f"k.hip sha256 prefix at measurement: {sha[:16]}.\n"
                    "  traffic_bytes_per_launch: 1.5e+09   (algorithmic ...)\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_PMC_TRAFFIC", {"k": ("p.txt", ["k.hip"])})
    assert bench._measured_traffic("k") == pytest.approx(1.5e9)
    assert bench._measured_traffic("other") is None
    src.write_text("kernel v2\n")                       # source changed since the counters
    assert bench._measured_traffic("k") is None
    sha2 = hashlib.sha256(src.read_bytes()).hexdigest()
    prof.write_text(prof.read_text() +
                    f"k.hip sha256 prefix after a comment-only edit: {sha2[:16]}\n")
    assert bench._measured_traffic("k") == pytest.approx(1.5e9)
    src.write_text("kernel  v2\n")
    assert bench._measured_traffic("k") is None
    sha3 = hashlib.sha256(src.read_bytes()).hexdigest()
    prof.write_text(prof.read_text() +
                    f"k.hip sha256 prefix after a whitespace-only edit: {sha3[:16]}\n")
    assert bench._measured_traffic("k") == pytest.approx(1.5e9)


def test_recorded_ksg_traffic_matches_the_current_source():
    """The committed counter profile belongs to the committed KSG source."""
    t = bench._measured_traffic("ksg_field")
    assert t is not None and 1.0e10 < t < 1.3e10


def test_recorded_ksg_issue_rates():
    """The KSG kernel's measured VALU issue and lane occupancy come from the same
    hash-checked counter profile."""
    issue, lanes = bench._measured_issue("ksg_field")
    assert 0.5 < issue <= 1.0 and 0.5 < lanes <= 1.0
    r = bench._ksg_roofline(48.0, 1000, 1_760_000)
    assert r["valu_issue_frac"] == issue and r["valu_lanes_active_frac"] == lanes


def test_tagged_traffic_lines(tmp_path, monkeypatch):
    """A profile of several kernels tags each traffic line with its row; a row reads
    its own line, and an untagged line serves a profile of one kernel."""
    src = tmp_path / "k.hip"
    src.write_text("kernel\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "p.txt"
    prof.write_text(f"k.hip sha256 prefix at measurement: {sha[:16]}\n"
                    "  traffic_bytes_per_launch[a]: 1.0e+09\n"
                    "  traffic_bytes_per_launch[b]: 2.0e+09\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_PMC_TRAFFIC", {r: ("p.txt", ["k.hip"]) for r in "abc"})
    assert bench._measured_traffic("a") == pytest.approx(1.0e9)
    assert bench._measured_traffic("b") == pytest.approx(2.0e9)
    assert bench._measured_traffic("c") is None


def test_recorded_traffic_matches_the_current_sources():
    """Every committed counter profile the benchmark reports belongs to the committed
    kernel sources (else the benchmark would report the row's traffic as null)."""
    for row, lo, hi in (("ndf_field", 0.9e8, 1.2e8), ("ndf_field_fp8", 0.9e8, 1.2e8),
                        ("pearson_b64", 7.0e9, 8.0e9), ("pearson_b256", 8.5e9, 9.5e9),
                        ("train_step", 4.0e9, 6.0e9)):
        t = bench._measured_traffic(row)
        assert t is not None and lo < t < hi, (row, t)
