"""Host logic of bench.py's report (no GPU): the roofline entries, the rule
that counter-measured traffic and VALU issue are reported only while the
kernel sources match the digest they were taken on, and the one-GPU limit."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_digest_ignores_comments_and_whitespace_only(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "a.hip").write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    (tmp_path / "b.hip").write_text("/* doc */ int f(int x)\n{ return x + 1; }\n")
    (tmp_path / "c.hip").write_text("int f(int x) { return x + 2; }\n")
    assert bench._source_digest(["a.hip"]) == bench._source_digest(["b.hip"])
    assert bench._source_digest(["a.hip"]) != bench._source_digest(["c.hip"])


def test_traffic_and_valu_follow_the_source_digest(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    digest = bench._source_digest(bench.KERNEL_SOURCES["features"])
    assert bench._traffic("w", "features") is None  # no file
    assert bench._valu_issue(1.0, "w", "features") is None
    (tmp_path / "w_features_traffic.json").write_text(
        json.dumps({"source_digest": digest, "bytes_per_launch": 123.0}))
    (tmp_path / "w_features_valu.json").write_text(
        json.dumps({"source_digest": digest, "sq_insts_valu_per_dispatch": 6.144e8}))
    assert bench._traffic("w", "features") == 123.0
    v = bench._valu_issue(1.0, "w", "features")  # 6.144e8 instructions in 1 ms
    assert v["achieved"] == pytest.approx(614.4) and v["frac"] == pytest.approx(1.0)
    (tmp_path / "w_features_traffic.json").write_text(
        json.dumps({"source_digest": "0" * 16, "bytes_per_launch": 123.0}))
    (tmp_path / "w_features_valu.json").write_text(
        json.dumps({"source_digest": "0" * 16, "sq_insts_valu_per_dispatch": 6.144e8}))
    assert bench._traffic("w", "features") is None  # taken on other sources
    assert bench._valu_issue(1.0, "w", "features") is None


def test_kernel_entries_and_roofline(monkeypatch):
    monkeypatch.setattr(bench, "_traffic", lambda wl, k: None)
    monkeypatch.setattr(bench, "_valu_issue", lambda ms, wl, k: None)
    feat = bench._kernel_entry(0.8, "hbm", 1.6e9, "ragged", "features")
    score = bench._kernel_entry(1.6, "mfma", 2.0 * 16384 * 1024 * 7552, "ragged", "score")
    assert feat["achieved"] == pytest.approx(2000.0)  # GB/s
    assert feat["frac"] == pytest.approx(2000.0 / 8000.0)
    assert score["achieved"] == pytest.approx(2.0 * 16384 * 1024 * 7552 / 1.6e-3 / 1e12)
    assert score["frac"] == pytest.approx(score["achieved"] / 157.3)
    roof = bench._roofline({"features": feat, "score_fp32": score})
    assert roof["kernel"] == "score_fp32" and roof["bound"] == "mfma"  # the slower kernel
    assert set(roof) == {"kernel", "bound", "achieved", "peak", "unit", "frac", "traffic"}


def test_committed_counters_match_the_current_sources():
    """The traffic and VALU files under profiles/ were taken on the kernel
    sources as they are (otherwise the bench line reports them as null)."""
    for wl in ("ragged", "uniform"):
        assert bench._traffic(wl, "features") is not None
        assert bench._traffic(wl, "score") is not None
        assert bench._valu_issue(1.0, wl, "features") is not None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stdout + r.stderr
