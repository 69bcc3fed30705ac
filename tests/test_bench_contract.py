"""Host-side pieces of bench.py: the one-GPU guard and the reading of the
committed counter records (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_matches_only_current_sources(tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = {"bench_kernel": "rcmc_azimuth", "source_sha256": bench.kernel_source_hash(),
            "fetch_bytes": 100, "write_bytes": 50, "source": "x"}
    stale = dict(good, source_sha256="0" * 16, fetch_bytes=1)
    (prof / "a.md").write_text("text\ntraffic-record: " + json.dumps(stale) + "\n")
    d = str(prof)
    assert bench.recorded_traffic("rcmc_azimuth", d) is None       # stale hash only
    (prof / "b.md").write_text("traffic-record: " + json.dumps(good) + "\n")
    rec = bench.recorded_traffic("rcmc_azimuth", d)
    assert rec["fetch_bytes"] == 100 and rec["write_bytes"] == 50
    assert bench.recorded_traffic("range_fused", d) is None


def test_kernel_source_hash_covers_the_kernel_files():
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2604_03585_amd", "csrc", f)), f
    assert len(bench.kernel_source_hash()) == 16


def test_issue_record_matches_only_current_sources(tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = {"bench_kernel": "rcmc_azimuth", "source_sha256": bench.kernel_source_hash(),
            "valu_wave_instr": 1000, "trans_wave_instr": 10, "lds_wave_instr": 5,
            "lds_conflict_ratio": 1.5, "source": "x"}
    stale = dict(good, source_sha256="f" * 16)
    (prof / "a.md").write_text("issue-record: " + json.dumps(stale) + "\n"
                               "traffic-record: " + json.dumps(good) + "\n")
    d = str(prof)
    assert bench.recorded_issue("rcmc_azimuth", d) is None          # stale, other tag
    (prof / "b.md").write_text("issue-record: " + json.dumps(good) + "\n")
    assert bench.recorded_issue("rcmc_azimuth", d)["valu_wave_instr"] == 1000
