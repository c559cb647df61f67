"""Host-side pieces of bench.py that need no GPU: the traffic record it
reports only while the library sources match, and the single-GPU guard."""
import subprocess
import sys

import pytest

import bench


def test_traffic_record_matches_sources():
    """The committed traffic record parses; bench.py reports it only while it
    was taken with the current library sources (skipped, not failed, after a
    change to the sources: the counters then have to be taken again)."""
    import glob
    import os
    files = glob.glob(os.path.join(bench.PROFILES, "*_traffic_*.md"))
    assert files
    for path in files:
        text = open(path).read()
        assert "traffic_bytes_per_launch:" in text and "library_source_sha256:" in text
    t = bench.recorded_traffic("cube1048576", "matvec")
    if t is None:
        pytest.skip("traffic record taken with other library sources")
    assert 1e6 < t < 1e13  # bytes per launch: above the inputs, below ~1 s of HBM time


def test_traffic_record_rejected_on_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "library_source_hash", lambda kernel="": "0" * 64)
    assert bench.recorded_traffic("cube1048576", "matvec") is None
    assert bench.recorded_traffic("cube2048") is None


def test_source_hash_is_stable():
    assert bench.library_source_hash() == bench.library_source_hash()
    assert len(bench.library_source_hash()) == 64
    # a family with its own sources hashes only those
    assert bench.library_source_hash("matvec") != bench.library_source_hash()
    assert bench.library_source_hash("gemm_f64") == bench.library_source_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_predicted_form_defaults():
    """The benchmark's learned-rank defaults: capped boxes sketched at the full
    width m - 8 (oversampling leaf - 8 - ceil(1.25 cap), 8 without a cap), and
    levels 1-7 on the full pivoted QR."""
    import workloads as W
    assert bench.default_oversample(W.cube1m()) == 256 - 8 - 160
    assert bench.default_oversample(W.small_cube()) == 64 - 8 - 40
    assert bench.SKETCH_MIN_LEVEL == 8
    import argparse
    assert bench.default_oversample(argparse.Namespace(leaf=256, rank_cap=0)) == 8
