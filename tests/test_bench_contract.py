"""Host-side parts of the benchmark's contract (no GPU): the one-GPU rule,
the algorithmic byte counts, and the HBM traffic figure read from the
committed counter summary."""
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
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_bytes():
    # inputs read once + outputs written once, per call of the large configuration
    assert bench.BYTES["scan_excl_i32_i64"] == (4 + 8) * 2 ** 27
    assert bench.BYTES["map_saxpy"] == (4 + 4 + 4) * 2 ** 26
    assert bench.BYTES["mapreduce_dot"] == (4 + 4) * 2 ** 26
    assert bench.BYTES["reduce_sum"] == 4 * 2 ** 26
    assert bench.BYTES["mapoverlap1d_5pt"] == (4 + 4) * 2 ** 26
    assert bench.BYTES["mapoverlap2d_9x9"] == (4 + 4) * 4096 * 4096
    assert set(bench.PLAIN) == set(bench.BYTES)


def test_traffic_figure_tracks_sources_and_variant():
    dom = bench.DOMINANT
    t = bench.traffic_from_profile(dom, bench.BYTES[dom], "S3_persistent_lookback")
    assert t is not None and abs(t / bench.BYTES[dom] - 1) < 0.01  # no wasted re-reads
    # counters taken on one variant say nothing about another
    assert bench.traffic_from_profile(dom, bench.BYTES[dom], "S2_decoupled_lookback") is None
    assert bench.traffic_from_profile("map_saxpy", bench.BYTES["map_saxpy"], "M2") is None
