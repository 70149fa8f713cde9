"""Host-side checks of bench.py (no GPU): the one-GPU contract and the
counter-derived traffic figure, which is reported only for the kernel source
and tile width its profile summary was taken on."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("tile_bits", [12, 14])
def test_traffic_only_for_the_profiled_tile_width(tile_bits):
    assert bench.measured_traffic(tile_bits) is None


def test_traffic_needs_the_profiled_kernel_source(monkeypatch):
    got = bench.measured_traffic(13)
    if got is not None:  # the summary matches the kernel source as built here
        assert 2.6e8 < got < 2.8e8  # one read and one write of a 128 MiB state, to within 4 %
    monkeypatch.setattr(bench, "kernel_source_digest", lambda *a, **k: "0" * 16)
    assert bench.measured_traffic(13) is None
