"""Host-side parts of bench.py's contract: it measures one GPU and refuses
--gpus N > 1 before touching a device, its roofline entries are the
algorithmic work over the measured time against the stated peak, and the
HBM traffic figure is reported only for the kernel sources it was taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bad_step_counts_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "0"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0 and r.stdout == ""


def test_roofline_entry_is_work_over_time_against_the_peak():
    # 2.5e12 FLOP in 2 ms = 1.25e15 FLOP/s = 1250 TFLOP/s, half of 2.5 PFLOP/s
    e = bench.roof(2.0, 2.5e12, 2.5e15, "TFLOP/s", "mfma", "test")
    assert e["achieved"] == pytest.approx(1250.0)
    assert e["peak"] == pytest.approx(2500.0)
    assert e["frac"] == pytest.approx(0.5)
    # 4e9 bytes in 1 ms = 4 TB/s = 4000 GB/s, half of 8 TB/s
    e = bench.roof(1.0, 4e9, 8e12, "GB/s", "hbm", "test")
    assert e["achieved"] == pytest.approx(4000.0) and e["frac"] == pytest.approx(0.5)


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    assert bench.sources_hash(bench.NN_TRAFFIC_SOURCES) == bench.sources_hash(tuple(bench.NN_TRAFFIC_SOURCES))
    monkeypatch.setattr(bench, "NN_TRAFFIC_HASH", bench.sources_hash(bench.NN_TRAFFIC_SOURCES))
    assert bench.nn_traffic() == bench.NN_TRAFFIC_BYTES
    monkeypatch.setattr(bench, "NN_TRAFFIC_HASH", "0" * 16)
    assert bench.nn_traffic() is None
