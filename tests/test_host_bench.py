"""Host checks of the benchmark driver (no GPU needed).

* More than one GPU is refused with a message and exit status 2: the path
  runs on a single device.
* The HBM traffic figures the benchmark reports (taken with rocprofv3
  counters) are tied to a digest of the kernel sources they were measured
  on: every stored figure matches the sources as committed, and a changed
  source turns the figure into null.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("kernel", sorted(bench.MEASURED_TRAFFIC))
def test_measured_traffic_matches_committed_sources(kernel):
    nbytes = bench.measured_traffic(kernel, "c5")
    assert nbytes == bench.MEASURED_TRAFFIC[kernel][2] and nbytes > 0
    # other workloads have no measured figure
    assert bench.measured_traffic(kernel, "c1") is None


def test_measured_traffic_null_after_a_source_change(monkeypatch):
    unit, digest, nbytes = bench.MEASURED_TRAFFIC["k_adj_strip/11"]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "k_adj_strip/11", (unit, "0" * 16, nbytes))
    assert bench.measured_traffic("k_adj_strip/11", "c5") is None
