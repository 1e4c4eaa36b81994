"""CPU: the benchmark's command line (no GPU work)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("points", [1024, 256, 64, 32, 16])
def test_kernel_hash_and_committed_traffic(points):
    """The committed PMC summaries were taken on the current level-kernel source."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_hash(points)
    assert len(h) == 16
    assert bench.read_traffic(points) is not None, f"profile for {points}-point rows is stale"


@pytest.mark.parametrize("name,points", [("k10_sieve_kernel_trace.txt", 1024),
                                         ("k10_narrow_c256_kernel_trace.txt", 256)])
def test_committed_kernel_traces_match_source(name, points):
    """The committed kernel-trace summaries name the source hash they were taken on."""
    sys.path.insert(0, ROOT)
    import bench
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert f"source hash: {bench.kernel_hash(points)}" in text, f"{name} is stale"
