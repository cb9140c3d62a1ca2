"""bench.py's contract on the host: more than one GPU is refused with a
message (the library measures one GPU), and the traffic figure is reported
only for the kernel sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_measured_sources(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    assert bench.traffic_for("fp64") is None
    monkeypatch.setitem(bench.TRAFFIC, "kernels_sha256", "0" * 64)
    assert bench.traffic_for("fp32") is None
