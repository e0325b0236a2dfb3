"""Host-side logic of bench.py (no GPU): the one-GPU guard and the recorded
HBM-traffic figure, which applies only to the kernel sources it was measured on
and scales with each run's algorithmic bytes per launch."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_recorded_traffic_needs_the_measured_sources(monkeypatch):
    b = _bench()
    rec = dict(b.TRAFFIC["c2"])
    assert b.recorded_traffic("no-such-workload", 1e9) is None
    monkeypatch.setitem(b.TRAFFIC, "c2", dict(rec, sources_sha256_16="0" * 16))
    assert b.recorded_traffic("c2", 1e9) is None


def test_recorded_traffic_scales_with_algorithmic_bytes(monkeypatch):
    import hashlib

    b = _bench()
    h = hashlib.sha256()
    for f in b.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    monkeypatch.setitem(b.TRAFFIC, "c2", {"sources_sha256_16": h.hexdigest()[:16], "bytes_per_launch": 1.0,
                                          "per_alg_byte": 0.25})
    assert b.recorded_traffic("c2", 4e9) == 1e9
    assert b.recorded_traffic("c2", 8e9) == 2e9
