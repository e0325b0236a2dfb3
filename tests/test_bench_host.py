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
    rec = {"sources_sha256_16": b.sources_digest(), "per_alg_byte": 0.25}
    monkeypatch.setitem(b.TRAFFIC, "c5", rec)
    assert b.recorded_traffic("no-such-workload", 1e9) is None
    assert b.recorded_traffic("c5", 1e9) == 0.25e9
    monkeypatch.setitem(b.TRAFFIC, "c5", dict(rec, sources_sha256_16="0" * 16))
    assert b.recorded_traffic("c5", 1e9) is None


def test_digest_covers_every_kernel_source_and_header():
    """Every file the intersection kernels are compiled from (the kernel sources
    and, transitively, every header they include) is in the digest the recorded
    traffic is keyed to: a change to any of them voids the record."""
    import re

    b = _bench()
    csrc = "paper_2103_14294_amd/csrc/"
    todo, seen = [csrc + "extend.hip", csrc + "mround.hip"], set()
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        for inc in re.findall(r'#include "([^"]+)"', open(os.path.join(ROOT, f)).read()):
            todo.append(os.path.normpath(os.path.join(os.path.dirname(f), inc)))
    assert seen <= set(b.KERNEL_SOURCES), seen - set(b.KERNEL_SOURCES)
    for f in b.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f


def test_heldout_patterns_are_outside_the_training_set():
    b = _bench()
    seen = b.training_patterns()
    qs = b.candidate_patterns(b.WORKLOADS["c5"])
    # every held-out class of 4-6 vertices is a candidate (fewer than the draw allows)
    assert b.WORKLOADS["c5"]["queries"][1]["count"] <= len(qs) <= b.WORKLOADS["c5"]["queries"][1]["draw"]
    assert len({(k, tuple(sorted(e))) for _, k, e in qs}) == len(qs)
    for name, k, e in qs:
        assert (k, tuple(sorted(e))) not in seen, name
        assert 4 <= k <= 6


def test_variants_workload_is_well_formed():
    """The variants line's items name patterns that exist, with one label per
    query vertex, and directed queries whose arcs join distinct query vertices
    of a connected skeleton."""
    from graphgen import patterns as P

    V = _bench().VARIANTS
    for name, ql in V["labelled"]:
        assert name in P.NAMED and len(ql) == P.NAMED[name][0], name
    for name in V["induced"] + V["oracle_motifs"]:
        assert name in P.NAMED, name
    for name in V["oracle_motifs"]:
        assert P.NAMED[name][0] in V["motif_k"], name
    for name, (k, arcs) in V["directed"].items():
        seen = {0}
        und = {tuple(sorted(a)) for a in arcs}
        assert all(a != b and 0 <= a < k and 0 <= b < k for a, b in arcs), name
        for _ in range(k):
            seen |= {b for a, b in und if a in seen} | {a for a, b in und if b in seen}
        assert seen == set(range(k)), name
