"""Host-side tests of the C ABI: every declared symbol is exported, and the
planner (host only) validates queries and orders and derives the
symmetry-breaking constraints.  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from graphgen import patterns as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def H():
    import paper_2103_14294_amd as H

    if not os.path.exists(H.LIB_PATH):
        from paper_2103_14294_amd import build as hb

        hb.build()
    H.load_library()
    return H


def _declared():
    txt = open(os.path.join(ROOT, "include", "huge.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(huge_[a-z0-9_]+)\s*\(", txt))
    names.discard("huge_emit_fn")
    return sorted(names)


def test_every_declared_symbol_is_exported(H):
    names = _declared()
    assert len(names) >= 13
    lib = ctypes.CDLL(H.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(H.EXPORTED) <= set(names)


def test_exec_opts_defaults(H):
    o = H.ExecOpts()
    assert H.load_library().huge_exec_opts_default(ctypes.byref(o)) == 0
    assert o.frontier_cap_bytes == 4 << 30
    assert o.strategy == -1 and o.engine == 0 and o.slice_count == 1 and o.work_stealing == 1
    assert H.load_library().huge_exec_opts_default(None) == -1


@pytest.mark.parametrize("k,edges,err", [
    (1, [(0, 0)], "HUGE_EQUERY"),
    (9, [(i, i + 1) for i in range(8)], "HUGE_EQUERY"),
    (3, [(0, 0), (1, 2)], "HUGE_EQUERY"),
    (3, [(0, 1), (1, 0), (1, 2)], "HUGE_EQUERY"),
    (4, [(0, 1), (2, 3)], "HUGE_EQUERY"),
    (3, [(0, 1), (1, 3)], "HUGE_EQUERY"),
])
def test_bad_queries_rejected(H, k, edges, err):
    with pytest.raises(H.HugeError) as ei:
        H.plan(None, k, edges)
    assert ei.value.name == err
    assert H.load_library().huge_last_error()


@pytest.mark.parametrize("order", [(0, 1, 2, 2), (0, 2, 1, 3), (0, 1, 2, 9)])
def test_bad_orders_rejected(H, order):
    k, e = P.NAMED["4-path"]  # 0-1-2-3
    with pytest.raises(H.HugeError) as ei:
        H.plan(None, k, e, order=order)
    assert ei.value.name == "HUGE_EORDER"


def test_constraints_match_oracle_grochow_kellis(H):
    pats = [P.NAMED[n] for n in P.NAMED] + [(p["k"], p["edges"]) for p in P.random_patterns(40, seed=5, kmin=3, kmax=7)]
    for k, e in pats:
        info = H.plan(None, k, e).info()
        assert sorted(info["sb_pairs"]) == sorted(oracle.sb_pairs(k, e)), (k, e)


def test_user_order_kept_and_default_is_first_connected(H):
    k, e = P.NAMED["house"]
    assert H.plan(None, k, e, order=(4, 1, 0, 2, 3)).info()["order"] == [4, 1, 0, 2, 3]
    # without statistics every order costs the same: the lexicographically first one wins
    assert H.plan(None, k, e).info()["order"] == [0, 1, 2, 3, 4]
    k, e = P.NAMED["4-path"]
    assert H.plan(None, k, e).info()["order"] == [0, 1, 2, 3]


def test_ctypes_mirrors_match_the_header_layout(H, tmp_path):
    """Sizes and field offsets of every public struct, as a C compiler lays them
    out from include/huge.h, equal those of the binding's ctypes mirrors."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"huge_result": H.Result, "huge_exec_opts": H.ExecOpts, "huge_tune_table": H.TuneTable,
               "huge_graph_info": H.GraphInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "huge.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_library_binds_to_torchs_hip_runtime():
    """Loading the library first loads torch, so that the process holds one HIP
    runtime (torch's) whose streams and memory the library shares."""
    import subprocess
    import sys

    code = ("import sys, paper_2103_14294_amd as H; H.load_library(); "
            "print('torch' in sys.modules)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().endswith("True")
