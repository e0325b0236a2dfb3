"""The graph engine's device scheduler (csrc/round_sched.h), run on the CPU:
over synthetic query trees it must take exactly the level engine's decisions
(the same prepare / emit / SINK actions in the same order as a model of the
host loop), count what a direct recursion over the tree counts, never
overfill a queue, and always finish.  Covers tiny queues (the yield to a
deeper level and the backtracking), one-row and empty inputs, and 3- to
7-vertex queries."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("hipcc")
    if cxx is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_harness")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2103_14294_amd", "csrc"), os.path.join(ROOT, "tests", "sched_harness.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


# k, level-2 rows, max bound per row, 1/emit probability, seed, rows per segment, queue rows
CASES = [
    (3, 3000, 20, 2, 3, 1000, 4096),
    (4, 2000, 12, 3, 1, 300, 4096),
    (4, 5000, 3, 1, 2, 4096, 4096),
    (5, 500, 10, 3, 7, 64, 512),
    (6, 300, 8, 2, 11, 32, 64),
    (6, 200, 10, 2, 5, 7, 16),
    (7, 100, 6, 2, 9, 16, 40),
    (4, 1, 5, 1, 3, 1, 8),
    (5, 0, 5, 2, 3, 10, 64),
]


@pytest.mark.parametrize("case", CASES)
def test_device_scheduler_matches_host_loop(harness, case):
    out = subprocess.run([harness] + [str(x) for x in case], check=True, capture_output=True, text=True).stdout
    f = out.split()
    r = {f[i]: int(f[i + 1]) for i in range(0, len(f), 2)}
    assert r["same"] == 1 and r["host_actions"] == r["device_actions"], r
    assert r["device_count"] == r["host_count"] == r["ground"], r
    assert r["overflow"] == 0 and r["error"] == 0, r
