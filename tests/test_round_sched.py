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


def _trace(harness, *args):
    out = subprocess.run([harness, "trace"] + [str(x) for x in args], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    f = out[0].split()
    r = {f[i]: int(f[i + 1]) for i in range(0, len(f), 2)}
    return r, out[1].split()[1:]


def _operator_runs(actions):
    """The operator scheduled in each time slot: consecutive actions of one level
    (its prepares and extends) are one scheduling of that level's operator."""
    runs = []
    for a in actions:
        w = int(a.split(":")[1])
        if not runs or runs[-1] != w:
            runs.append(w)
    return runs


def test_example_5_1_trace(harness):
    """Section 5.2, Example 5.1: a plan SCAN_1 -> EXTEND_2 -> EXTEND_3 -> SINK_4
    with output queues of three batches.  Here a batch is one row; the SCAN's
    output (level 2) is read by the level-2 extend, so EXTEND_2, EXTEND_3 and
    SINK_4 are the extends of levels 2, 3 and 4 of a 5-vertex query.  With three
    level-2 rows and two candidates per row at levels 2 and 3 (one at the SINK),
    the scheduler must run EXTEND_2 until its queue is full (T2), then EXTEND_3
    (T3), then SINK_4 until its input is empty (T4), backtrack to EXTEND_3 whose
    input is not yet empty (T5), go forward to SINK_4 again (T6), find EXTEND_3's
    input empty on backtracking and move back to EXTEND_2 (T7), and so on until
    every level is drained."""
    r, actions = _trace(harness, 5, 3, 3, 3, 2, 2, 1)
    assert r["same"] == 1 and r["error"] == 0 and r["overflow"] == 0, r
    assert r["device_count"] == r["ground"] == 3 * 2 * 2, r
    runs = _operator_runs(actions)
    assert runs[:6] == [2, 3, 4, 3, 4, 2], runs
    # T1..T4 in detail: the level-2 batch is read, EXTEND_2 fills its queue of
    # three rows and yields with input left, EXTEND_3 fills its queue and yields
    # with input left, SINK_4 consumes all of its input
    assert actions[:7] == ["P:2", "E:2", "P:3", "E:3", "P:4", "S:4", "E:3"], actions
    # every scheduling of EXTEND_2 / EXTEND_3 is followed by its successor, every
    # SINK by a backtrack
    for a, b in zip(runs, runs[1:]):
        assert b == a + 1 or (a == 4 and b == 3) or (b < a), (a, b)


def test_example_5_1_without_yield_is_bfs(harness):
    """The same plan with queues large enough for everything runs breadth-first:
    each operator once, in order, then the scheduler backtracks to the end."""
    r, actions = _trace(harness, 5, 3, 3, 1000, 2, 2, 1)
    assert r["same"] == 1 and r["device_count"] == 12, r
    assert _operator_runs(actions) == [2, 3, 4], actions
