"""The task-graph scheduler of graph mode (csrc/fz_taskgraph.h), checked on
the CPU: dependencies inferred from access modes for the compression and
decompression stage lists (two concurrent branches each), and on random
access lists every pair of conflicting tasks ordered by the stream order and
the cross-stream waits, every kept dependency a real conflict."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_task_graph_schedule(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tg_check")
    src = os.path.join(ROOT, "tests", "taskgraph", "tg_check.cpp")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "0 failed checks" in r.stdout
