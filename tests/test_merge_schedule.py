"""The order in which one launch runs every merge-split phase of every
sub-array merged through HBM (csrc/merge_sched.h), checked on the host: the
order covers every work item once, every item's predecessors come before it
(so waiting only ever targets items already taken by running workgroups),
and a simulated run with several workers neither deadlocks nor leaves a
sub-array unsorted.  Built with g++ from tests/merge_sched_check.cpp."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_merge_schedule_order(tmp_path):
    exe = tmp_path / "merge_sched_check"
    src = os.path.join(HERE, "merge_sched_check.cpp")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
