"""CPU check of the grouped batch schedule (csrc/batch_plan.cpp), which the
HIP device executes eagerly and inside the stream capture of a batch graph.

tests/cpp/test_batch_plan.cpp restates the rules of streams, events and
stream capture and replays the planner's operation lists against them: data
dependencies per request (copy-in, launch, copy-out, completion), every
operation of a capture on a capturing stream, and every stream forked into a
capture joined back into the origin after its last operation.  It also
replays the earlier capture schedule, which joined compute stream 1 right
after its kernels and before the small copy-outs queued behind them, a
schedule with a missing wait for the host-to-device FIFO, and a graph
launched without first waiting for its input pieces: the check must reject
all three.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_batch_plan_dependencies_and_capture_joins(tmp_path):
    exe = str(tmp_path / "test_batch_plan")
    cmd = ["g++", "-O1", "-std=c++17", "-Wall", "-Werror", f"-I{ROOT}/include", f"-I{ROOT}/paper_1511_07658_amd/csrc",
           f"{ROOT}/tests/cpp/test_batch_plan.cpp", f"{ROOT}/paper_1511_07658_amd/csrc/batch_plan.cpp", "-o", exe]
    subprocess.run(cmd, check=True)
    p = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert p.returncode == 0, p.stdout
    assert "early join detected: a stream forked into the capture is not joined" in p.stdout, p.stdout
    assert "missing input wait detected" in p.stdout, p.stdout
    assert "graph without the input wait detected" in p.stdout, p.stdout
    assert p.stdout.strip().endswith("ok: 0 failures"), p.stdout
