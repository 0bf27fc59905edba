"""The persistent batched launch's queue, exercised on the CPU.

``tests/emul/pq_emul.cpp`` drives the worker loop the kernel runs
(``csrc/batch_queue.h``) with host threads standing in for waves, fewer of
them resident than launched, and checks that every unit runs once and only
after its grid's earlier passes, that no wait runs out, that the last wave
leaves the queue cleared for the next launch, and that two planted mistakes
are caught (a wait that can never be met ends through the time limit and the
abort flag; a dependency count one too low shows up as violations).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1502_03504_amd", "csrc")


def test_persistent_queue_emulation(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "pq_emul")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "emul", "pq_emul.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
