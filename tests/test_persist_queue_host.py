"""The persistent launch's work queue (csrc/eq_persist_queue.hpp), checked on the CPU.

tests/native/persist_queue_host.cpp includes the library's header, compiles it for the host
(hipcc --cuda-host-only) and decodes every queue position for batch sizes 1-100, item counts
per stage 1-768 and lags 1-12: each (stage, field, index) appears exactly once, and every
waiting item sits after all the items it waits for (the property that keeps the queue free
of deadlock: a waiter only waits on items claimed by running workgroups)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "persist_queue_host.cpp")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_queue_decode_is_a_bijection_with_waits_after_dependencies(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "persist_queue_host")
    cmd = [HIPCC, "-O1", "-std=c++17", "-x", "hip", "--cuda-host-only",
           "-I", os.path.join(ROOT, "paper_2105_01612_amd", "csrc"), SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok ") and int(r.stdout.split()[1]) > 1000
