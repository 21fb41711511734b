"""A program that uses libeq through include/eq.h alone (tests/native/capi_gpu_consumer.cpp,
built by build() into tests/native/bin): no Python, no torch, device buffers from hipMalloc.

On the CPU it loads libeq.so and has the bad grid refused before any device work; on the GPU
every check passes (plane-wave closed form, residual, idempotence, out + removed = in, for both
operators in FP64)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "native", "bin", "capi_gpu_consumer")


def run_consumer():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built: run __graft_entry__.build() (or python -m paper_2105_01612_amd.build)")
    return subprocess.run([EXE], capture_output=True, text=True, timeout=120)


def test_consumer_loads_libeq_and_refuses_a_bad_grid():
    r = run_consumer()
    lines = r.stdout.splitlines()
    assert lines and lines[0].startswith("libeq "), r.stdout + r.stderr
    assert any(l.startswith("PASS nx = 14 refused with EQ_ERR_SIZE") for l in lines), r.stdout
    assert r.returncode in (0, 1)          # 1 without a GPU: eq_plan reports EQ_ERR_DEVICE


@pytest.mark.gpu
def test_consumer_passes_every_check_on_the_gpu():
    r = run_consumer()
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    assert lines[-1] == "ALL PASSED"
    assert sum(l.startswith("PASS ") for l in lines) == 11 and not any(l.startswith("FAIL") for l in lines)
