"""The register FFT engine's arithmetic and Stockham indexing, emulated on the CPU.

tests/native/fft_engine_host.cpp includes the library's eq_fft.hpp, compiles it for
the host (hipcc --cuda-host-only) and runs every thread of one line stage by stage
in barrier order, for each radix schedule the library uses, both directions and
all four register/LDS entry and exit modes; the result is compared with a direct
O(n^2) DFT sum."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "fft_engine_host.cpp")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# (E, radices) of the schedules the planner picks (see factor_axis in eq_capi.cpp)
SCHEDULES = [
    (8, [8]), (8, [8, 2]), (8, [8, 4]), (8, [8, 8]), (16, [16, 8]), (16, [16, 16]), (16, [16, 8, 4]),
    (16, [16, 16, 4]), (24, [8, 3]), (24, [8, 2, 3]), (24, [8, 4, 3]), (24, [8, 8, 3]), (24, [8, 8, 2, 3]),
    (24, [8, 3, 3]), (40, [8, 5]), (40, [8, 4, 5]), (40, [8, 8, 5]), (40, [8, 5, 5, 5]),
    (12, [4, 4, 2, 3]), (12, [4, 4, 4, 3]), (12, [4, 4, 4, 2, 3]), (20, [4, 4, 2, 5]), (20, [4, 4, 4, 5]),
]


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("fft") / "fft_host")
    cmd = [HIPCC, "-O1", "-std=c++17", "-x", "hip", "--cuda-host-only",
           "-I", os.path.join(ROOT, "paper_2105_01612_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.parametrize("E,radices", SCHEDULES)
def test_register_engine_matches_direct_dft(emulator, E, radices):
    r = subprocess.run([emulator, str(E)] + [str(x) for x in radices], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split()
    assert len(lines) == 6 * 16
    for k in range(0, len(lines), 6):
        n, e, direction, prec, modes, err = lines[k:k + 6]
        tol = 2e-15 if prec == "f64" else 5e-7
        assert float(err) <= tol, (n, e, direction, prec, modes, err)
