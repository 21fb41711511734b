"""The C ABI's host logic under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/native/capi_host_check.cpp includes eq_capi.cpp, so validation, radix
factorization, the workspace layout, the EQ_TUNE parser, the status strings and a
plan's failure path run instrumented; it links the library's own kernel objects (built
by paper_2105_01612_amd.build, host code uninstrumented) and launches nothing.  The
sanitizers instrument host code only: each -fsanitize flag of the hipcc line is
preceded by -Xarch_host, and the executable is linked by g++."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "capi_host_check.cpp")
CSRC = os.path.join(ROOT, "paper_2105_01612_amd", "csrc")
OBJDIR = os.path.join(ROOT, "paper_2105_01612_amd", "_build")
KERNEL_OBJS = ["eq_kernels.o", "eq_plane.o", "eq_sched_pow2_f32.o", "eq_sched_pow2_f64.o", "eq_sched_mixed.o"]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_capi_host_logic_is_clean_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC) or not shutil.which("g++"):
        pytest.skip("hipcc or g++ not available")
    objs = [os.path.join(OBJDIR, o) for o in KERNEL_OBJS]
    if not all(os.path.exists(o) for o in objs):
        from paper_2105_01612_amd import build

        build.build(incremental=True)
    obj = str(tmp_path / "check.o")
    exe = str(tmp_path / "check")
    compile_cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
                   "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", SRC, "-o", obj]
    r = subprocess.run(compile_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    link_cmd = ["g++", "-fsanitize=address,undefined", obj] + objs + [
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(link_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("EQ_TUNE", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert int(r.stdout.split()[1]) > 5000
