"""Build libeq.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2105_01612_amd.build [--incremental]

Compiles every translation unit under csrc/ for gfx950 and links them into
paper_2105_01612_amd/libeq.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libeq.so")
SOURCES = ["eq_kernels.hip", "eq_plane.hip", "eq_sched_pow2_f32.hip", "eq_sched_pow2_f64.hip", "eq_sched_mixed.hip", "eq_capi.cpp"]
ARCH = os.environ.get("EQ_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def common_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        "-Wno-unused-command-line-argument",
    ]


def _up_to_date(src: str, obj: str) -> bool:
    """Object newer than its source, every csrc header and the public header."""
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src), os.path.join(INCLUDE, "eq.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, verbose: bool, incremental: bool = False) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    if incremental and _up_to_date(src, obj):
        return obj
    cmd = [hipcc()] + common_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if verbose and warn:
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit (incremental: only those older than their inputs) and link."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


CONSUMER_SRC = os.path.join(ROOT, "tests", "native", "capi_gpu_consumer.cpp")
CONSUMER = os.path.join(ROOT, "tests", "native", "bin", "capi_gpu_consumer")


def build_consumer(verbose: bool = False) -> str:
    """Build the test program that calls libeq through include/eq.h only (no Python), linked
    against the libeq.so next to this file (found at run time through a relative rpath)."""
    os.makedirs(os.path.dirname(CONSUMER), exist_ok=True)
    rpath = "-Wl,-rpath,$ORIGIN/" + os.path.relpath(HERE, os.path.dirname(CONSUMER))
    cmd = ([hipcc()] + common_flags() + ["-x", "hip", CONSUMER_SRC, "-x", "none", "-L", HERE, "-leq", rpath,
                                         "-o", CONSUMER + ".tmp"])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {CONSUMER_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(CONSUMER + ".tmp", CONSUMER)
    return CONSUMER


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv[1:]))
    print(build_consumer(verbose=True))
