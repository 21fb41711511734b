"""Host logic of bench.py (no GPU): the slowest-kernel choice, the roofline arithmetic,
the counter-record lookup keyed by the kernel-source digest, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def stats(**avg_ms):
    """pass_stats-shaped records: 10 launches, 1 GB per launch, the given average time."""
    return {k: {"launches": 10, "total_ms": 10 * v, "bytes_per_launch": 1e9} for k, v in avg_ms.items()}


def test_slowest_pass_ignores_non_projection_kernels():
    st = stats(z_r2c=0.15, x_proj=0.18, z_c2r=0.32, div_ddo=0.11, reduce_final=5.0)
    assert bench.slowest_pass(st) == "z_c2r"
    st["z_c2r"]["launches"] = 0
    assert bench.slowest_pass(st) == "x_proj"
    assert bench.slowest_pass({}) is None


def test_roofline_arithmetic():
    timed = stats(z_c2r=0.25)                       # only the slowest kernel bracketed
    table = stats(z_r2c=0.125, z_c2r=0.25)          # every kernel, earlier steps
    vox = 256 ** 3
    roof, per_pass = bench.roofline(timed, table, "no_such_workload", vox, "fp32", removed=True)
    assert roof["kernel"] == "z_c2r" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    # algorithmic bytes of the pass that writes the removed part: 48 + 24 B per voxel
    assert roof["algorithmic_bytes_per_voxel"] == 72
    assert roof["achieved"] == pytest.approx(72 * vox / 0.25e-3 / 1e9, rel=1e-4)
    assert roof["peak"] == bench.HBM_PEAK_GBS
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    # the pass's own bytes (the event records' 1 GB) are reported beside it
    assert roof["pass_bytes_per_launch"] == 1e9 and roof["pass_frac"] == pytest.approx(0.5)
    assert roof["traffic"] is None                             # no counter record for this workload
    roof64, _ = bench.roofline(timed, table, "no_such_workload", vox, "fp64", removed=False)
    assert roof64["algorithmic_bytes_per_voxel"] == 96
    assert set(per_pass) == {"z_r2c", "z_c2r"}
    assert per_pass["z_r2c"]["GB_s"] == pytest.approx(8000.0)


def test_traffic_record_requires_current_sources(tmp_path, monkeypatch):
    rec = {"z_c2r@w": {"traffic_bytes": 123.0, "source_digest": "a" * 16},
           "x_proj@w": {"traffic_bytes": 456.0, "source_digest": "b" * 16}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "a" * 16)
    assert bench.load_traffic("z_c2r", "w") == 123.0
    assert bench.load_traffic("x_proj", "w") is None          # counted on other kernel sources
    assert bench.load_traffic("z_r2c", "w") is None           # never profiled


def test_kernel_source_digest_tracks_the_sources():
    d = bench.kernel_source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
    assert bench.kernel_source_digest() == d


def test_committed_traffic_records_name_their_summaries():
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert data
    for key, rec in data.items():
        assert os.path.exists(os.path.join(ROOT, rec["summary"])), key
        assert rec["traffic_bytes"] > 0 and len(rec["source_digest"]) == 16, key


def test_roundoff_amplification():
    import numpy as np

    rng = np.random.default_rng(1)
    S = rng.standard_normal((6, 4, 4, 4)) + 3.0
    assert bench.roundoff_amplification(S, S) == pytest.approx(1.0)
    c0 = S.mean(axis=(1, 2, 3), keepdims=True)
    assert bench.roundoff_amplification(S, c0 + 0.5 * (S - c0)) == pytest.approx(2.0)
    assert bench.roundoff_amplification(S, np.broadcast_to(c0, S.shape)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tune_source_names_the_plans_searched_in_the_run(monkeypatch):
    class A:
        no_autotune = False
    monkeypatch.setattr(bench, "SEARCHED", [])
    monkeypatch.delenv("EQ_AUTOTUNE_CACHE", raising=False)
    monkeypatch.delenv("EQ_TUNE_SOURCE", raising=False)
    assert bench.tune_source(A) == "autotuned in this run"
    monkeypatch.setenv("EQ_AUTOTUNE_CACHE", "/tmp/copy.json")
    monkeypatch.setenv("EQ_TUNE_SOURCE", "profiles/tune_mi355x.json")
    assert bench.tune_source(A) == "profiles/tune_mi355x.json (every plan of this run)"
    bench.SEARCHED.append(("fp32", "ddo", "96x96x96"))
    assert bench.tune_source(A).endswith("absent from it: fp32 ddo 96x96x96")
    A.no_autotune = True
    assert bench.tune_source(A) == "library defaults"
