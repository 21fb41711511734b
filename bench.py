#!/usr/bin/env python3
"""Benchmark of the equilibrium projection on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload headline|small|largest|gb_heavy|batched]

One step is the whole hot path over one batch of synthetic input already
resident in HBM: forward 3-D real DFT of the six stress components, the
per-frequency projection, the inverse DFT with the removed part (eq_project),
then the divergence residual of the result (eq_residual).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "equilibrated voxels/s at 256^3 (FP32 vs FP64, % HBM roofline); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PAPER_CONTEXT = {"value": 16777216 / 473.0, "unit": "voxels/s",
                 "source": "one filter application on a 256^3 field in 473 s (Section 6)",
                 "hardware": "Intel Core i7-8700 CPU"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """sha256 (first 16 hex) over every device source file (csrc/*.hip, csrc/*.hpp, sorted)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2105_01612_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if the kernels are unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    rec = data.get(f"{kernel}@{workload}")
    if not rec or rec.get("source_digest") != kernel_source_digest():
        return None
    return rec.get("traffic_bytes")


def make_workload(name: str, prec: str):
    from paper_2105_01612_amd import workload as wl

    dt = np.float32 if prec == "fp32" else np.float64
    if name == "batched":
        specs = wl.batched_specs()
        S = np.stack([wl.voronoi_field(sp, dtype=dt) for sp in specs])
        desc = "64 x 128^3 fields, periodic Voronoi 300 grains each, N(0,100)+N(0,5) MPa, seeds 300-363"
        return S, desc
    spec = wl.CONFIG_SPECS[name]
    S = wl.voronoi_field(spec, dtype=dt)
    nz, ny, nx = spec.shape
    desc = (f"{nx}^3 single field, periodic Voronoi {spec.grains} grains, grain stress N(0,{spec.sigma_grain:g}) MPa"
            + (f" + gradient N(0,{spec.sigma_grad:g}) MPa/voxel" if spec.sigma_grad else "")
            + f" + noise N(0,{spec.sigma_noise:g}) MPa, seed {spec.seed}")
    return S[None], desc


TUNE_FILE = os.path.join(ROOT, "profiles", "tune_mi355x.json")


SEARCHED = []   # (prec, op, grid) of the plans whose tuning was searched in this run, not read


def tune_source(args) -> str:
    if args.no_autotune:
        return "library defaults"
    src = os.environ.get("EQ_TUNE_SOURCE") or os.environ.get("EQ_AUTOTUNE_CACHE")
    if not src:
        return "autotuned in this run"
    if not SEARCHED:
        return f"{src} (every plan of this run)"
    return f"{src}; searched in this run, absent from it: " + ", ".join(f"{p} {o} {g}" for p, o, g in SEARCHED)


def run_gpu(S_host, op, prec, steps, warmup, with_residual=True, timing=True, tune=True, removed=True):
    """Time `steps` steps of eq_project (+ eq_residual of the result) on device-resident input.
    removed=False and with_residual=False time the projection alone (no removed part)."""
    import torch
    import paper_2105_01612_amd as eq

    B, _, nz, ny, nx = S_host.shape
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = eq.plan(nx, ny, nz, batch=B, op=op, prec=prec)
        x = torch.from_numpy(S_host).to("cuda")
        out = torch.empty_like(x)
        rem = torch.empty_like(x) if removed else None
        norms = None
        tuned = None
        if tune:
            from paper_2105_01612_amd.autotune import autotune

            tuned = autotune(plan, x, out, torch.empty_like(x) if rem is None else rem, reps=3,
                             use_cache=bool(os.environ.get("EQ_AUTOTUNE_CACHE")))
            if not tuned.get("from_cache"):
                SEARCHED.append((prec, op, "x".join(map(str, (nx, ny, nz))) + (f" x{B}" if B > 1 else "")))
            log(f"[bench] tuning {prec} {op} ({'cached' if tuned.get('from_cache') else 'searched'}): "
                f"{tuned['tune']} -> {tuned['resolved']}")
        for _ in range(warmup):
            plan.project(x, out, rem)
            if with_residual:
                norms = plan.residual(out)
        torch.cuda.synchronize()
        # per-pass table: every launch bracketed by events, over as many steps as the timed
        # region, before it; the timed region then brackets only the slowest kernel (two
        # event records per step instead of two per launch)
        all_stats, only = {}, None
        if timing:
            plan.reset_stats()
            plan.set_timing(True)
            for _ in range(steps):
                plan.project(x, out, rem)
                if with_residual:
                    plan.residual(out)
            all_stats = plan.pass_stats()
            plan.set_timing(False)
            only = slowest_pass(all_stats)
        plan.reset_stats()
        plan.set_timing(timing, only=only)
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            plan.project(x, out, rem)
            if with_residual:
                norms = plan.residual(out)
            else:
                stream.synchronize()
            lat.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        plan.set_timing(False)
        stats = plan.pass_stats()
        result = out.cpu()
        rem_host = rem.cpu() if removed else None
        resolved = plan.get_tune()
        plan.destroy()
    return {"elapsed_s": elapsed, "lat_ms": lat, "stats": stats, "all_stats": all_stats, "out": result,
            "removed": rem_host, "norms": norms, "tune": resolved}


PROJECT_PASSES = ("z_r2c", "y_fwd", "x_proj", "y_inv", "z_c2r", "plane_r2c", "z_proj", "plane_c2r", "div_ddo")

# Algorithmic bytes per voxel of one pass in FP32 (doubled for FP64): one read and one
# write of the six components (48 B), plus the removed part's write (24 B) on the pass
# that produces it; the DDO residual reads the field once (24 B).
SEC8D_BYTES_FP32 = {"z_r2c": 48, "y_fwd": 48, "x_proj": 48, "y_inv": 48, "z_c2r": 48, "plane_r2c": 48,
                    "z_proj": 48, "plane_c2r": 48, "div_ddo": 24}
REMOVED_PASSES = ("z_c2r", "plane_c2r")


def sec8d_bytes(name, voxels, prec, removed):
    b = SEC8D_BYTES_FP32.get(name, 0) + (24 if removed and name in REMOVED_PASSES else 0)
    return b * voxels * (2 if prec == "fp64" else 1)


def slowest_pass(stats):
    best = None
    for name in PROJECT_PASSES:
        st = stats.get(name)
        if st and st["launches"]:
            avg = st["total_ms"] / st["launches"]
            if best is None or avg > best[1]:
                best = (name, avg)
    return best[0] if best else None


def roofline(stats, all_stats, workload, voxels, prec="fp32", removed=True):
    """The slowest kernel's rate from the timed region's events, on the algorithmic bytes per
    voxel of one pass (48 B FP32, + 24 B for the removed part's write, 24 B for the DDO
    residual); the bytes that pass actually moves (its own reads of the input for the removed
    part included) are reported beside it.  The per-pass table comes from the fully
    instrumented steps before the timed region."""
    best = None
    for name in PROJECT_PASSES:
        st = stats.get(name)
        if not st or st["launches"] == 0:
            continue
        avg = st["total_ms"] / st["launches"]
        if best is None or avg > best[1]:
            best = (name, avg, st["bytes_per_launch"])
    if best is None:
        return None, {}
    name, avg_ms, by = best
    alg = sec8d_bytes(name, voxels, prec, removed)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    per_pass = {}
    for n, st in (all_stats or stats).items():
        if st["launches"]:
            a = st["total_ms"] / st["launches"]
            per_pass[n] = {"avg_ms": round(a, 5), "GB_s": round(st["bytes_per_launch"] / (a * 1e-3) / 1e9, 1),
                           "launches": st["launches"]}
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": alg, "algorithmic_bytes_per_voxel": alg / voxels,
            "pass_bytes_per_launch": by, "pass_bytes_per_voxel": round(by / voxels, 2),
            "pass_frac": round(by / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": load_traffic(name, workload)}, per_pass


def frob_err(got, ref):
    w = np.array([1, 1, 1, 2, 2, 2], dtype=np.float64).reshape(1, 6, 1, 1, 1)
    d = got.astype(np.float64) - ref
    return math.sqrt(float(np.sum(w * d * d)) / float(np.sum(w * ref * ref))), float(np.abs(d).max())


def roundoff_amplification(S, S_eq):
    """||S - c0|| / ||S_eq - c0|| (Frobenius, off-diagonals twice; c0 = the per-component
    mean): the factor by which the input's round-off grows relative to the output."""
    w = np.array([1, 1, 1, 2, 2, 2], dtype=np.float64).reshape(6, 1, 1, 1)
    c0 = S.mean(axis=(1, 2, 3), keepdims=True)
    num = float(np.sum(w * (S - c0) ** 2))
    den = float(np.sum(w * (S_eq - c0) ** 2))
    return math.sqrt(num / den) if den > 0 else None


def batched_errors(S32, out, op):
    """The oracle error of every field of a batch (FP32 result against the FP64 oracle on the
    same input bytes): max and median rel-L2 and the largest max-abs."""
    import oracle

    os.environ["ORACLE_WORKERS"] = str(os.cpu_count() or 1)
    t = time.perf_counter()
    rel, mab = [], []
    for b in range(S32.shape[0]):
        ref, _ = oracle.project(S32[b].astype(np.float64), op)
        e = frob_err(out[b:b + 1], ref[None])
        rel.append(e[0])
        mab.append(e[1])
    log(f"[bench] oracle error of {len(rel)} fields in {time.perf_counter() - t:.1f} s: max rel-L2 {max(rel):.2e}")
    return {"fields": len(rel), "rel_l2_max": max(rel), "rel_l2_median": float(np.median(rel)),
            "max_abs_mpa": max(mab), "tol": 1e-5}


def cpu_baseline(S_field64, op):
    """The FP64 oracle on the host, on one whole field (the bounded sample)."""
    import oracle

    cores = os.cpu_count() or 1
    vox = S_field64[0].size
    grid = "x".join(map(str, S_field64.shape[1:][::-1]))

    def timed(workers, max_runs, budget_s):
        os.environ["ORACLE_WORKERS"] = str(workers)
        runs, dt, ref = 0, 0.0, None
        while runs < max_runs and (runs == 0 or dt < budget_s):
            t0 = time.perf_counter()
            ref, _ = oracle.project(S_field64, op)
            dt += time.perf_counter() - t0
            runs += 1
        return ref, runs, dt

    # all host cores (scipy.fft workers = os.cpu_count()), repeated to about 10 s; then one core
    ref, runs, dt = timed(cores, 5, 10.0)
    _, runs1, dt1 = timed(1, 1, 0.0)
    log(f"[bench] oracle host: os.cpu_count() = {cores}; {runs} runs in {dt:.2f} s with {cores} workers, "
        f"{dt1:.2f} s with 1")
    return ref, {"value": vox * runs / dt, "unit": "voxels/s", "cores": cores, "kind": "oracle",
                 "sample": f"{runs} x one whole field ({grid}), FP64, {op.upper()}, numpy + scipy.fft with "
                           f"workers = os.cpu_count() = {cores}, {dt:.2f} s in total",
                 "single_core": {"value": vox * runs1 / dt1, "unit": "voxels/s", "cores": 1,
                                 "sample": f"{runs1} x one whole field ({grid}), scipy.fft workers = 1, "
                                           f"{dt1:.2f} s"}}


def run_serve(args):
    """Poisson stream of requests over six size classes, continuous batching (serve.py)."""
    import torch
    from paper_2105_01612_amd import workload as wl
    from paper_2105_01612_amd.serve import GpuBackend, Request, Server

    sizes = wl.SERVING_SIZES
    pool_n = {64: 8, 96: 8, 128: 4, 192: 4, 256: 2, 384: 2}
    t = time.perf_counter()
    pools = {}
    for n in sizes:
        arr = np.stack([wl.voronoi_field(wl.serving_spec(n, j), dtype=np.float32) for j in range(pool_n[n])])
        pools[n] = torch.from_numpy(arr).cuda()
        del arr
    torch.cuda.synchronize()
    log(f"[bench] serve pools generated in {time.perf_counter() - t:.1f}s: {pool_n}")
    # each class's plans take the tune file's entry for their configuration (no search while serving)
    cache = None if args.no_autotune else os.environ.get("EQ_AUTOTUNE_CACHE")
    tuned_classes = []
    if cache:
        import types

        from paper_2105_01612_amd.autotune import cache_key, load_cache

        entries = load_cache(cache)
        tuned_classes = [n for n in sizes if cache_key(types.SimpleNamespace(nx=n, ny=n, nz=n, batch=1, prec="fp32",
                                                                             op=args.op)) in entries]
        cache_name = os.environ.get("EQ_TUNE_SOURCE") or cache
    be = GpuBackend(pools, prec="fp32", op=args.op, tune_cache=cache, graphs=not args.serve_no_graphs)
    srv = Server(be, int(args.budget_gb * 2 ** 30))          # smallest first, at most 8 in flight
    srv.warm(sizes)
    ns = wl.request_sizes(args.requests, seed=4000, sizes=sizes)
    rng = np.random.Generator(np.random.PCG64(4002))
    fields = [int(rng.integers(0, pool_n[int(n)])) for n in ns]
    # saturation: every request present at t = 0
    sat = srv.run([Request(i, int(n), 0.0, f) for i, (n, f) in enumerate(zip(ns, fields))])
    lam = 0.7 * sat["requests_per_s"]
    arr = wl.poisson_arrivals(args.requests, lam, seed=4000)
    res = srv.run([Request(i, int(n), float(a), f) for i, (n, a, f) in enumerate(zip(ns, arr, fields))])
    # admission policies at the same arrivals: in-flight cap and smallest-first
    policies = {}
    for order, cap in (("fifo", None), ("fifo", 4), ("sjf", 4), ("sjf", 8), ("sjf", 16)):
        srv.order, srv.max_inflight = order, cap
        r = srv.run([Request(i, int(n), float(a), f) for i, (n, a, f) in enumerate(zip(ns, arr, fields))])
        policies[f"{order}_cap{cap}"] = {k: r[k] for k in ("requests_per_s", "p50_ms", "p99_ms", "mean_ms", "max_ms")}
        policies[f"{order}_cap{cap}"]["per_size"] = r["per_size"]
        log(f"[bench] serve 0.7x {order} cap {cap}: p50 {r['p50_ms']:.2f} ms p99 {r['p99_ms']:.2f} ms")
    srv.order, srv.max_inflight = "sjf", 8
    over = srv.run([Request(i, int(n), float(a), f) for i, (n, a, f) in
                    enumerate(zip(ns, wl.poisson_arrivals(args.requests, 1.2 * sat["requests_per_s"], 4001), fields))])
    srv.close()
    # H2D-inclusive variant: the pools in pinned host memory, so that each request's service starts
    # with its input's transfer over PCIe (the first requests of the same stream, its own
    # saturation and 0.7 x that rate)
    del be, srv
    torch.cuda.empty_cache()
    host_pools = {n: p.cpu().pin_memory() for n, p in pools.items()}
    del pools
    torch.cuda.empty_cache()
    m = min(args.requests, 500)
    be_h = GpuBackend(host_pools, prec="fp32", op=args.op, tune_cache=cache, graphs=not args.serve_no_graphs)
    srv_h = Server(be_h, int(args.budget_gb * 2 ** 30))
    srv_h.warm(sizes)
    sat_h = srv_h.run([Request(i, int(n), 0.0, f) for i, (n, f) in enumerate(zip(ns[:m], fields[:m]))])
    arr_h = wl.poisson_arrivals(m, 0.7 * sat_h["requests_per_s"], seed=4003)
    res_h = srv_h.run([Request(i, int(n), float(a), f) for i, (n, a, f) in enumerate(zip(ns[:m], arr_h, fields[:m]))])
    srv_h.close()
    log(f"[bench] serve H2D-inclusive: saturated {sat_h['requests_per_s']:.0f} requests/s, 0.7x p50 "
        f"{res_h['p50_ms']:.2f} ms p99 {res_h['p99_ms']:.2f} ms")
    h2d = {"requests": m, "saturated": sat_h, "arrival_rate_per_s": 0.7 * sat_h["requests_per_s"],
           "at_0.7_saturation": res_h}
    return {"metric": METRIC, "value": res["voxels_per_s"], "unit": "voxels/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic: serving pools " + str(pool_n),
            "config": {"workload": f"serve: {args.requests} Poisson requests, N uniform over {list(sizes)}, "
                                   f"one grain per 16^3 voxels, FP32 {args.op.upper()}, graphs per slot, "
                                   f"budget {args.budget_gb} GiB"},
            "arrival_rate_per_s": lam, "p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"],
            "p99_ms_by_size": {k: v["p99_ms"] for k, v in res["per_size"].items()},
            "policy": "smallest first, 8 in flight, 4 streams by size class, "
                      + ("pass launches per request" if args.serve_no_graphs else "a captured graph per slot"),
            "tune_source": f"{cache_name} (classes with an entry: {tuned_classes})" if cache else "library defaults",
            "saturated": sat, "at_0.7_saturation": res, "at_1.2_saturation": over,
            "policies_at_0.7_saturation": policies, "h2d_inclusive": h2d}


def run_grain_avg(args):
    """Grain-averaging recovery study (Section 5.1 protocol on synthetic equilibrated truth):
    the paper's 64^3 / 100-grain cell and a 256^3 / 1000-grain cell, CDO and DDO, FP64 and FP32."""
    from paper_2105_01612_amd import workload as wl
    from paper_2105_01612_amd.studies import grain_average_recovery

    cells = [wl.FieldSpec((64, 64, 64), grains=100, sigma_grain=100.0, sigma_noise=5.0, seed=64),
             wl.FieldSpec((256, 256, 256), grains=1000, sigma_grain=200.0, sigma_noise=10.0, seed=256)]
    rows = []
    t0 = time.perf_counter()
    for spec in cells:
        for op in ("cdo", "ddo"):
            for prec in ("fp64", "fp32"):
                r = grain_average_recovery(spec, op=op, prec=prec)
                log(f"[bench] grain_avg {spec.shape[0]}^3 {op} {prec}: |A-T| {r['average_vs_truth']['rel_l2']:.4f} "
                    f"-> |R-T| {r['recovered_vs_truth']['rel_l2']:.4f}")
                rows.append(r)
    return {"metric": "grain-average recovery error vs synthetic equilibrated truth (Table 1 protocol)",
            "value": rows[1]["recovered_vs_truth"]["rel_l2"], "unit": "rel-L2 (64^3, DDO, FP64)",
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic: periodic Voronoi truth projected "
            "with the same operator, then grain-averaged", "config": {"workload": "grain_avg"},
            "wall_s": time.perf_counter() - t0, "results": rows}


def _inloop_rate(plan, a, b, stream, k):
    """Asynchronous rate of k ping-pong projections (graph replays) and 40 synchronous calls;
    `b` ends as P applied to the previous iterate."""
    for _ in range(5):
        plan.project(a, b)
        plan.project(b, a)
    stream.synchronize()
    t = time.perf_counter()
    for _ in range(k // 2):
        plan.project(a, b)
        plan.project(b, a)
    stream.synchronize()
    dt = (time.perf_counter() - t) / k
    lat = []
    for _ in range(40):
        t1 = time.perf_counter()
        plan.project(a, b)
        stream.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    return dt, lat


def run_inloop(args):
    """Repeated projection inside an iterative loop over one resident plan (Section 6: the
    filter as a step of an iterative reconstruction): x <- P(x) ping-pongs between two buffers,
    each call either replaying the plan's captured hipGraph ("graph") or launching the passes on
    the plan's stream ("stream"); at 64^3 and 128^3 also the persistent single launch.  Reports
    the asynchronous rate and the synchronous per-call latency of each.  P is a projection, so
    every iterate is P(x0) up to rounding: at 64^3 and 128^3 the first projection and the last
    buffer are compared with the FP64 oracle's P(x0).  The first is held to 1e-5; the FP32 round
    trip's fixed rounding bias compounds over the replays (the error grows linearly, reported
    per projection)."""
    import torch
    import paper_2105_01612_amd as eq
    from paper_2105_01612_amd import workload as wl

    rows = []
    refs = {}
    for n in (64, 128, 256):
        x0 = wl.voronoi_field(wl.serving_spec(n, 0), dtype=np.float32)
        for mode in (("graph", "stream", "persistent") if n < 256 else ("graph", "stream")):
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                flags = {"graph": ["capture_graph"], "stream": [], "persistent": ["persistent"]}[mode]
                plan = eq.plan(n, op=args.op, prec="fp32", flags=flags, stream=stream)
                a = torch.from_numpy(x0).cuda()
                b = torch.empty_like(a)
                tune = None
                if mode != "persistent" and not args.no_autotune:
                    from paper_2105_01612_amd.autotune import autotune

                    tuned = autotune(plan, a, b, None, reps=3, use_cache=bool(os.environ.get("EQ_AUTOTUNE_CACHE")))
                    if not tuned.get("from_cache"):
                        SEARCHED.append(("fp32", args.op, f"{n}x{n}x{n}"))
                    tune = tuned["resolved"]
                plan.project(a, b)
                first = b.cpu().numpy()
                dt, lat = _inloop_rate(plan, a, b, stream, 200 if n < 256 else 60)
                plan.destroy()
                final = b.cpu().numpy()
            row = {"n": n, "launch": mode, "tune": tune, "replays": (200 if n < 256 else 60) + 50,
                   "projections_per_s": 1.0 / dt, "voxels_per_s": n ** 3 / dt,
                   "p50_ms": statistics.median(lat), "p99_ms": float(np.percentile(lat, 99))}
            if n < 256:
                if n not in refs:
                    import oracle

                    refs[n] = oracle.project(x0.astype(np.float64), args.op)[0]
                rel1, mab1 = frob_err(first[None], refs[n][None])
                rel, mab = frob_err(final[None], refs[n][None])
                k = row["replays"] + 1
                row["error_vs_oracle"] = {"first_projection_rel_l2": rel1, "first_projection_max_abs_mpa": mab1,
                                          "tol": 1e-5, "after_all_rel_l2": rel, "projections": k,
                                          "drift_per_projection": rel / k}
            rows.append(row)
            log(f"[bench] inloop {n}^3 {mode}: {1.0 / dt:.0f} projections/s, sync p50 {rows[-1]['p50_ms']:.3f} ms"
                + (f", oracle rel-L2 first {row['error_vs_oracle']['first_projection_rel_l2']:.2e}, after "
                   f"{row['error_vs_oracle']['projections']} {row['error_vs_oracle']['after_all_rel_l2']:.2e}"
                   if "error_vs_oracle" in row else ""))
    head = max((r for r in rows if r["n"] == 128 and r["launch"] != "persistent"), key=lambda r: r["projections_per_s"])
    return {"metric": "repeated in-loop projections (one plan, x <- P(x))", "value": head["projections_per_s"],
            "unit": "projections/s (128^3 FP32)", "higher_is_better": True, "n_gpus": 1,
            "data": "synthetic: serving pool field 0 per size",
            "config": {"workload": "inloop", "op": args.op, "launch": head["launch"]},
            "error_vs_oracle_tol": 1e-5, "tune_source": tune_source(args),
            "results": rows}


def run_persistent(args):
    """Batches of 64 fields (64^3 and 128^3, 300 grains each, seeds 300..363) projected by the
    per-pass three-pass schedule (its default z stage, and the four-element z stage the
    persistent launch uses) and by one persistent launch; ms per batch over `steps` calls."""
    import torch
    import paper_2105_01612_amd as eq
    from paper_2105_01612_amd import workload as wl

    rows = []
    for n in (64, 128):
        S = np.stack([wl.voronoi_field(sp, dtype=np.float32) for sp in wl.batched_specs(n=n)])
        x = torch.from_numpy(S).cuda()
        out = torch.empty_like(x)
        rem = torch.empty_like(x)
        for label, flags, tune in (("three_pass", [], dict(schedule=3)), ("three_pass_zp4", [], dict(schedule=3, zp_e=4)),
                                   ("persistent", ["persistent"], None)):
            plan = eq.plan(n, batch=64, op=args.op, prec="fp32", flags=flags)
            if tune:
                plan.tune(**tune)
            for _ in range(args.warmup):
                plan.project(x, out, rem)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                plan.project(x, out, rem)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) / args.steps * 1e3
            plan.destroy()
            rows.append({"n": n, "batch": 64, "path": label, "ms_per_batch": ms, "voxels_per_s": 64 * n ** 3 / (ms * 1e-3),
                         "hbm_frac_168B": 64 * n ** 3 * 168 / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)})
            log(f"[bench] 64 x {n}^3 {label}: {ms:.3f} ms")
        del x, out, rem
        torch.cuda.empty_cache()
    head = next(r for r in rows if r["n"] == 64 and r["path"] == "persistent")
    return {"metric": "batched projection, one persistent launch vs three launches", "value": head["voxels_per_s"],
            "unit": "voxels/s (64 x 64^3 FP32, persistent)", "higher_is_better": True, "n_gpus": 1,
            "data": "synthetic: 64 Voronoi fields per size, 300 grains, seeds 300-363",
            "config": {"workload": "persistent", "op": args.op}, "results": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "small", "largest", "gb_heavy", "batched", "serve", "grain_avg",
                             "inloop", "persistent"])
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget for slots")
    ap.add_argument("--serve-no-graphs", action="store_true",
                    help="serve: launch each request's passes instead of replaying a captured graph per slot")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch shapes")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune results file (read if present, else written): a profiled run reuses an "
                         "earlier run's results instead of launching the search's trial kernels")
    ap.add_argument("--op", default="ddo", choices=["ddo", "cdo"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 and CDO side runs")
    ap.add_argument("--no-timing", action="store_true", help="no per-pass events in the timed region")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of 512 MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.tune_cache:
        os.environ["EQ_AUTOTUNE_CACHE"] = os.path.abspath(args.tune_cache)
    elif not args.no_autotune and os.path.exists(TUNE_FILE):
        # the committed tuning, so that bench lines and the committed profiles describe the same
        # kernel instantiations; read from a private copy, so that a configuration it lacks is
        # tuned in this run without rewriting the committed file
        import shutil
        import tempfile

        fd, copy = tempfile.mkstemp(prefix="eq_tune_", suffix=".json")
        os.close(fd)
        shutil.copyfile(TUNE_FILE, copy)
        os.environ["EQ_AUTOTUNE_CACHE"] = copy
        os.environ["EQ_TUNE_SOURCE"] = os.path.relpath(TUNE_FILE, ROOT)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every field runs on a single MI355X "
              "(sharding across GPUs is described, not implemented). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2105_01612_amd as eq

    eq.lib()
    log(f"[bench] workload={args.workload} op={args.op} steps={args.steps} warmup={args.warmup}")
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.workload == "grain_avg":
        print(json.dumps(run_grain_avg(args)), flush=True)
        return
    if args.workload == "inloop":
        print(json.dumps(run_inloop(args)), flush=True)
        return
    if args.workload == "persistent":
        print(json.dumps(run_persistent(args)), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 512 MiB device copies (read 512 MiB + write 512 MiB each)")
        del src, dst
    t = time.perf_counter()
    S32, desc = make_workload(args.workload, "fp32")
    log(f"[bench] generated input in {time.perf_counter() - t:.1f}s: {desc}")
    B, _, nz, ny, nx = S32.shape
    vox = B * nz * ny * nx

    r32 = run_gpu(S32, args.op, "fp32", args.steps, args.warmup, timing=not args.no_timing,
                  tune=not args.no_autotune)
    ms32 = r32["elapsed_s"] / args.steps * 1e3
    log(f"[bench] fp32 {args.op}: {ms32:.3f} ms/step")
    roof, per_pass = roofline(r32["stats"], r32["all_stats"], args.workload, vox, "fp32", removed=True)

    line = {
        "metric": METRIC,
        "value": vox / r32["elapsed_s"] * args.steps,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: " + desc,
        "config": {"workload": f"{args.workload}: {desc}; {args.op.upper()} operator, FP32 bulk with FP64 "
                               f"twiddles and symbols; step = eq_project (with removed part) + eq_residual",
                   "grid": [nx, ny, nz], "batch": B, "op": args.op, "prec": "fp32"},
        "p50_ms": statistics.median(r32["lat_ms"]),
        "p99_ms": float(np.percentile(r32["lat_ms"], 99)),
        "p10_ms": float(np.percentile(r32["lat_ms"], 10)),
        "p90_ms": float(np.percentile(r32["lat_ms"], 90)),
        "roofline": roof,
        "passes": per_pass,
        "hbm_frac_144B_schedule_min": (vox / r32["elapsed_s"] * args.steps) * 144 / (HBM_PEAK_GBS * 1e9),
        # read S, write S_eq only: what a fully fused path would still move
        "hbm_frac_compulsory_48B": (vox / r32["elapsed_s"] * args.steps) * 48 / (HBM_PEAK_GBS * 1e9),
        "residual_of_output": r32["norms"][0] if r32["norms"] else None,
        "tune": r32["tune"],
        "tune_source": tune_source(args),
        "paper_context": PAPER_CONTEXT,
    }
    if roof:
        # beside the slowest kernel's fraction: where the whole step stands against the schedule's
        # three-round-trip minimum
        roof["step_frac_of_144B_minimum"] = round(line["hbm_frac_144B_schedule_min"], 4)
    if r32["all_stats"]:
        # algorithmic bytes of every launch of one step, and the rate the whole step sustains
        step_bytes = sum(st["bytes_per_launch"] * st["launches"] for st in r32["all_stats"].values()) / args.steps
        line["step_bytes_per_voxel"] = round(step_bytes / vox, 2)
        line["hbm_frac_step_bytes"] = step_bytes / (ms32 * 1e-3) / (HBM_PEAK_GBS * 1e9)

    if not args.no_compare:
        # the projection alone (no removed part, no residual): 144 B/voxel is its three-pass minimum
        rp = run_gpu(S32, args.op, "fp32", args.steps, 2, with_residual=False, timing=False,
                     tune=not args.no_autotune, removed=False)
        msp = rp["elapsed_s"] / args.steps * 1e3
        log(f"[bench] fp32 {args.op} projection only: {msp:.3f} ms")
        line["project_only"] = {"ms": msp, "value": vox / (msp * 1e-3), "unit": "voxels/s",
                                "hbm_frac_144B_schedule_min": vox / (msp * 1e-3) * 144 / (HBM_PEAK_GBS * 1e9),
                                "tune": rp["tune"]}
        if roof:
            roof["project_only_frac_of_144B_minimum"] = round(line["project_only"]["hbm_frac_144B_schedule_min"], 4)
        del rp
    if args.workload == "batched" and not args.no_cpu_baseline:
        line["error_vs_oracle"] = batched_errors(S32, r32["out"].numpy(), args.op)
    if not args.no_compare and args.workload != "batched":
        S64 = S32.astype(np.float64)
        r64 = run_gpu(S64, args.op, "fp64", max(3, args.steps // 2), 2, timing=False, tune=not args.no_autotune)
        ms64 = r64["elapsed_s"] / max(3, args.steps // 2) * 1e3
        log(f"[bench] fp64 {args.op}: {ms64:.3f} ms/step")
        other = "cdo" if args.op == "ddo" else "ddo"
        rc = run_gpu(S32, other, "fp32", max(3, args.steps // 2), 2, timing=False, tune=not args.no_autotune)
        msc = rc["elapsed_s"] / max(3, args.steps // 2) * 1e3
        line["fp64"] = {"value": vox / (ms64 * 1e-3), "ms_per_step": ms64,
                        "p50_ms": statistics.median(r64["lat_ms"]), "p99_ms": float(np.percentile(r64["lat_ms"], 99)),
                        "hbm_frac_288B_schedule_min": vox / (ms64 * 1e-3) * 288 / (HBM_PEAK_GBS * 1e9)}
        line[f"{other}_fp32"] = {"value": vox / (msc * 1e-3), "ms_per_step": msc}
        if not args.no_cpu_baseline:
            ref, cb = cpu_baseline(S64[0], args.op)
            line["cpu_baseline"] = cb
            e32 = frob_err(r32["out"].numpy()[:1], ref[None])
            e64 = frob_err(r64["out"].numpy()[:1], ref[None])
            line["error_vs_oracle"] = {"fp32": {"rel_l2": e32[0], "max_abs_mpa": e32[1], "tol": 1e-5},
                                       "fp64": {"rel_l2": e64[0], "max_abs_mpa": e64[1], "tol": 1e-12},
                                       "roundoff_amplification": roundoff_amplification(S64[0], ref)}
            log(f"[bench] oracle {cb['sample']}; fp32 rel-L2 {e32[0]:.2e}, fp64 rel-L2 {e64[0]:.2e}")
            # the other operator's FP32 result against its own oracle
            import oracle

            os.environ["ORACLE_WORKERS"] = str(os.cpu_count() or 1)
            ref_o, _ = oracle.project(S64[0], other)
            eo = frob_err(rc["out"].numpy()[:1], ref_o[None])
            line[f"{other}_fp32"]["error_vs_oracle"] = {"rel_l2": eo[0], "max_abs_mpa": eo[1], "tol": 1e-5}
            log(f"[bench] {other} fp32 rel-L2 {eo[0]:.2e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
