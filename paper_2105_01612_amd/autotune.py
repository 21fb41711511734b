"""Autotuner for libeq plans: radix schedule per axis and launch shape per pass.

Every knob (eq_plan_tune) affects one kind of pass only -- the z passes, the y
passes, the x pass or the three-pass z projection -- so the search is per pass:

1. five-pass radix schedule: time the plan once with every axis on radix-8 stages
   and once with every axis on radix-16 stages; each axis keeps whichever its own
   passes ran faster with;
2. five-pass tile shapes: sweep tx_z, tx_y and rw_x, each against its own pass time, then
   radix-4 x stages with a few rw_x values against the x pass;
3. where the grid allows the three-pass schedule: sweep tc_zp against the z
   projection's time, then keep whichever schedule projects faster in total.

Times come from the plan's per-pass hipEvents (eq_plan_pass_stats) over a few
projections of the caller's data.  Results are cached as JSON keyed by
(gfx arch, grid, batch, precision, operator) at $EQ_AUTOTUNE_CACHE, default
~/.cache/eqproj/autotune.json.  Tuning never changes what is computed: every
setting runs the same transform (radix changes only reorder rounding).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

from . import EqError

CACHE_ENV = "EQ_AUTOTUNE_CACHE"
Z_PASSES = ("z_r2c", "z_c2r")
Y_PASSES = ("y_fwd", "y_inv")
X_PASSES = ("x_proj",)
FIVE_PASSES = Z_PASSES + Y_PASSES + X_PASSES
THREE_PASSES = ("plane_r2c", "z_proj", "plane_c2r")


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "eqproj", "autotune.json"))


def _arch() -> str:
    import torch

    return getattr(torch.cuda.get_device_properties(torch.cuda.current_device()), "gcnArchName", "gfx")


def cache_key(plan, arch: Optional[str] = None) -> str:
    arch = arch or _arch()
    return f"{arch}|{plan.nx}x{plan.ny}x{plan.nz}|b{plan.batch}|{plan.prec}|{plan.op}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    try:
        with open(path or cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply_cached(plan, path: Optional[str] = None) -> Optional[dict]:
    """Apply the cached tuning of the plan's configuration (the file at `path`, else the default
    cache) and return it; without an entry, return None and leave the plan's defaults.  Never
    searches, so it is cheap enough for plans made while requests are being served."""
    entry = load_cache(path).get(cache_key(plan))
    if not entry:
        return None
    plan.tune(**entry["tune"])
    return entry["tune"]


def save_cache(cache: Dict[str, dict]) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _pass_times(plan, x, out, rem, reps: int) -> Dict[str, float]:
    import torch

    for _ in range(2):
        plan.project(x, out, rem)
    torch.cuda.synchronize()
    plan.reset_stats()
    plan.set_timing(True)
    for _ in range(reps):
        plan.project(x, out, rem)
    stats = plan.pass_stats()
    plan.set_timing(False)
    return {k: v["total_ms"] / v["launches"] for k, v in stats.items() if v["launches"]}


def _cost(times: Dict[str, float], passes) -> float:
    return sum(times.get(p, 0.0) for p in passes)


def autotune(plan, x, out, rem=None, reps: int = 5, use_cache: bool = True, verbose: bool = False) -> dict:
    """Tune `plan` on the caller's buffers (x -> out, rem); apply and return the result."""
    key = cache_key(plan)
    cache = load_cache() if use_cache else {}
    if key in cache:
        plan.tune(**cache[key]["tune"])
        return dict(cache[key], from_cache=True)

    def trial(**kw):
        try:
            plan.tune(**kw)
        except EqError:
            return None
        return _pass_times(plan, x, out, rem, reps)

    # 1. radix schedule per axis (five passes)
    t8 = trial(radix16=0, schedule=5)
    t16 = trial(radix16=7, schedule=5)
    mask = 0
    if t16 is not None and t8 is not None:
        if _cost(t16, X_PASSES) < _cost(t8, X_PASSES):
            mask |= 1
        if _cost(t16, Y_PASSES) < _cost(t8, Y_PASSES):
            mask |= 2
        if _cost(t16, Z_PASSES) < _cost(t8, Z_PASSES):
            mask |= 4
    best = {"tx_y": 0, "tx_z": 0, "rw_x": 0, "chunk": 0, "radix16": mask, "schedule": 5, "tc_zp": 0, "radix4": 0,
            "xsplit": 0, "zp_e": 0}
    base = trial(**best)
    log = {"radix16_all8": t8, "radix16_all16": t16, "default_shapes": base}

    # 2. tile shapes, one knob per pass kind
    for knob, passes, values in (("tx_z", Z_PASSES, (8, 16, 32, 64, 128)),
                                 ("tx_y", Y_PASSES, (4, 8, 16, 32, 64)),
                                 ("rw_x", X_PASSES, (1, 2, 3, 4, 8))):
        best_v, best_c = best[knob], _cost(base, passes) if base else float("inf")
        for v in values:
            t = trial(**dict(best, **{knob: v}))
            if t is None:
                continue
            c = _cost(t, passes)
            log[f"{knob}={v}"] = c
            if c < best_c:
                best_v, best_c = v, c
        best[knob] = best_v
    # x kernel: six components per lane or split over wavefront halves, radix-8 or
    # radix-4 stages (fewer registers per lane), rows per workgroup
    best_x = _cost(trial(**best) or {}, X_PASSES) or float("inf")
    for xsplit in (1, 2):
        for radix4 in (0, 1):
            for rw in (0, 1, 2, 4, 8):
                t = trial(**dict(best, xsplit=xsplit, radix4=radix4, rw_x=rw))
                got = plan.get_tune()
                if t is None or got["radix4"] != radix4 or got["xsplit"] != xsplit:
                    continue
                c = _cost(t, X_PASSES)
                log[f"xsplit={xsplit} radix4={radix4} rw_x={rw}"] = c
                if c < best_x:
                    best_x = c
                    best = dict(best, xsplit=xsplit, radix4=radix4, rw_x=rw)
    five = trial(**best)
    cost5 = _cost(five, FIVE_PASSES) if five else float("inf")
    # 3. three-pass schedule, where the grid allows it
    three = trial(**dict(best, schedule=3))
    if three is not None:
        best3, c3 = dict(best, schedule=3), _cost(three, ("z_proj",))
        for v in (1, 2, 4, 8, 16, 32):
            t = trial(**dict(best3, tc_zp=v))
            if t is None:
                continue
            c = _cost(t, ("z_proj",))
            log[f"tc_zp={v}"] = c
            if c < c3:
                best3, c3 = dict(best3, tc_zp=v), c
        # the z projection with four elements per thread (FP32): half the registers per thread
        for v in (4, 8, 16):
            t = trial(**dict(best3, zp_e=4, tc_zp=v))
            if t is None or plan.get_tune()["zp_e"] != 4:
                continue
            c = _cost(t, ("z_proj",))
            log[f"zp_e=4 tc_zp={v}"] = c
            if c < c3:
                best3, c3 = dict(best3, zp_e=4, tc_zp=v), c
        t3 = trial(**best3)
        cost3 = _cost(t3, THREE_PASSES)
        log["project_ms_five"], log["project_ms_three"] = cost5, cost3
        if cost3 < cost5:
            best = best3
    plan.tune(**best)
    final = _pass_times(plan, x, out, rem, reps)
    result = {"tune": best, "resolved": plan.get_tune(), "pass_ms": final,
              "project_ms": sum(final.get(p, 0.0) for p in FIVE_PASSES + THREE_PASSES)}
    if verbose:
        result["search"] = log
    if use_cache:
        cache = load_cache()
        cache[key] = {k: v for k, v in result.items() if k != "search"}
        save_cache(cache)
    result["from_cache"] = False
    return result
