"""EQ_F_PERSISTENT: the three passes of a batch as one launch over a device-side work queue.

Against the per-pass three-pass schedule with the same z radix schedule (zp_e = 4): bitwise
equal, field by field, for batches whose stages overlap across fields (below eight fields and
from eight on, where items are four times larger), both operators, with and without the
removed part, over repeated calls (the counters reset themselves) and graph replays.  Against the FP64 oracle: every field of 64 x 64^3 and 64 x 128^3 batches (the
batched workload's sizes), rel-L2 <= 1e-5."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2105_01612_amd import workload as wl

pytestmark = pytest.mark.gpu
W6 = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0]).reshape(6, 1, 1, 1)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def frob_rel(got, ref):
    d = got.astype(np.float64) - ref
    return math.sqrt(float(np.sum(W6 * d * d)) / float(np.sum(W6 * ref * ref)))


def batch(shape, n, seed, grains=30):
    return np.stack([wl.voronoi_field(wl.FieldSpec(shape, grains=grains, sigma_grain=100.0, sigma_noise=5.0,
                                                   seed=seed + b), dtype=np.float32) for b in range(n)])


@pytest.mark.parametrize("op", ["ddo", "cdo"])
@pytest.mark.parametrize("shape,b", [((64, 64, 64), 5), ((128, 64, 64), 3), ((256, 64, 64), 2), ((64, 128, 128), 3),
                                     ((128, 128, 128), 2), ((64, 64, 64), 9)])
def test_persistent_equals_three_pass(op, shape, b):
    import torch
    import paper_2105_01612_amd as eq

    nz, ny, nx = shape
    say("persistent", op, shape, b)
    S = batch(shape, b, 700 + nz + nx)
    x = torch.from_numpy(S).cuda()
    per = eq.plan(nx, ny, nz, batch=b, op=op, prec="fp32")
    per.tune(schedule=3, zp_e=4)
    assert per.get_tune()["zp_e"] == 4
    ps = eq.plan(nx, ny, nz, batch=b, op=op, prec="fp32", flags=["persistent"])
    assert ps.get_tune()["schedule"] == 3 and ps.get_tune()["zp_e"] == 4
    ref_out, ref_rem = torch.empty_like(x), torch.empty_like(x)
    per.project(x, ref_out, ref_rem)
    # a dependency wait that gave up is reported by the residual (the kernel always ends)
    ps.project(x, torch.empty_like(x))
    ps.residual(ref_out)
    say("  first persistent call done")
    for call in range(3):
        out, rem = torch.full_like(x, float("nan")), torch.full_like(x, float("nan"))
        y = x if call != 1 else x * 1.0
        ps.project(y, out, rem if call != 2 else None)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out), call
        if call != 2:
            assert torch.equal(rem, ref_rem), call
    norms = ps.residual(out)                 # also reports a dependency wait that gave up
    assert max(n[2] for n in norms) <= 2e-6
    for f in range(b):
        ref, _ = O.project(S[f].astype(np.float64), op)
        assert frob_rel(ref_out[f].cpu().numpy(), ref) <= 1e-5
    per.destroy()
    ps.destroy()


def test_persistent_graph_replay_and_timing():
    import torch
    import paper_2105_01612_amd as eq

    n, b = 64, 4
    S = batch((n, n, n), b, 900)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x = torch.from_numpy(S).cuda()
        eager = eq.plan(n, batch=b, op="ddo", prec="fp32", flags=["persistent"])
        ref = eager.project(x)
        g = eq.plan(n, batch=b, op="ddo", prec="fp32", flags=["persistent", "capture_graph"], stream=s)
        out = torch.empty_like(x)
        for i in range(4):
            out.zero_()
            g.project(x, out)
            s.synchronize()
            assert torch.equal(out, ref), i
            _ = eager.project(x * 1.0)
            torch.cuda.synchronize()
        eager.set_timing(True)
        eager.project(x)
        st = eager.pass_stats()
        eager.set_timing(False)
        assert st["persist"]["launches"] == 1 and st["persist"]["total_ms"] > 0
        assert st["plane_r2c"]["launches"] == 0 and st["z_proj"]["launches"] == 0
        eager.destroy()
        g.destroy()


def test_persistent_refuses_unsupported_plans():
    import paper_2105_01612_amd as eq

    for kw in (dict(nx=64, prec="fp64"), dict(nx=256, prec="fp32"), dict(nx=96, prec="fp32")):
        n = kw["nx"]
        with pytest.raises(eq.EqError) as ei:
            eq.plan(n, op="ddo", prec=kw["prec"], flags=["persistent"])
        assert ei.value.code == "EQ_ERR_ARG"


@pytest.mark.parametrize("n", [64, 128])
def test_persistent_batch_of_64_every_field_against_oracle(n):
    """64 fields of n^3 (300 grains each, seeds 300..363, as the batched workload), one
    persistent launch: the oracle error of every field."""
    import torch
    import paper_2105_01612_amd as eq

    say("persistent 64 x", n)
    specs = wl.batched_specs(n=n)
    S = np.stack([wl.voronoi_field(sp, dtype=np.float32) for sp in specs])
    x = torch.from_numpy(S).cuda()
    ps = eq.plan(n, batch=64, op="ddo", prec="fp32", flags=["persistent"])
    out = torch.empty_like(x)
    rem = torch.empty_like(x)
    ps.project(x, out, rem)
    norms = ps.residual(out)
    got = out.cpu().numpy()
    ps.destroy()
    del x, out, rem
    torch.cuda.empty_cache()
    errs = []
    for f in range(64):
        ref, _ = O.project(S[f].astype(np.float64), "ddo")
        errs.append(frob_rel(got[f], ref))
    say("  per-field rel-L2 max", max(errs), "median", float(np.median(errs)))
    assert max(errs) <= 1e-5
    assert max(v[2] for v in norms) <= 2e-6


def test_persistent_wait_that_gives_up_is_reported(monkeypatch):
    """A poll limit of one makes the z and inverse items give up waiting (every wait still ends,
    the launch completes); eq_residual then reports EQ_ERR_DEVICE for the plan, on every call."""
    import torch
    import paper_2105_01612_amd as eq

    monkeypatch.setenv("EQ_PERSIST_SPIN_LIMIT", "1")
    S = batch((64, 64, 64), 9, 950, grains=8)
    x = torch.from_numpy(S).cuda()
    ps = eq.plan(64, batch=9, op="ddo", prec="fp32", flags=["persistent"])
    out = ps.project(x)
    torch.cuda.synchronize()
    for _ in range(2):
        with pytest.raises(eq.EqError) as ei:
            ps.residual(out)
        assert ei.value.code == "EQ_ERR_DEVICE"
    ps.destroy()
    monkeypatch.delenv("EQ_PERSIST_SPIN_LIMIT")
    # a new plan is unaffected
    ok = eq.plan(64, batch=9, op="ddo", prec="fp32", flags=["persistent"])
    ok.project(x, out)
    ok.residual(out)
    ok.destroy()


@pytest.mark.parametrize("shape", [(64, 64, 64), (256, 64, 64), (128, 128, 128)])
@pytest.mark.parametrize("b", [1, 7, 8, 13])
def test_persistent_batch_counts_around_the_item_size_switch(shape, b):
    """Batches of 1, 7, 8 and 13 fields (items grow fourfold from eight fields on, and the queue's
    last step is partly empty for odd counts): bitwise equal to the per-pass three-pass schedule
    with the same z stage, with the removed part, both on the first call and on a repeated one."""
    import torch
    import paper_2105_01612_amd as eq

    nz, ny, nx = shape
    say("persistent batch count", shape, b)
    S = batch(shape, b, 1300 + b + nz, grains=10)
    x = torch.from_numpy(S).cuda()
    per = eq.plan(nx, ny, nz, batch=b, op="ddo", prec="fp32")
    per.tune(schedule=3, zp_e=4)
    ref, ref_rem = torch.empty_like(x), torch.empty_like(x)
    per.project(x, ref, ref_rem)
    ps = eq.plan(nx, ny, nz, batch=b, op="ddo", prec="fp32", flags=["persistent"])
    for call in range(2):
        out, rem = torch.full_like(x, float("nan")), torch.full_like(x, float("nan"))
        ps.project(x, out, rem)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(rem, ref_rem), call
    ps.residual(out)                         # reports a dependency wait that gave up
    per.destroy()
    ps.destroy()
