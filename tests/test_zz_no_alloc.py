"""eq_residual_noalloc (the residual with its scratch in a static device array) against
eq_residual (the plan's allocated scratch), through the C ABI: two calls in a row, the
second on a smaller input, FP32 and FP64.  The norms are FP64 results of the same kernels
and reduction order; only the final square roots and division run on the device instead of
the host, so they agree to the FP64 bar (1e-12 relative); the divergence fields are the same
kernel's output and agree bit for bit."""
import numpy as np
import pytest

from paper_2105_01612_amd import workload as wl

pytestmark = pytest.mark.gpu


def _fields(shape, batch, seed, prec):
    dt = np.float32 if prec == "fp32" else np.float64
    return np.stack([wl.voronoi_field(wl.FieldSpec(shape, grains=9, sigma_grain=80.0, sigma_noise=4.0, sigma_grad=1.0,
                                                   seed=seed + b), dtype=dt) + 300.0 for b in range(batch)])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_residual_equals_plan_residual(prec):
    import torch
    import paper_2105_01612_amd as eq

    h = 0.7
    stream = torch.cuda.Stream()
    # two calls in a row on the same static scratch, the second on a smaller input
    for (nz, ny, nx), batch, seed in (((48, 40, 64), 5, 11), ((16, 12, 20), 2, 23)):
        S = _fields((nz, ny, nx), batch, seed, prec)
        x = torch.from_numpy(S).cuda()
        plan = eq.plan(nx, ny, nz, batch=batch, op="ddo", prec=prec, h=h)
        div_ref = torch.empty((batch, 3, nz, ny, nx), dtype=x.dtype, device="cuda")
        ref = plan.residual(x, div_ref)
        plan.destroy()
        norms = torch.full((batch, 3), float("nan"), dtype=torch.float64, device="cuda")
        div = torch.full_like(div_ref, float("nan"))
        with torch.cuda.stream(stream):
            eq.residual_noalloc(x, norms, nx, ny, nz, batch=batch, prec=prec, h=h, div_out=div, stream=stream)
        stream.synchronize()
        got = norms.cpu().numpy()
        for b in range(batch):
            for k in range(3):
                r = ref[b][k]
                assert abs(got[b, k] - r) <= 1e-12 * abs(r), (prec, (nz, ny, nx), b, k, got[b, k], r)
        assert torch.equal(div, div_ref)
        # without the divergence field: the same norms
        norms2 = torch.zeros_like(norms)
        with torch.cuda.stream(stream):
            eq.residual_noalloc(x, norms2, nx, ny, nz, batch=batch, prec=prec, h=h, stream=stream)
        stream.synchronize()
        assert torch.equal(norms2, norms)


def test_noalloc_residual_refuses_before_any_device_work():
    import torch
    import paper_2105_01612_amd as eq

    x = torch.zeros((65, 6, 4, 4, 4), dtype=torch.float64, device="cuda")
    norms = torch.zeros((65, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(eq.EqError) as ei:
        eq.residual_noalloc(x, norms, 4, batch=65)
    assert ei.value.code == "EQ_ERR_SIZE"
