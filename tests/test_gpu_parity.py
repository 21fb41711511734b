"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: rel-L2 (Frobenius, off-diagonals weigh 2) <= 1e-12 for FP64 and <= 1e-5 for
FP32; FP32 runs are compared on the FP64 up-cast of the same FP32 input bytes.  The
removed part S - S_eq is held to the same bars relative to ||S - c0||_F: its absolute
rounding error is that of S_eq, so the size of the data the projection acts on, not
its own (possibly small) norm, is the scale.  The potential y is held to the bars
relative to its own norm.  Residual norms: relative to their own value.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2105_01612_amd import workload as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
W6 = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def torch_mod():
    import torch

    return torch


def eqmod():
    import paper_2105_01612_amd as eq

    return eq


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def frob(x):
    w = W6.reshape((6,) + (1,) * (x.ndim - 1)) if x.shape[0] == 6 else W6.reshape((1, 6) + (1,) * (x.ndim - 2))
    return math.sqrt(float(np.sum(w * x.astype(np.float64) ** 2)))


def rel_l2(got, ref):
    return frob(got - ref) / frob(ref)


def removed_rel(rem, ref_rem, S):
    """||rem - ref_rem||_F / ||S - c0||_F for one field (6, ...) or a batch."""
    S = np.asarray(S, dtype=np.float64)
    axes = tuple(range(S.ndim - 3, S.ndim))
    return frob(rem - ref_rem) / frob(S - S.mean(axis=axes, keepdims=True))


def to_dev(a, prec):
    torch = torch_mod()
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def run_project(S, op, prec, h=1.0, removed=True, flags=0, schedule=None, tuning=None):
    eq = eqmod()
    torch = torch_mod()
    batch = S.shape[0] if S.ndim == 5 else 1
    nz, ny, nx = S.shape[-3:]
    plan = eq.plan(nx, ny, nz, batch=batch, op=op, prec=prec, h=h, flags=flags)
    if tuning is not None:
        tuning(plan)
    if schedule is not None:
        plan.tune(schedule=schedule)
        assert plan.get_tune()["schedule"] == schedule
    x = to_dev(S, prec)
    out = torch.empty_like(x)
    rem = torch.empty_like(x) if removed else None
    plan.project(x, out, rem)
    torch.cuda.synchronize()
    res = (out.double().cpu().numpy(), rem.double().cpu().numpy() if removed else None)
    plan.destroy()
    return res


def upcast(S, prec):
    return S.astype(np.float32).astype(np.float64) if prec == "fp32" else S


# ----------------------------------------------------------------- stages ---

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 16), (20, 12, 30), (32, 48, 40)])
def test_forward_spectrum(prec, shape):
    """eq_debug_forward: half spectrum along z of the unnormalized forward DFT."""
    eq = eqmod()
    torch = torch_mod()
    say("forward", prec, shape)
    S = wl.random_field(shape, seed=3, scale=10.0)
    Su = upcast(S, prec)
    nz, ny, nx = shape
    plan = eq.plan(nx, ny, nz, op="ddo", prec=prec)
    spec = torch.empty(plan.spectrum_shape, dtype=plan.dtype, device="cuda")
    plan.debug_forward(to_dev(S, prec), spec)
    torch.cuda.synchronize()
    got = spec.double().cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.fftn(Su, axes=(1, 2, 3))[None, :, : nz // 2 + 1]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= (1e-14 if prec == "fp64" else 2e-6), err
    plan.destroy()


@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projection_kernel_on_spectrum(op, prec):
    """eq_debug_project_spectrum against the oracle's per-frequency P A P on identical spectra."""
    eq = eqmod()
    torch = torch_mod()
    shape = (12, 10, 16)
    nz, ny, nx = shape
    h = 0.6
    rng = np.random.default_rng(4)
    spec = rng.standard_normal((1, 6, nz // 2 + 1, ny, nx, 2))
    if prec == "fp32":
        spec = spec.astype(np.float32).astype(np.float64)
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=h)
    t = to_dev(spec, prec)
    plan.debug_project_spectrum(t)
    torch.cuda.synchronize()
    got = t.double().cpu().numpy()
    A = spec[0, ..., 0] + 1j * spec[0, ..., 1]
    sx = O.axis_symbol(op, nx, h)
    sy = O.axis_symbol(op, ny, h)
    sz = O.axis_symbol(op, nz, h)[: nz // 2 + 1]
    s = np.stack(np.broadcast_arrays(sx[None, None, :], sy[None, :, None], sz[:, None, None]))
    ref = O.matrix_to_voigt(O.project_spectrum_pap(O.voigt_to_matrix(A), s))
    g = got[0, ..., 0] + 1j * got[0, ..., 1]
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert err <= (1e-14 if prec == "fp64" else 1e-6), err
    plan.destroy()


# ------------------------------------------------------------ end to end ----

@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_config_small_fp64(op):
    """32^3, 20 grains, FP64: S_eq and the removed part against the oracle."""
    say("small fp64", op)
    S = wl.config_field("small")
    got, rem = run_project(S, op, "fp64")
    ref, ref_rem = O.project(S, op)
    assert rel_l2(got, ref) <= TOL["fp64"]
    assert removed_rel(rem, ref_rem, S) <= TOL["fp64"]
    assert np.max(np.abs(got + rem - S)) <= 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (20, 12, 30), (36, 40, 48), (96, 96, 96), (6, 10, 4)])
def test_project_parity(prec, op, shape):
    say("project", prec, op, shape)
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=12, sigma_grain=100.0, sigma_noise=5.0, sigma_grad=1.0,
                                      seed=sum(shape)))
    got, rem = run_project(S, op, prec, h=0.5)
    Su = upcast(S, prec)
    ref, ref_rem = O.project(Su, op, 0.5)
    assert rel_l2(got, ref) <= TOL[prec]
    assert removed_rel(rem, ref_rem, Su) <= TOL[prec]


# Three-pass schedule (xy planes resident on one workgroup): nx == ny in {64, 128, 256}
# (FP64 up to 128), nz in {64, 128, 256}; (nz, ny, nx) below.
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (128, 64, 64), (64, 128, 128), (256, 128, 128), (64, 256, 256)])
def test_three_pass_parity(prec, op, shape):
    eq = eqmod()
    if prec == "fp64" and shape[-1] > 128:
        plan = eq.plan(shape[2], shape[1], shape[0], op=op, prec=prec)
        assert plan.get_tune()["schedule"] == 5           # falls back to five passes
        with pytest.raises(eq.EqError) as ei:
            plan.tune(schedule=3)
        assert ei.value.code == "EQ_ERR_ARG"
        plan.destroy()
        return
    say("three-pass", prec, op, shape)
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=40, sigma_grain=100.0, sigma_noise=5.0, sigma_grad=1.0,
                                      seed=7 + sum(shape)))
    got3, rem3 = run_project(S, op, prec, h=0.5, schedule=3)
    Su = upcast(S, prec)
    ref, ref_rem = O.project(Su, op, 0.5)
    err3 = rel_l2(got3, ref)
    say("  rel-L2 three-pass", err3)
    assert err3 <= TOL[prec]
    assert removed_rel(rem3, ref_rem, Su) <= TOL[prec]
    got5, _ = run_project(S, op, prec, h=0.5, removed=False, schedule=5)
    assert rel_l2(got5, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_pass_batch_and_plane_edges(prec):
    """Batch of 2 on the three-pass route: each field equals its single-field run bitwise;
    Nyquist-corner and DC planes (checkerboards, constants) survive exactly as the oracle says."""
    n = 64
    rng = np.random.default_rng(11)
    x = np.arange(n)
    cb = ((-1.0) ** (x[:, None, None] + x[None, :, None] + x[None, None, :]))     # (N/2, N/2, N/2) mode
    f0 = wl.voronoi_field(wl.FieldSpec((n, n, n), grains=30, sigma_grain=100.0, sigma_noise=5.0, seed=21))
    f1 = rng.standard_normal((6, n, n, n)) * 10.0 + cb[None] * np.array([3.0, -1.0, 2.0, 0.5, 0.0, 1.0])[:, None, None, None]
    S = np.stack([f0, f1])
    gotb, _ = run_project(S, "ddo", prec, removed=False, schedule=3)
    for b in range(2):
        single, _ = run_project(S[b], "ddo", prec, removed=False, schedule=3)
        assert np.array_equal(single, gotb[b])
        ref, _ = O.project(upcast(S[b], prec), "ddo")
        assert rel_l2(gotb[b], ref) <= TOL[prec]


@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(16, 12, 32), (20, 8, 64), (8, 6, 128), (4, 4, 256), (4, 4, 512)])
def test_radix4_x_parity(op, shape):
    """FP32 with radix-4 x stages (the six-component x kernel holding 6 x 4 values per lane)."""
    eq = eqmod()
    torch = torch_mod()
    nz, ny, nx = shape
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=6, sigma_grain=80.0, sigma_noise=4.0, seed=nx + 1))
    plan = eq.plan(nx, ny, nz, op=op, prec="fp32")
    for rw in (0, 1, 2):
        plan.tune(schedule=5, radix4=1, rw_x=rw)
        assert plan.get_tune()["radix4"] == 1
        x = to_dev(S, "fp32")
        got = plan.project(x).double().cpu().numpy()
        ref, _ = O.project(upcast(S, "fp32"), op)
        assert rel_l2(got, ref) <= TOL["fp32"], rw
    plan.destroy()


@pytest.mark.parametrize("nx", [96, 160, 192, 384])
def test_radix4_on_3_5_smooth_x_takes_the_split_kernel(nx):
    """radix4 = 1 on a 3- or 5-smooth x edge (E = 12 or 20) with the x kernel left to the
    library: the split kernel serves it and the projection matches the oracle.  With the
    unsplit kernel asked for, radix4 is ignored there (no unsplit kernel has these schedules):
    the radix-8 line kernel runs, and the projection still matches."""
    eq = eqmod()
    shape = (4, 6, nx)
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=5, sigma_grain=80.0, sigma_noise=4.0, seed=nx + 1))
    ref, _ = O.project(upcast(S, "fp32"), "ddo")
    plan = eq.plan(nx, 6, 4, op="ddo", prec="fp32")
    plan.tune(schedule=5, radix4=1)
    t = plan.get_tune()
    assert t["radix4"] == 1 and t["xsplit"] == 2, t
    got = plan.project(to_dev(S, "fp32")).double().cpu().numpy()
    assert rel_l2(got, ref) <= TOL["fp32"]
    plan.tune(schedule=5, radix4=1, xsplit=1)
    t = plan.get_tune()
    assert t["radix4"] == 0 and t["xsplit"] == 1, t
    got = plan.project(to_dev(S, "fp32")).double().cpu().numpy()
    assert rel_l2(got, ref) <= TOL["fp32"]
    plan.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape,radix,P", [((16, 12, 32), {}, 4), ((20, 6, 64), {}, 8), ((8, 10, 128), {}, 16),
                                           ((4, 10, 256), {}, 32), ((6, 18, 96), {}, 4), ((6, 10, 160), {}, 4),
                                           ((4, 6, 192), {}, 8), ((6, 10, 128), {"radix4": 1}, 32),
                                           ((6, 18, 96), {"radix4": 1}, 8), ((6, 10, 160), {"radix4": 1}, 8),
                                           ((4, 6, 192), {"radix4": 1}, 16), ((4, 6, 384), {"radix4": 1}, 32),
                                           ((4, 6, 256), {"radix16": 1}, 16), ((4, 6, 512), {}, 64)])
def test_xsplit_parity(prec, op, shape, radix, P):
    """The x pass split over wavefront halves (three rows per lane, frequencies divided
    between the halves): projection, the spectral divergence of the CDO residual and the
    potential, against the oracle, for ragged row counts and rows per workgroup that do
    not fill a wavefront.  P = nx / E lanes per row."""
    eq = eqmod()
    torch = torch_mod()
    nz, ny, nx = shape
    if "radix4" in radix and prec == "fp64":
        # radix-4 x stages exist in FP32 only: an FP64 plan accepts the knob and reports it off
        plan = eq.plan(nx, ny, nz, op=op, prec=prec)
        plan.tune(schedule=5, radix4=1)
        assert plan.get_tune()["radix4"] == 0
        plan.destroy()
        return
    say("xsplit", prec, op, shape, radix)
    h = 0.7
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=6, sigma_grain=80.0, sigma_noise=4.0, sigma_grad=1.0,
                                      seed=nx + ny))
    Su = upcast(S, prec)
    ref, ref_rem = O.project(Su, op)
    ref_pot = O.removed_potential(Su, op, h)
    ref_norms = O.residual_norms(Su, op, h)
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=h)
    eb = 8 if prec == "fp32" else 16

    def lds_ok(rw):   # six skewed lines per row of every row the wavefronts cover, within 64 KiB
        rows = -(-rw * 2 * P // 64) * 64 // (2 * P)
        return 6 * rows * (nx + nx // 16 + 1) * eb <= 65536

    for rw in [r for r in sorted({0, 1, 3, max(1, 32 // P)}) if r == 0 or lds_ok(r)]:
        plan.tune(schedule=5, rw_x=rw, xsplit=2, **radix)
        assert plan.get_tune()["xsplit"] == 2
        x = to_dev(S, prec)
        out = torch.empty_like(x)
        rem = torch.empty_like(x)
        plan.project(x, out, rem)
        assert rel_l2(out.double().cpu().numpy(), ref) <= TOL[prec], rw
        assert removed_rel(rem.double().cpu().numpy(), ref_rem, Su) <= TOL[prec], rw
        Y = plan.potential(x).double().cpu().numpy()
        assert np.linalg.norm(Y - ref_pot) / np.linalg.norm(ref_pot) <= TOL[prec], rw
        norms = plan.residual(x)[0]
        tol = TOL[prec]
        for g, r in zip(norms, ref_norms):
            assert abs(g - r) <= tol * abs(r), (rw, norms, ref_norms)
    # the unsplit kernel gives the same projection to rounding
    plan.tune(schedule=5, xsplit=1, **radix)
    assert plan.get_tune()["xsplit"] == 1
    x = to_dev(S, prec)
    assert rel_l2(plan.project(x).double().cpu().numpy(), ref) <= TOL[prec]
    plan.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(4, 6, 1024), (6, 1024, 4), (1024, 4, 6), (4, 6, 960), (1000, 4, 6),
                                   (6, 768, 4)])
def test_maximum_edges(prec, op, shape):
    """Edges at the 1024 limit and 3/5-smooth edges near it, on every axis."""
    say("max edge", prec, op, shape)
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=5, sigma_grain=50.0, sigma_noise=3.0, seed=sum(shape)))
    got, rem = run_project(S, op, prec)
    ref, ref_rem = O.project(upcast(S, prec), op)
    assert rel_l2(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_equals_single_and_oracle(prec):
    eq = eqmod()
    torch = torch_mod()
    n = 32
    specs = wl.batched_specs(n=n, fields=3, grains=30, first_seed=300)
    S = np.stack([wl.voronoi_field(sp) for sp in specs])
    gotb, _ = run_project(S, "ddo", prec, removed=False)
    for b in range(3):
        single, _ = run_project(S[b], "ddo", prec, removed=False)
        assert np.array_equal(single, gotb[b])
        ref, _ = O.project(upcast(S[b], prec), "ddo")
        assert rel_l2(gotb[b], ref) <= TOL[prec]


def test_in_place_and_determinism():
    eq = eqmod()
    torch = torch_mod()
    S = wl.config_field("small")
    plan = eq.plan(32, op="ddo", prec="fp64")
    x = to_dev(S, "fp64")
    a = plan.project(x.clone())
    b = plan.project(x.clone())
    y = x.clone()
    plan.project(y, y)                  # in place
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, y)
    plan.destroy()


@pytest.mark.parametrize("route", [
    # (prec, grid, batch, schedule asked for, flags, schedule taken)
    ("fp32", (96, 96, 96), 1, None, (), 5),                    # five passes (3/5-smooth edge)
    ("fp32", (64, 64, 64), 2, 5, (), 5),                       # five passes on a three-pass grid
    ("fp32", (64, 64, 64), 2, 3, (), 3),                       # three passes
    ("fp64", (64, 64, 64), 2, 3, (), 3),
    ("fp32", (128, 128, 128), 1, 3, (), 3),
    ("fp32", (64, 64, 64), 9, None, ("persistent",), 3),       # one launch, items of four planes
    ("fp32", (128, 128, 128), 2, None, ("persistent",), 3),
])
def test_in_place_on_every_route(route):
    """s_eq == s_in gives the bits of the out-of-place call, with and without the removed part:
    the last pass reads each input value it overwrites before writing it."""
    eq = eqmod()
    torch = torch_mod()
    prec, (nz, ny, nx), b, schedule, flags, taken = route
    say("in place", route)
    S = np.stack([wl.voronoi_field(wl.FieldSpec((nz, ny, nx), grains=12, sigma_grain=80.0, sigma_noise=6.0,
                                                seed=70 + f)) for f in range(b)])
    x = to_dev(S, prec)
    plan = eq.plan(nx, ny, nz, batch=b, op="ddo", prec=prec, flags=list(flags))
    if schedule is not None:
        plan.tune(schedule=schedule)
    assert plan.get_tune()["schedule"] == taken
    ref, ref_rem = torch.empty_like(x), torch.empty_like(x)
    plan.project(x, ref, ref_rem)
    for with_removed in (True, False):
        y = x.clone()
        rem = torch.full_like(x, float("nan")) if with_removed else None
        plan.project(y, y, rem)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), with_removed
        if with_removed:
            assert torch.equal(rem, ref_rem)
    plan.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_invariants_on_gpu_output(prec):
    eq = eqmod()
    torch = torch_mod()
    n = 48
    S = wl.voronoi_field(wl.FieldSpec((n, n, n), grains=40, sigma_grain=100.0, sigma_noise=5.0, seed=8))
    for op in ("cdo", "ddo"):
        plan = eq.plan(n, op=op, prec=prec)
        x = to_dev(S, prec)
        y = plan.project(x)
        z = plan.project(y)
        torch.cuda.synchronize()
        Y = y.double().cpu().numpy()
        Z = z.double().cpu().numpy()
        Su = upcast(S, prec)
        tol = 1e-12 if prec == "fp64" else 2e-6
        # idempotent
        assert rel_l2(Z, Y) <= tol
        # mean kept
        assert np.abs(Y.mean(axis=(1, 2, 3)) - Su.mean(axis=(1, 2, 3))).max() <= tol * np.abs(Su).max() * 10
        # divergence-free in the same operator (oracle residual of the GPU output)
        l2, mx, rel = O.residual_norms(Y, op)
        assert rel <= (1e-14 if prec == "fp64" else 1e-6)
        # orthogonality of removed part and the demeaned result
        R = Su - Y
        dev = Y - Y.mean(axis=(1, 2, 3), keepdims=True)
        assert abs(O.frobenius_dot(R, dev)) <= (1e-12 if prec == "fp64" else 1e-5) * O.frobenius_norm(R) * O.frobenius_norm(dev)
        plan.destroy()


# -------------------------------------------------------- zero-stress buffer ---

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("case", [
    ((16, 24, 20), (13, 17), (3, 4)),     # odd sample, interior
    ((16, 24, 20), (20, 11), (0, 13)),    # full width, flush with the top edge
    ((12, 30, 36), (25, 1), (11, 0)),     # one row
    ((64, 64, 64), (40, 48), (12, 8)),    # a grid the three-pass schedule would otherwise take
])
def test_project_embedded_parity(op, prec, case):
    eq = eqmod()
    torch = torch_mod()
    (nz, ny, nx), (nx0, ny0), (ox, oy) = case
    say("embedded", op, prec, case)
    S = wl.voronoi_field(wl.FieldSpec((nz, ny0, nx0), grains=8, sigma_grain=60.0, sigma_noise=4.0, seed=nx0 + ny0))
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=0.9)
    x = to_dev(S, prec)
    rem = torch.empty_like(x)
    y = plan.project_embedded(x, nx0, ny0, ox, oy, s_removed=rem)
    torch.cuda.synchronize()
    ref, ref_rem = O.project_embedded(upcast(S, prec), (nx, ny), (ox, oy), op, 0.9)
    got = y.double().cpu().numpy()
    assert rel_l2(got, ref) <= TOL[prec]
    assert removed_rel(rem.double().cpu().numpy(), ref_rem, upcast(S, prec)) <= TOL[prec]
    # in place gives the same bits
    z = x.clone()
    plan.project_embedded(z, nx0, ny0, ox, oy, s_eq=z)
    torch.cuda.synchronize()
    assert torch.equal(z, y)
    plan.destroy()


def test_project_embedded_rejects_bad_geometry():
    eq = eqmod()
    torch = torch_mod()
    plan = eq.plan(16, op="ddo", prec="fp32")
    x = torch.zeros((6, 16, 8, 8), dtype=torch.float32, device="cuda")
    for nx0, ny0, ox, oy in ((8, 8, 9, 0), (8, 8, 0, -1), (8, 8, 0, 9)):
        with pytest.raises(eq.EqError) as ei:
            plan.project_embedded(x, nx0, ny0, ox, oy)
        assert ei.value.code == "EQ_ERR_ARG"
    plan.destroy()


# ------------------------------------------- potential of the removed part ---

@pytest.mark.parametrize("shape", [(16, 24, 20), (6, 10, 4), (32, 32, 32)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_potential_parity(op, prec, shape):
    """eq_potential vs the oracle's least-squares potential; and the GPU's own removed
    part equals the symmetric gradient of the GPU potential."""
    eq = eqmod()
    torch = torch_mod()
    say("potential", op, prec, shape)
    h = 0.6
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=10, sigma_grain=50.0, sigma_noise=3.0, sigma_grad=1.0,
                                      seed=13 + sum(shape)))
    Su = upcast(S, prec)
    nz, ny, nx = shape
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=h)
    x = to_dev(S, prec)
    y = plan.potential(x)
    out = torch.empty_like(x)
    rem = torch.empty_like(x)
    plan.project(x, out, rem)
    torch.cuda.synchronize()
    Y = y.double().cpu().numpy()
    ref = O.removed_potential(Su, op, h)
    err = float(np.linalg.norm(Y - ref) / np.linalg.norm(ref))
    say("  rel-L2", err)
    assert err <= TOL[prec]
    # the GPU's own removed part is the symmetric gradient of the GPU's potential
    sg = O.sym_grad_central_difference(Y, h) if op == "ddo" else O.sym_grad(Y, op, h)
    assert removed_rel(sg, rem.double().cpu().numpy(), Su) <= TOL[prec]
    plan.destroy()


def test_potential_rejects_overlap():
    eq = eqmod()
    torch = torch_mod()
    plan = eq.plan(8, op="ddo", prec="fp64")
    x = torch.zeros((6, 8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(eq.EqError) as ei:
        plan.potential(x, x[:3])
    assert ei.value.code == "EQ_ERR_ARG"
    plan.destroy()


# -------------------------------------------------------------- residual ----

@pytest.mark.parametrize("shape", [(16, 24, 20), (6, 10, 4), (40, 32, 96), (8, 120, 72)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_residual_parity(op, prec, shape):
    eq = eqmod()
    torch = torch_mod()
    nz, ny, nx = shape
    h = 0.8
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=10, sigma_grain=50.0, sigma_noise=3.0, seed=5))
    Su = upcast(S, prec)
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=h)
    x = to_dev(S, prec)
    div = torch.empty((1, 3, nz, ny, nx), dtype=plan.dtype, device="cuda")
    norms = plan.residual(x, div)[0]
    norms2 = plan.residual(x)[0]
    ref = O.residual_norms(Su, op, h)
    rdiv = O.divergence(Su, op, h)
    tol = TOL[prec]
    for g, r in zip(norms, ref):
        assert abs(g - r) <= tol * abs(r), (norms, ref)
    assert norms == norms2
    if op == "ddo":
        # batched residual: each field's norms equal its single-field norms bitwise
        plan_b = eq.plan(nx, ny, nz, batch=3, op=op, prec=prec, h=h)
        xb = torch.stack([x[0] * 1.0, x[0] * -0.5, x[0] + 3.0]) if x.dim() == 5 else torch.stack([x, -0.5 * x, x + 3.0])
        nb = plan_b.residual(xb)
        assert nb[0] == norms
        plan_b.destroy()
    d = div.double().cpu().numpy()[0]
    assert np.abs(d - rdiv).max() <= tol * np.abs(rdiv).max() * 10
    plan.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_residual_plain_load_path(prec, monkeypatch):
    """The DDO stencil's plain-load path (taken when a component array passes 2 GB)
    against the oracle, forced on a small grid."""
    eq = eqmod()
    shape = (40, 32, 96)
    nz, ny, nx = shape
    h = 0.8
    S = wl.voronoi_field(wl.FieldSpec(shape, grains=10, sigma_grain=50.0, sigma_noise=3.0, seed=5))
    Su = upcast(S, prec)
    ref = O.residual_norms(Su, "ddo", h)
    tol = TOL[prec]
    for flag in ("0", "1"):
        monkeypatch.setenv("EQ_DDO_BUF", flag)
        plan = eq.plan(nx, ny, nz, op="ddo", prec=prec, h=h)
        norms = plan.residual(to_dev(S, prec))[0]
        for g, r in zip(norms, ref):
            assert abs(g - r) <= tol * abs(r), (flag, norms, ref)
        plan.destroy()


def test_residual_of_projection_is_roundoff():
    eq = eqmod()
    n = 64
    S = wl.voronoi_field(wl.FieldSpec((n, n, n), grains=60, sigma_grain=100.0, sigma_noise=5.0, seed=9))
    for prec, bound in (("fp64", 1e-14), ("fp32", 2e-6)):
        for op in ("cdo", "ddo"):
            plan = eq.plan(n, op=op, prec=prec)
            x = to_dev(S, prec)
            before = plan.residual(x)[0]
            after = plan.residual(plan.project(x))[0]
            assert before[2] > 1e-3
            assert after[2] <= bound, (prec, op, after)
            plan.destroy()


# ------------------------------------------------------------ ABI paths -----

def test_check_finite_flag():
    eq = eqmod()
    torch = torch_mod()
    S = wl.random_field((8, 8, 8), seed=1)
    S[2, 3, 4, 5] = np.nan
    plan = eq.plan(8, op="ddo", prec="fp64", flags=["check_finite"])
    with pytest.raises(eq.EqError) as ei:
        plan.project(to_dev(S, "fp64"))
    assert ei.value.code == "EQ_ERR_NONFINITE"
    S[2, 3, 4, 5] = 0.0
    plan.project(to_dev(S, "fp64"))
    plan.destroy()


def test_fault_injection_alloc(monkeypatch):
    eq = eqmod()
    monkeypatch.setenv("EQ_FAULT_INJECT", "alloc")
    with pytest.raises(eq.EqError) as ei:
        eq.plan(16, op="ddo", prec="fp64")
    assert ei.value.code == "EQ_ERR_NOMEM"


def test_aliasing_rejected():
    eq = eqmod()
    torch = torch_mod()
    plan = eq.plan(8, op="ddo", prec="fp64")
    x = to_dev(wl.random_field((8, 8, 8), seed=2), "fp64")
    with pytest.raises(eq.EqError) as ei:
        plan.project(x, torch.empty_like(x), x)
    assert ei.value.code == "EQ_ERR_ARG"
    plan.destroy()


@pytest.mark.parametrize("n", [32, 64])
def test_graph_replay_matches_eager(n):
    """Captured graph replays (several, with eager work and syncs between) equal eager runs
    (32^3: five-pass schedule, 64^3: three-pass)."""
    eq = eqmod()
    torch = torch_mod()
    s = torch.cuda.Stream()
    S = wl.config_field("small") if n == 32 else wl.voronoi_field(wl.FieldSpec((n, n, n), grains=20, sigma_grain=100.0, sigma_noise=5.0, seed=3))
    with torch.cuda.stream(s):
        eager = eq.plan(n, op="ddo", prec="fp32")
        graph = eq.plan(n, op="ddo", prec="fp32", flags=["capture_graph"])
        x = to_dev(S, "fp32")
        ref = eager.project(x)
        out = torch.empty_like(x)
        rem = torch.empty_like(x)
        for i in range(4):
            out.zero_()
            graph.project(x, out, rem)
            s.synchronize()
            assert torch.equal(out, ref), i
            assert torch.equal(rem, x - ref) or torch.allclose(rem, x - ref, atol=1e-4)
            _ = eager.project(x * 1.0)         # unrelated eager work between replays
            torch.cuda.synchronize()
    eager.destroy()
    graph.destroy()


def test_timing_stats():
    eq = eqmod()
    torch = torch_mod()
    plan = eq.plan(32, op="ddo", prec="fp32")
    x = to_dev(wl.config_field("small"), "fp32")
    plan.set_timing(True)
    for _ in range(3):
        plan.project(x)
    st = plan.pass_stats()
    for name in ("z_r2c", "y_fwd", "x_proj", "y_inv", "z_c2r"):
        assert st[name]["launches"] == 3 and st[name]["total_ms"] > 0 and st[name]["bytes_per_launch"] > 0
    plan.reset_stats()
    assert plan.pass_stats()["x_proj"]["launches"] == 0
    # one pass bracketed: only its launches are counted
    plan.set_timing(True, only="z_c2r")
    out = plan.project(x)
    plan.residual(out)
    st = plan.pass_stats()
    assert st["z_c2r"]["launches"] == 1 and st["z_c2r"]["total_ms"] > 0
    assert all(v["launches"] == 0 for k, v in st.items() if k != "z_c2r")
    with pytest.raises(eq.EqError):
        plan.set_timing(True, only="no_such_pass")
    plan.set_timing(False)
    plan.destroy()
    plan = eq.plan(64, op="ddo", prec="fp32")
    x = to_dev(wl.voronoi_field(wl.FieldSpec((64, 64, 64), grains=20, sigma_grain=100.0, sigma_noise=5.0, seed=4)), "fp32")
    plan.set_timing(True)
    for _ in range(2):
        plan.project(x)
    st = plan.pass_stats()
    for name in ("plane_r2c", "z_proj", "plane_c2r"):
        assert st[name]["launches"] == 2 and st[name]["total_ms"] > 0 and st[name]["bytes_per_launch"] > 0
    assert st["z_r2c"]["launches"] == 0
    plan.destroy()


# ------------------------------------------------------------- full size ----

@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_headline_256_parity(prec, bench_tuning):
    """256^3, 1000 grains with gradients: the benchmark workload in the launch configuration the
    benchmark times (the committed tuning), whole-field oracle."""
    say("headline 256", prec)
    S = wl.config_field("headline", dtype=np.float32 if prec == "fp32" else np.float64)
    got, rem = run_project(S, "ddo", prec, tuning=bench_tuning)
    ref, _ = O.project(S.astype(np.float64), "ddo")
    err = rel_l2(got, ref)
    say("headline rel-L2", prec, err, "max-abs", float(np.abs(got - ref).max()))
    assert err <= TOL[prec]
