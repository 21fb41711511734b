"""Host-only checks of the C ABI: the library loads, exports every entry point that
include/eq.h declares, and rejects bad descriptors with exact status codes before
any device call.  No compute calls are made here."""
import ctypes
import os
import re

import pytest

import paper_2105_01612_amd as eq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eq_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    L = eq.lib()
    names = declared_functions()
    assert "eq_plan" in names and "eq_project" in names and "eq_residual" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in eq.h but not exported"
    assert set(names) == set(eq.exported_symbols)
    assert "gfx950" in eq.version()


def test_status_strings():
    L = eq.lib()
    for code, name in eq.STATUS.items():
        assert L.eq_status_str(code).decode() == name
    assert L.eq_status_str(99).decode() == "EQ_ERR_UNKNOWN"


def _plan_status(**kw):
    base = dict(nx=32, ny=32, nz=32, batch=1, op="ddo", prec="fp64", h=1.0, flags=0)
    base.update(kw)
    d = eq._desc(**base)
    h = ctypes.c_void_p()
    st = eq.lib().eq_plan(ctypes.byref(d), None, ctypes.byref(h))
    assert not h.value
    return st


@pytest.mark.parametrize("kw,code", [
    (dict(nx=33), 2), (dict(ny=14), 2), (dict(nz=2), 2), (dict(nx=2048), 2), (dict(nx=0), 2),
    (dict(nx=-8), 2), (dict(nx=28), 2),          # 28 = 4 * 7: prime factor 7
    (dict(nx=450), 2), (dict(nx=900), 2),        # x pass would need > 1024 threads
    (dict(batch=0), 1), (dict(batch=-3), 1), (dict(op=2), 1), (dict(prec=7), 1),
    (dict(h=0.0), 1), (dict(h=-1.0), 1), (dict(h=float("nan")), 1), (dict(h=float("inf")), 1),
    (dict(flags=4), 1), (dict(flags=64), 1),
])
def test_plan_rejects_bad_descriptors(kw, code):
    assert _plan_status(**kw) == code
    assert eq.lib().eq_last_error().decode() != ""


def test_null_arguments():
    L = eq.lib()
    h = ctypes.c_void_p()
    assert L.eq_plan(None, None, ctypes.byref(h)) == 1
    d = eq._desc(8, 8, 8, 1, "ddo", "fp64", 1.0, 0)
    assert L.eq_plan(ctypes.byref(d), None, None) == 1
    assert L.eq_project(None, None, None, None) == 1
    norms = (ctypes.c_double * 3)()
    assert L.eq_residual(None, None, norms, None) == 1
    assert L.eq_plan_destroy(None) == 1
    assert L.eq_plan_footprint(ctypes.byref(d), None) == 1
    assert L.eq_plan_set_timing(None, 1) == 1
    assert L.eq_debug_forward(None, None, None) == 1


def test_footprint_matches_layout():
    for (n, b, prec) in [(32, 1, "fp64"), (256, 1, "fp32"), (128, 64, "fp32"), (96, 2, "fp64")]:
        es = 8 if prec == "fp64" else 4
        w = b * 6 * (n // 2 + 1) * n * n * 2 * es
        got = eq.footprint(n, n, n, b, "ddo", prec)
        assert w <= got <= w + b * 1024 * 14 * 8 + b * 14 * 8 + 3 * n * 40 + 256   # tables: 2 symbol sets + 2 twiddle sets
    with pytest.raises(eq.EqError) as ei:
        eq.footprint(30, 31, 30)
    assert ei.value.code == "EQ_ERR_SIZE"


def test_accepted_sizes():
    for n in (4, 6, 8, 10, 12, 30, 32, 96, 160, 192, 384, 512, 640, 720, 1000, 1024):
        assert eq.footprint(n, n, n) > 0


def test_noalloc_residual_refuses_bad_arguments_before_any_device_call():
    """eq_residual_noalloc checks its descriptor, operator, batch limit and pointers on the
    host; none of these paths touches a device."""
    L = eq.lib()
    fake = ctypes.c_void_p(0x10000)

    def status(**kw):
        base = dict(nx=16, ny=16, nz=16, batch=1, op="ddo", prec="fp64", h=1.0, flags=0)
        base.update(kw)
        d = eq._desc(**base)
        return L.eq_residual_noalloc(ctypes.byref(d), None, fake, ctypes.c_void_p(0x20000000), None)

    assert status(op="cdo") == 1                       # EQ_ERR_ARG: DDO only
    assert status(batch=65) == 2                       # EQ_ERR_SIZE: beyond the static scratch
    assert status(nx=14) == 2                          # EQ_ERR_SIZE: 7 is not a factor
    assert status(h=-1.0) == 1
    d = eq._desc(16, 16, 16, 1, "ddo", "fp64", 1.0, 0)
    assert L.eq_residual_noalloc(None, None, fake, fake, None) == 1
    assert L.eq_residual_noalloc(ctypes.byref(d), None, None, fake, None) == 1
    assert L.eq_residual_noalloc(ctypes.byref(d), None, fake, None, None) == 1
    # norms overlapping the field
    assert L.eq_residual_noalloc(ctypes.byref(d), None, fake, ctypes.c_void_p(0x10008), None) == 1
    assert "overlaps" in eq.lib().eq_last_error().decode()
