"""paper_2105_01612_amd -- equilibrium projection of voxelized stress fields on MI355X.

Thin ctypes binding over libeq.so (include/eq.h).  Every step of the projection
runs in the library's HIP kernels; this module only marshals arguments (device
pointers of torch tensors, the stream handle) and turns status codes into
exceptions.  If libeq.so is missing the import of the binding fails loudly:
there is no CPU fallback.

    import torch, paper_2105_01612_amd as eq
    plan = eq.plan(256, 256, 256, op="ddo", prec="fp32")
    s_eq = torch.empty_like(s_in); removed = torch.empty_like(s_in)
    plan.project(s_in, s_eq, removed)          # stream-ordered on the current stream
    l2, mx, rel = plan.residual(s_eq)[0]
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Tuple

__all__ = ["EqError", "Plan", "plan", "footprint", "lib", "library_path", "OP", "PREC", "FLAGS",
           "STATUS", "version", "exported_symbols", "residual_noalloc"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libeq.so")

OP = {"cdo": 0, "ddo": 1}
PREC = {"fp64": 0, "fp32": 1}
FLAGS = {"check_finite": 1, "capture_graph": 2, "persistent": 4, "own_stream": 8}
STATUS = {0: "EQ_OK", 1: "EQ_ERR_ARG", 2: "EQ_ERR_SIZE", 3: "EQ_ERR_NOMEM", 4: "EQ_ERR_DEVICE",
          5: "EQ_ERR_NONFINITE"}

# Entry points declared in include/eq.h.
exported_symbols = (
    "eq_plan", "eq_project", "eq_residual", "eq_plan_destroy", "eq_plan_footprint", "eq_status_str",
    "eq_last_error", "eq_plan_set_stream", "eq_plan_set_timing", "eq_plan_pass_stats",
    "eq_plan_reset_stats", "eq_debug_forward", "eq_debug_project_spectrum", "eq_version", "eq_plan_tune",
    "eq_plan_get_tune", "eq_potential", "eq_project_embedded", "eq_plan_set_timing_pass", "eq_residual_noalloc",
)


class EqDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("batch", ctypes.c_int),
                ("op", ctypes.c_int), ("prec", ctypes.c_int), ("h", ctypes.c_double), ("flags", ctypes.c_uint)]


class EqTune(ctypes.Structure):
    _fields_ = [("tx_y", ctypes.c_int), ("tx_z", ctypes.c_int), ("rw_x", ctypes.c_int), ("chunk", ctypes.c_int),
                ("radix16", ctypes.c_int), ("schedule", ctypes.c_int), ("tc_zp", ctypes.c_int),
                ("radix4", ctypes.c_int), ("xsplit", ctypes.c_int), ("zp_e", ctypes.c_int)]


class EqEmbed(ctypes.Structure):
    _fields_ = [("nx0", ctypes.c_int), ("ny0", ctypes.c_int), ("ox", ctypes.c_int), ("oy", ctypes.c_int)]


class EqError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        self.code = STATUS.get(status, f"EQ_ERR_{status}")
        super().__init__(f"{where}: {self.code}: {msg}")


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libeq.so (built by paper_2105_01612_amd.build); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise ImportError(f"libeq.so not built at {library_path}; run `python -m paper_2105_01612_amd.build`")
    L = ctypes.CDLL(library_path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.eq_plan.argtypes = [ctypes.POINTER(EqDesc), vp, ctypes.POINTER(vp)]
    L.eq_project.argtypes = [vp, vp, vp, vp]
    L.eq_residual.argtypes = [vp, vp, dp, vp]
    L.eq_potential.argtypes = [vp, vp, vp]
    L.eq_residual_noalloc.argtypes = [ctypes.POINTER(EqDesc), vp, vp, vp, vp]
    L.eq_project_embedded.argtypes = [vp, ctypes.POINTER(EqEmbed), vp, vp, vp]
    L.eq_plan_destroy.argtypes = [vp]
    L.eq_plan_footprint.argtypes = [ctypes.POINTER(EqDesc), ctypes.POINTER(ctypes.c_size_t)]
    L.eq_status_str.argtypes = [ip]
    L.eq_status_str.restype = ctypes.c_char_p
    L.eq_last_error.argtypes = []
    L.eq_last_error.restype = ctypes.c_char_p
    L.eq_version.argtypes = []
    L.eq_version.restype = ctypes.c_char_p
    L.eq_plan_set_stream.argtypes = [vp, vp]
    L.eq_plan_set_timing.argtypes = [vp, ip]
    L.eq_plan_reset_stats.argtypes = [vp]
    L.eq_plan_set_timing_pass.argtypes = [vp, ctypes.c_char_p]
    L.eq_plan_pass_stats.argtypes = [vp, ip, ctypes.POINTER(ip), ctypes.POINTER(ctypes.c_char_p),
                                     ctypes.POINTER(ctypes.c_longlong), dp, dp]
    L.eq_debug_forward.argtypes = [vp, vp, vp]
    L.eq_plan_tune.argtypes = [vp, ctypes.POINTER(EqTune)]
    L.eq_plan_get_tune.argtypes = [vp, ctypes.POINTER(EqTune)]
    L.eq_debug_project_spectrum.argtypes = [vp, vp]
    for name in exported_symbols:
        if name not in ("eq_status_str", "eq_last_error", "eq_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def version() -> str:
    return lib().eq_version().decode()


def _check(status: int, where: str):
    if status != 0:
        raise EqError(status, where, lib().eq_last_error().decode(errors="replace"))


def _desc(nx, ny, nz, batch, op, prec, h, flags) -> EqDesc:
    opv = OP[op] if isinstance(op, str) else int(op)
    pv = PREC[prec] if isinstance(prec, str) else int(prec)
    fv = 0
    if isinstance(flags, (list, tuple, set)):
        for f in flags:
            fv |= FLAGS[f]
    else:
        fv = int(flags)
    return EqDesc(int(nx), int(ny), int(nz), int(batch), opv, pv, float(h), fv)


def footprint(nx, ny, nz, batch=1, op="ddo", prec="fp64", h=1.0, flags=0) -> int:
    """Device bytes a plan would allocate (host-only; no device call)."""
    out = ctypes.c_size_t(0)
    _check(lib().eq_plan_footprint(ctypes.byref(_desc(nx, ny, nz, batch, op, prec, h, flags)), ctypes.byref(out)),
           "eq_plan_footprint")
    return int(out.value)


def _ptr(t, name: str, plan: "Plan", shape) -> int:
    """Device pointer of a torch tensor after checking it matches the plan."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    import torch

    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != plan.dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, plan expects {plan.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape) and t.numel() != _numel(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, plan expects {tuple(shape)}")
    return t.data_ptr()


def _numel(shape):
    n = 1
    for s in shape:
        n *= s
    return n


def _stream_handle(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """A libeq plan (eq_plan ... eq_plan_destroy)."""

    def __init__(self, nx, ny, nz, batch=1, op="ddo", prec="fp64", h=1.0, flags=0, stream="current"):
        self.nx, self.ny, self.nz, self.batch = int(nx), int(ny), int(nz), int(batch)
        self.op = op
        self.prec = prec
        self.h = float(h)
        self._d = _desc(nx, ny, nz, batch, op, prec, h, flags)
        import torch

        self.dtype = torch.float64 if self._d.prec == 0 else torch.float32
        if stream is None:
            self._d.flags |= FLAGS["own_stream"]
            handle = 0
        else:
            handle = _stream_handle(None if isinstance(stream, str) and stream == "current" else stream)
        self._h = ctypes.c_void_p()
        _check(lib().eq_plan(ctypes.byref(self._d), ctypes.c_void_p(handle) if handle else None,
                             ctypes.byref(self._h)), "eq_plan")

    # shapes
    @property
    def field_shape(self):
        return (self.batch, 6, self.nz, self.ny, self.nx)

    @property
    def spectrum_shape(self):
        """(batch, 6, nz/2+1, ny, nx, 2): the half spectrum along z as (re, im)."""
        return (self.batch, 6, self.nz // 2 + 1, self.ny, self.nx, 2)

    def _shape_of(self, t):
        if t is not None and not isinstance(t, int) and t.dim() == 4 and self.batch == 1:
            return (6, self.nz, self.ny, self.nx)
        return self.field_shape

    def project(self, s_in, s_eq=None, s_removed=None):
        """eq_project; returns s_eq (allocated like s_in when omitted)."""
        if s_eq is None:
            import torch

            s_eq = torch.empty_like(s_in)
        shape = self._shape_of(s_in)
        _check(lib().eq_project(self._h, _ptr(s_in, "s_in", self, shape), _ptr(s_eq, "s_eq", self, shape),
                                _ptr(s_removed, "s_removed", self, shape) or None), "eq_project")
        return s_eq

    def residual(self, s, div_out=None) -> List[Tuple[float, float, float]]:
        """eq_residual; returns [(l2, max, rel)] per field (blocks)."""
        norms = (ctypes.c_double * (3 * self.batch))()
        shape = self._shape_of(s)
        dshape = (self.batch, 3, self.nz, self.ny, self.nx)
        _check(lib().eq_residual(self._h, _ptr(s, "s", self, shape), norms,
                                 _ptr(div_out, "div_out", self, dshape) or None), "eq_residual")
        return [(norms[3 * b], norms[3 * b + 1], norms[3 * b + 2]) for b in range(self.batch)]

    def project_embedded(self, s_in, nx0, ny0, ox, oy, s_eq=None, s_removed=None):
        """eq_project_embedded: s_in (batch, 6, nz, ny0, nx0) sits at (ox, oy) in this plan's
        (nx, ny) box with zero stress around it; returns s_eq of the sample's shape."""
        if s_eq is None:
            import torch

            s_eq = torch.empty_like(s_in)
        shape = (self.batch, 6, self.nz, int(ny0), int(nx0))
        if s_in.dim() == 4:
            shape = shape[1:]
        e = EqEmbed(int(nx0), int(ny0), int(ox), int(oy))
        _check(lib().eq_project_embedded(self._h, ctypes.byref(e), _ptr(s_in, "s_in", self, shape),
                                         _ptr(s_eq, "s_eq", self, shape),
                                         _ptr(s_removed, "s_removed", self, shape) or None), "eq_project_embedded")
        return s_eq

    def potential(self, s_in, y_out=None):
        """eq_potential: the potential y of the removed part (its symmetric gradient is
        s_in - project(s_in)); returns y_out, shape (batch, 3, nz, ny, nx), allocated when omitted."""
        shape = self._shape_of(s_in)
        yshape = (self.batch, 3, self.nz, self.ny, self.nx)
        if y_out is None:
            import torch

            y_out = torch.empty(yshape if s_in.dim() == 5 else yshape[1:], dtype=s_in.dtype, device=s_in.device)
        _check(lib().eq_potential(self._h, _ptr(s_in, "s_in", self, shape), _ptr(y_out, "y_out", self, yshape)),
               "eq_potential")
        return y_out

    def set_stream(self, stream=None):
        """Rebind to `stream` (a torch stream or raw handle; None = torch's current stream)."""
        handle = _stream_handle(stream)
        _check(lib().eq_plan_set_stream(self._h, ctypes.c_void_p(handle) if handle else None), "eq_plan_set_stream")

    def tune(self, tx_y=0, tx_z=0, rw_x=0, chunk=0, radix16=-1, schedule=0, tc_zp=0, radix4=0, xsplit=0, zp_e=0):
        """eq_plan_tune: set launch shapes / radix schedule / pass schedule (0 or -1 = default);
        raises EqError if they do not fit this grid."""
        t = EqTune(int(tx_y), int(tx_z), int(rw_x), int(chunk), int(radix16), int(schedule), int(tc_zp), int(radix4),
                   int(xsplit), int(zp_e))
        _check(lib().eq_plan_tune(self._h, ctypes.byref(t)), "eq_plan_tune")

    def get_tune(self):
        t = EqTune()
        _check(lib().eq_plan_get_tune(self._h, ctypes.byref(t)), "eq_plan_get_tune")
        return {"tx_y": t.tx_y, "tx_z": t.tx_z, "rw_x": t.rw_x, "chunk": t.chunk, "radix16": t.radix16,
                "schedule": t.schedule, "tc_zp": t.tc_zp, "radix4": t.radix4, "xsplit": t.xsplit, "zp_e": t.zp_e}

    def set_timing(self, enable: bool, only: str = None):
        """eq_plan_set_timing; `only` names the one pass to bracket with events (None: all)."""
        _check(lib().eq_plan_set_timing_pass(self._h, (only or "").encode()), "eq_plan_set_timing_pass")
        _check(lib().eq_plan_set_timing(self._h, 1 if enable else 0), "eq_plan_set_timing")

    def reset_stats(self):
        _check(lib().eq_plan_reset_stats(self._h), "eq_plan_reset_stats")

    def pass_stats(self) -> Dict[str, dict]:
        n = 32
        count = ctypes.c_int(0)
        names = (ctypes.c_char_p * n)()
        launches = (ctypes.c_longlong * n)()
        ms = (ctypes.c_double * n)()
        by = (ctypes.c_double * n)()
        _check(lib().eq_plan_pass_stats(self._h, n, ctypes.byref(count), names, launches, ms, by),
               "eq_plan_pass_stats")
        out = {}
        for i in range(min(count.value, n)):
            out[names[i].decode()] = {"launches": int(launches[i]), "total_ms": float(ms[i]),
                                      "bytes_per_launch": float(by[i])}
        return out

    def debug_forward(self, s_in, spec_out):
        _check(lib().eq_debug_forward(self._h, _ptr(s_in, "s_in", self, self._shape_of(s_in)),
                                      spec_out.data_ptr()), "eq_debug_forward")
        return spec_out

    def debug_project_spectrum(self, spec):
        _check(lib().eq_debug_project_spectrum(self._h, spec.data_ptr()), "eq_debug_project_spectrum")
        return spec

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().eq_plan_destroy(self._h), "eq_plan_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def residual_noalloc(s, norms_dev, nx, ny=None, nz=None, batch=1, prec="fp64", h=1.0, div_out=None, stream=None):
    """eq_residual_noalloc: the DDO residual of `s` without any allocation (no plan); the norms
    (l2, max, rel) per field go to the device tensor `norms_dev` (batch, 3) of float64,
    asynchronously on `stream` (None: torch's current stream)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    d = _desc(nx, ny, nz, batch, "ddo", prec, h, 0)
    import torch

    dt = torch.float64 if d.prec == 0 else torch.float32
    for t, name in ((s, "s"), (div_out, "div_out")):
        if t is not None and (not t.is_cuda or t.dtype != dt or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous device tensor of {dt}")
    if s.numel() != batch * 6 * nx * ny * nz:
        raise ValueError("s does not hold batch * 6 * nz * ny * nx elements")
    if div_out is not None and div_out.numel() != batch * 3 * nx * ny * nz:
        raise ValueError("div_out does not hold batch * 3 * nz * ny * nx elements")
    if (not norms_dev.is_cuda or norms_dev.dtype != torch.float64 or not norms_dev.is_contiguous()
            or norms_dev.numel() < 3 * batch):
        raise ValueError("norms_dev must be a contiguous float64 device tensor of batch * 3 elements")
    handle = _stream_handle(stream)
    _check(lib().eq_residual_noalloc(ctypes.byref(d), ctypes.c_void_p(handle) if handle else None, s.data_ptr(),
                                     norms_dev.data_ptr(), div_out.data_ptr() if div_out is not None else None),
           "eq_residual_noalloc")
    return norms_dev


def plan(nx, ny=None, nz=None, batch=1, op="ddo", prec="fp64", h=1.0, flags=0, stream="current") -> Plan:
    """eq_plan.  ny, nz default to nx.  stream: "current" (torch's current stream at
    creation), None (a plan-owned stream), a torch.cuda.Stream or a raw hipStream_t handle."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Plan(nx, ny, nz, batch, op, prec, h, flags, stream)
