"""Recovery studies built on the library (not on the hot path).

Grain-averaging recovery (Section 5.1, Table 1 protocol, on synthetic truth): an
equilibrated "ground truth" T is made by projecting a periodic Voronoi field with the
same operator (so div T = 0 exactly in that operator); the measurement model is the
grain average A of T (what a grain-resolved diffraction method would report); the filter
returns R = project(A).  Because T is a fixed point of the projection, R - T = P(A - T):
the filter removes exactly the symmetric-gradient part of the averaging error and keeps
its divergence-free part (Section 5.1, the claim tested with Fig. 3's perturbations), so
||R - T||^2 + ||(A - T) - P(A - T)||^2 = ||A - T||^2 (Frobenius).

All projections run on the GPU through the C ABI; the grain averaging is input
preparation on the host.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

from . import workload as wl

__all__ = ["frobenius", "grain_average_recovery"]

_W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0]).reshape(6, 1, 1, 1)


def frobenius(X: np.ndarray) -> float:
    """Frobenius L2 norm of a Voigt field (off-diagonals weigh 2)."""
    X = X.astype(np.float64, copy=False)
    return math.sqrt(float(np.sum(_W * X * X)))


def _errors(X: np.ndarray, ref: np.ndarray) -> Dict[str, float]:
    d = X.astype(np.float64) - ref.astype(np.float64)
    return {"rel_l2": frobenius(d) / frobenius(ref), "max_abs_mpa": float(np.abs(d).max())}


def grain_average_recovery(spec: wl.FieldSpec, op: str = "ddo", prec: str = "fp64", h: float = 1.0,
                           keep_fields: bool = False) -> dict:
    """Run the protocol on one field; returns errors of A and R against T and of R against A,
    and the Pythagoras check of the decomposition of the averaging error."""
    import torch

    import paper_2105_01612_amd as eq

    nz, ny, nx = spec.shape
    dtype = torch.float64 if prec == "fp64" else torch.float32
    plan = eq.plan(nx, ny, nz, op=op, prec=prec, h=h)
    try:
        S0 = wl.voronoi_field(spec)
        T = plan.project(torch.from_numpy(S0).to("cuda", dtype)).double().cpu().numpy()
        labels = wl.grain_labels(spec)
        A = wl.grain_average(T, labels, spec.grains)
        x = torch.from_numpy(A).to("cuda", dtype)
        rem = torch.empty_like(x)
        R = plan.project(x, None, rem).double().cpu().numpy()
        removed = rem.double().cpu().numpy()
        norms_T = plan.residual(torch.from_numpy(T).to("cuda", dtype))[0]
        norms_A = plan.residual(x)[0]
    finally:
        plan.destroy()
    e_avg, e_rec = frobenius(A - T), frobenius(R - T)
    out = {
        "op": op, "prec": prec, "grid": [nx, ny, nz], "grains": spec.grains,
        "average_vs_truth": _errors(A, T),
        "recovered_vs_truth": _errors(R, T),
        "recovered_vs_average": _errors(R, A),
        "removed_rel": frobenius(removed) / frobenius(T),
        "pythagoras_rel_gap": abs(e_rec ** 2 + frobenius(removed) ** 2 - e_avg ** 2) / e_avg ** 2,
        "residual_rel_truth": norms_T[2],
        "residual_rel_average": norms_A[2],
    }
    if keep_fields:
        out["fields"] = {"T": T, "A": A, "R": R}
    return out
