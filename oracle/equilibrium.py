"""Plain FP64 CPU oracle: the L2-nearest divergence-free symmetric stress field.

TEST INFRASTRUCTURE ONLY -- never imported by the library.  Only the tests,
``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may call it.

What it computes (Zhou, Lebensohn, Reischig, Ludwig, Bhattacharya, "Imposing
equilibrium on measured 3-D stress fields using Hodge decomposition and
FFT-based optimization"):

  S_equil = argmin { ||S - S_exp||_2 : S periodic symmetric, div S = 0 }
                                                  (Section 3.2, problem statement)

following the paper's solution strategy (Section 3.3): take the mean c0
(Section 3.2, c0 = average of S_exp), transform the demeaned field (Section 4,
eqnFFT/eqniFFT pair), solve the biharmonic Euler-Lagrange equation
nabla^4 H = curl S~ curl (eqnELH) per frequency with the gauge mean(H) = 0,
compose S_equil = curl H curl + c0 (eq:sequil), and transform back.  Each
derivative is replaced by its Fourier symbol: the continuous operator CDO
(Section 4.1, eq:cdo) or the central-difference operator DDO (Section 4.2,
eq:diff and its substitution).

Conventions (the paper's DFT formulas are garbled; readings listed here):
  * fields are arrays (6, nz, ny, nx), x fastest, Voigt order
    (11, 22, 33, 23, 13, 12), tensor index 1 = x, 2 = y, 3 = z;
  * forward DFT  F(q) = sum_x f(x) exp(-2 pi i q.x / N) on 0-based integer
    indices, unnormalized; inverse carries 1/(nx ny nz);
  * CDO symbol xi(q) = 2 pi k(q) / (n h), k = q below n/2, q - n above, and 0 at
    the Nyquist index q = n/2 (eq:cdo); higher derivatives are plain products of
    first-derivative symbols (the Nyquist "modification" of Section 4.1 is not
    applied: it would break idempotence of the projection);
  * DDO symbol s(q) = sin(2 pi q / n) / h, exactly 0 at q = 0 and q = n/2;
    each axis uses its own index;
  * biharmonic symbol = (sum_a s_a^2)^2.  For DDO the paper prints a cosine
    expansion (with a misplaced parenthesis); its corrected form is identical
    to (sum_a s_a^2)^2 and is provided as ``ddo_biharmonic_cosine`` for the
    pins, but not used on the main route because it cancels catastrophically
    at low |q|;
  * modes whose symbol vector vanishes (DC and the 7 Nyquist corners) are
    divergence-free under the discrete operator, so the argmin keeps them
    unchanged (the literal composition curl H curl would zero them);
  * the L2 norm of a symmetric-matrix field is Frobenius: off-diagonal Voigt
    components weigh 2.

Parity pins (tests/test_oracle_pins.py): direct O(N^6) DFT, a dense weighted
least-squares argmin built without any Fourier transform (DDO) or from the
closed-form cotangent differentiation matrix (CDO), the paper's printed
25-point stencil, a single-plane-wave closed form, and the invariants
(divergence-free, idempotent, fixed points, symmetric gradients removed,
orthogonality, Parseval, linearity, independence of L and h, mean kept).
"""
from __future__ import annotations

import math
import os
from typing import Tuple

import numpy as np
import scipy.fft as sfft

__all__ = [
    "VOIGT_PAIRS", "FROB_WEIGHT", "levi_civita", "signed_wavenumber", "cdo_symbol",
    "ddo_symbol", "axis_symbol", "ddo_biharmonic_cosine", "dft3", "idft3",
    "voigt_to_matrix", "matrix_to_voigt", "incompatibility", "project_spectrum_literal",
    "project_spectrum_pap", "project", "divergence", "divergence_central_difference",
    "residual_norms", "frobenius_dot", "frobenius_norm", "max_symbol_norm",
    "sym_grad", "sym_grad_central_difference", "removed_potential", "potential_spectrum",
    "embed_in_buffer", "project_embedded",
]

# Voigt component c <-> tensor indices (i, j), 0-based with 0 = x, 1 = y, 2 = z.
VOIGT_PAIRS: Tuple[Tuple[int, int], ...] = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
FROB_WEIGHT = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def _workers() -> int:
    return int(os.environ.get("ORACLE_WORKERS", os.cpu_count() or 1))


def levi_civita() -> np.ndarray:
    """epsilon_ijk (Theorem 2 index form)."""
    e = np.zeros((3, 3, 3))
    for (i, j, k) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        e[i, j, k] = 1.0
        e[i, k, j] = -1.0
    return e


# ---------------------------------------------------------------- symbols ---

def signed_wavenumber(n: int) -> np.ndarray:
    """Integer wavenumber per 0-based index with the CDO Nyquist rule (Section 4.1, eq:cdo)."""
    q = np.arange(n)
    k = np.where(2 * q < n, q, q - n).astype(np.float64)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def cdo_symbol(n: int, h: float) -> np.ndarray:
    """xi(q) = 2 pi k(q) / L with L = n h (Section 4.1, eq:cdo)."""
    return 2.0 * math.pi * signed_wavenumber(n) / (n * h)


def ddo_symbol(n: int, h: float) -> np.ndarray:
    """Central-difference symbol sin(2 pi q / n) / h (Section 4.2, eq:diff substitution).

    sin(pi) is not 0 in floating point; the exact zeros at q = 0 and q = n/2 are
    imposed so the harmonic modes are recognised exactly."""
    q = np.arange(n)
    s = np.sin(2.0 * math.pi * q / n) / h
    s[(2 * q) % n == 0] = 0.0
    return s


def axis_symbol(op: str, n: int, h: float) -> np.ndarray:
    if op == "cdo":
        return cdo_symbol(n, h)
    if op == "ddo":
        return ddo_symbol(n, h)
    raise ValueError(f"unknown operator {op!r}")


def ddo_biharmonic_cosine(qx, qy, qz, nx: int, ny: int, nz: int, h: float):
    """The paper's Fourier symbol of the 25-point biharmonic stencil (Section 4.2),
    with the misplaced parenthesis corrected so all three cos(4 pi q / n) terms
    carry the factor -24, and the factor 1/(16 h^4) applied."""
    c4 = [np.cos(4.0 * math.pi * np.asarray(q, dtype=np.float64) / n)
          for q, n in ((qx, nx), (qy, ny), (qz, nz))]
    c8 = [np.cos(8.0 * math.pi * np.asarray(q, dtype=np.float64) / n)
          for q, n in ((qx, nx), (qy, ny), (qz, nz))]
    val = (42.0 - 24.0 * (c4[0] + c4[1] + c4[2]) + 2.0 * (c8[0] + c8[1] + c8[2])
           + 8.0 * (c4[0] * c4[1] + c4[1] * c4[2] + c4[0] * c4[2]))
    return val / (16.0 * h ** 4)


def max_symbol_norm(op: str, shape, h: float) -> float:
    """max over the grid of |s(q)| (the symbol is separable per axis)."""
    return float(math.sqrt(sum(float(np.max(axis_symbol(op, n, h) ** 2)) for n in shape)))


# ---------------------------------------------------------------- DFT -------

def dft3(f: np.ndarray) -> np.ndarray:
    """Forward DFT over the last three axes, unnormalized, exponent -2 pi i q.x / N
    (Section 4, the analysis formula), Hermitian half along x."""
    return sfft.rfftn(f, axes=(-3, -2, -1), workers=_workers())


def idft3(F: np.ndarray, shape) -> np.ndarray:
    """Inverse of ``dft3`` with the 1/(nx ny nz) factor (synthesis formula, Section 4)."""
    return sfft.irfftn(F, s=tuple(shape), axes=(-3, -2, -1), workers=_workers())


# ---------------------------------------------------- tensor helpers --------

def voigt_to_matrix(V: np.ndarray) -> np.ndarray:
    """(6, ...) Voigt -> (3, 3, ...) symmetric matrix."""
    M = np.empty((3, 3) + V.shape[1:], dtype=V.dtype)
    for c, (i, j) in enumerate(VOIGT_PAIRS):
        M[i, j] = V[c]
        M[j, i] = V[c]
    return M


def matrix_to_voigt(M: np.ndarray) -> np.ndarray:
    return np.stack([M[i, j] for (i, j) in VOIGT_PAIRS])


def incompatibility(A: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Inc(A)_kn = eps_ijk eps_lmn s_i s_l A_jm (Theorem 2 index form, each
    nabla replaced by a real symbol vector s; the factors i*i = -1 of the two
    derivatives are applied by the caller).  A: (3, 3, ...), s: (3, ...)."""
    eps = levi_civita()
    C = np.einsum("ijk,i...->kj...", eps, s)          # C_kj = eps_ijk s_i
    return np.einsum("kj...,jm...,nm...->kn...", C, A, C)


# ------------------------------------------- per-frequency projection -------

def project_spectrum_literal(A: np.ndarray, s: np.ndarray) -> np.ndarray:
    """The paper's route per frequency: RHS = symbol of curl S~ curl, H = RHS / |s|^4
    (eqnELH, gauge mean(H) = 0 where the symbol vanishes), S_eq = symbol of curl H curl
    (eq:sequil).  Zero-symbol modes are kept (they satisfy div = 0 exactly).

    A: (3, 3, ...) complex spectrum of the demeaned field; s: (3, ...) real symbols."""
    ss = np.sum(s * s, axis=0)
    denom = ss * ss                                   # biharmonic symbol (sum s_a^2)^2
    rhs = -incompatibility(A, s)                      # (i s_i)(i s_l) = -s_i s_l
    live = denom > 0.0
    H = np.where(live, rhs / np.where(live, denom, 1.0), 0.0)
    out = -incompatibility(H, s)
    return np.where(live, out, A)


def project_spectrum_pap(A: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Independent route: P A P with P = I - n n^T, n = s / |s| (n = 0, P = I where s = 0)."""
    ss = np.sum(s * s, axis=0)
    nrm = np.sqrt(ss)
    n = np.where(nrm > 0.0, s / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    eye = np.eye(3).reshape((3, 3) + (1,) * (s.ndim - 1))
    P = eye - n[:, None] * n[None, :]
    PA = np.einsum("ij...,jk...->ik...", P, A)
    return np.einsum("ij...,jk...->ik...", PA, P)


def _grid_symbols(op: str, shape, h: float, z0: int, z1: int):
    nz, ny, nx = shape
    sx = axis_symbol(op, nx, h)[: nx // 2 + 1]
    sy = axis_symbol(op, ny, h)
    sz = axis_symbol(op, nz, h)[z0:z1]
    return np.stack(np.broadcast_arrays(sx[None, None, :], sy[None, :, None], sz[:, None, None]))


def project(S: np.ndarray, op: str = "ddo", h: float = 1.0, route: str = "literal",
            chunk_planes: int = 8):
    """Equilibrate one field (6, nz, ny, nx) or a batch (B, 6, nz, ny, nx).

    Returns (S_equil, removed) with removed = S_exp - S_equil (the symmetrized
    gradient part of Section 3.2).  Computation in FP64."""
    S = np.asarray(S, dtype=np.float64)
    if S.ndim == 5:
        pairs = [project(f, op, h, route, chunk_planes) for f in S]
        return np.stack([p[0] for p in pairs]), np.stack([p[1] for p in pairs])
    if S.ndim != 4 or S.shape[0] != 6:
        raise ValueError("expected (6, nz, ny, nx)")
    shape = S.shape[1:]
    c0 = S.mean(axis=(1, 2, 3))                                   # Section 3.2
    F = dft3(S - c0[:, None, None, None])                         # demeaned field
    step = project_spectrum_literal if route == "literal" else project_spectrum_pap
    out = np.empty_like(F)
    for z0 in range(0, shape[0], chunk_planes):
        z1 = min(shape[0], z0 + chunk_planes)
        s = _grid_symbols(op, shape, h, z0, z1)
        out[:, z0:z1] = matrix_to_voigt(step(voigt_to_matrix(F[:, z0:z1]), s))
    out[:, 0, 0, 0] = 0.0                                         # mean handled in real space
    Seq = idft3(out, shape) + c0[:, None, None, None]
    return Seq, S - Seq


# ------------------------------------------------ zero-stress buffer ---------

def embed_in_buffer(S: np.ndarray, box_xy, offset_xy) -> np.ndarray:
    """Place a non-periodic sample (6, nz, ny0, nx0) at (ox, oy) inside a periodic box of
    (nx, ny) voxels laterally, zero stress elsewhere; z keeps its extent, so top and bottom
    are periodically connected (Section 3.3; Section 5.2, experimental sample)."""
    S = np.asarray(S, dtype=np.float64)
    nx, ny = box_xy
    ox, oy = offset_xy
    nz, ny0, nx0 = S.shape[1:]
    if ox < 0 or oy < 0 or ox + nx0 > nx or oy + ny0 > ny:
        raise ValueError("sample does not fit the box")
    B = np.zeros((6, nz, ny, nx))
    B[:, :, oy:oy + ny0, ox:ox + nx0] = S
    return B


def project_embedded(S: np.ndarray, box_xy, offset_xy, op: str = "ddo", h: float = 1.0):
    """Equilibrate the buffered box and return (S_equil, removed) on the sample's voxels."""
    S = np.asarray(S, dtype=np.float64)
    nz, ny0, nx0 = S.shape[1:]
    ox, oy = offset_xy
    Seq, _ = project(embed_in_buffer(S, box_xy, offset_xy), op, h)
    Seq = Seq[:, :, oy:oy + ny0, ox:ox + nx0]
    return Seq, S - Seq


# ------------------------------------------------------- divergence ---------

def divergence(S: np.ndarray, op: str, h: float = 1.0) -> np.ndarray:
    """r_i = sum_j D_j S_ij with the operator's symbol (Section 4.1 / 4.2); (3, nz, ny, nx)."""
    S = np.asarray(S, dtype=np.float64)
    shape = S.shape[1:]
    F = dft3(S)
    s = _grid_symbols(op, shape, h, 0, shape[0])
    M = voigt_to_matrix(F)
    R = np.stack([sum(1j * s[j] * M[i, j] for j in range(3)) for i in range(3)])
    return idft3(R, shape)


def divergence_central_difference(S: np.ndarray, h: float = 1.0) -> np.ndarray:
    """Real-space periodic central differences (f(x+e) - f(x-e)) / (2h) (Section 4.2, eq:diff)."""
    S = np.asarray(S, dtype=np.float64)
    M = voigt_to_matrix(S)
    axis_of = {0: 2, 1: 1, 2: 0}                  # tensor index x, y, z -> array axis of (nz, ny, nx)

    def d(f, j):
        a = axis_of[j]
        return (np.roll(f, -1, axis=a) - np.roll(f, 1, axis=a)) / (2.0 * h)

    return np.stack([sum(d(M[i, j], j) for j in range(3)) for i in range(3)])


# ------------------------------------------ potential of the removed part ---

def sym_grad(y: np.ndarray, op: str, h: float = 1.0) -> np.ndarray:
    """(grad y + grad y^T) / 2 of a periodic vector field y (3, nz, ny, nx) as a Voigt
    field, each derivative by the operator's symbol (Section 4.1 / 4.2)."""
    y = np.asarray(y, dtype=np.float64)
    shape = y.shape[1:]
    F = dft3(y)
    s = _grid_symbols(op, shape, h, 0, shape[0])
    G = np.empty((3, 3) + F.shape[1:], dtype=complex)
    for i in range(3):
        for j in range(3):
            G[i, j] = 0.5j * (s[j] * F[i] + s[i] * F[j])
    return idft3(matrix_to_voigt(G), shape)


def sym_grad_central_difference(y: np.ndarray, h: float = 1.0) -> np.ndarray:
    """Real-space periodic central differences (Section 4.2, eq:diff) of y, symmetrized."""
    y = np.asarray(y, dtype=np.float64)
    axis_of = {0: 2, 1: 1, 2: 0}

    def d(f, j):
        a = axis_of[j]
        return (np.roll(f, -1, axis=a) - np.roll(f, 1, axis=a)) / (2.0 * h)

    return np.stack([0.5 * (d(y[i], j) + d(y[j], i)) for (i, j) in VOIGT_PAIRS])


def removed_potential(S: np.ndarray, op: str = "ddo", h: float = 1.0) -> np.ndarray:
    """The field y of the decomposition S_exp = S_equil + (grad y + grad y^T)/2 (Section 3.2):
    the least-squares preimage of the removed part under the symmetric gradient, with zero
    mean.  Per frequency with a nonzero symbol s the normal equations of
    min_y sum_ij |R_ij - (i/2)(y_i s_j + s_i y_j)|^2 are (1/2)(|s|^2 I + s s^T) y = -i R s,
    with R the removed part's spectrum; y = 0 where s = 0.  Returns (3, nz, ny, nx)."""
    S = np.asarray(S, dtype=np.float64)
    shape = S.shape[1:]
    _, removed = project(S, op, h)
    R = voigt_to_matrix(dft3(removed))
    s = _grid_symbols(op, shape, h, 0, shape[0])
    return idft3(potential_spectrum(R, s), shape)


def potential_spectrum(R: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Per frequency: solve (1/2)(|s|^2 I + s s^T) y = -i R s where |s| > 0, else y = 0.
    R: (3, 3, ...) symmetric spectra; s: (3, ...) symbols.  Returns (3, ...)."""
    rhs = -1j * np.einsum("ij...,j...->i...", R, s)
    ss = np.sum(s * s, axis=0)
    eye = np.eye(3).reshape((3, 3) + (1,) * ss.ndim)
    N = 0.5 * (ss[None, None] * eye + s[:, None] * s[None, :])
    Y = np.zeros_like(rhs)
    m = ss > 0
    Nm = np.moveaxis(N[:, :, m], -1, 0)                    # (k, 3, 3)
    bm = np.moveaxis(rhs[:, m], -1, 0)[..., None]          # (k, 3, 1)
    Y[:, m] = np.moveaxis(np.linalg.solve(Nm.astype(complex), bm)[..., 0], 0, -1)
    return Y


def frobenius_dot(A: np.ndarray, B: np.ndarray) -> float:
    """<A, B> = sum_x sum_ij A_ij B_ij for Voigt arrays (off-diagonals weigh 2)."""
    w = FROB_WEIGHT.reshape((6,) + (1,) * (A.ndim - 1))
    return float(np.sum(w * A * B))


def frobenius_norm(A: np.ndarray) -> float:
    return math.sqrt(max(frobenius_dot(A, A), 0.0))


def residual_norms(S: np.ndarray, op: str, h: float = 1.0):
    """(l2, max, rel) of the divergence of one field (Section 5, divergence maps):
    l2 = sqrt(sum_x |r(x)|^2), max = max_x |r(x)|, rel = l2 / (max_q |s(q)| ||S - c0||_F)."""
    S = np.asarray(S, dtype=np.float64)
    r = divergence_central_difference(S, h) if op == "ddo" else divergence(S, op, h)
    mag2 = np.sum(r * r, axis=0)
    l2 = math.sqrt(float(np.sum(mag2)))
    mx = math.sqrt(float(np.max(mag2)))
    c0 = S.mean(axis=(1, 2, 3))
    denom = max_symbol_norm(op, S.shape[1:], h) * frobenius_norm(S - c0[:, None, None, None])
    rel = l2 / denom if denom > 0 else 0.0
    return l2, mx, rel
