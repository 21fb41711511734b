"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* P1  direct O(N^6) DFT sums against the oracle's transform pair (Section 4);
* P2  a dense weighted least-squares argmin of the problem of Section 3.2, with the
      divergence built in real space: periodic central differences for DDO
      (Section 4.2, eq:diff), the closed-form cotangent (Fourier) differentiation
      matrix with the Nyquist mode dropped for CDO (Section 4.1, eq:cdo);
* P3  the paper's printed 25-point biharmonic stencil (Section 4.2, golden
      fixture) against the DDO symbol, and the corrected cosine expansion;
* P4  a single plane wave, whose projection is the textbook P A P;
* I1-I9 the invariants the method fixes (Sections 3.2 and 5.1);
* planted mistakes in the oracle that each of these pins must catch.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2105_01612_amd.workload import random_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
W6 = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


# ------------------------------------------------------------- helpers ------

def direct_dft3(f):
    """F(q) = sum_x f(x) exp(-2 pi i q.x / N), written out as one dense sum."""
    nz, ny, nx = f.shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = (np.multiply.outer(Z.ravel(), Z.ravel()) / nz + np.multiply.outer(Y.ravel(), Y.ravel()) / ny
          + np.multiply.outer(X.ravel(), X.ravel()) / nx)
    return (np.exp(-2j * math.pi * ph) @ f.ravel()).reshape(f.shape)


def central_difference_matrix(n, h):
    d = np.zeros((n, n))
    for i in range(n):
        d[i, (i + 1) % n] += 1.0 / (2.0 * h)
        d[i, (i - 1) % n] -= 1.0 / (2.0 * h)
    return d


def cotangent_matrix(n, h):
    """Fourier differentiation matrix on n (even) periodic points of spacing h:
    D_jk = (pi / L) (-1)^(j-k) cot((j-k) pi / n), 0 on the diagonal, L = n h.
    (Textbook closed form; it is the derivative of the trigonometric interpolant
    with the Nyquist coefficient's derivative set to 0.)"""
    assert n % 2 == 0
    L = n * h
    d = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            if j != k:
                d[j, k] = (math.pi / L) * (-1.0) ** (j - k) / math.tan((j - k) * math.pi / n)
    return d


def axis_ops(shape, d1):
    """3-D derivative matrices (tensor index 0=x,1=y,2=z) on (nz, ny, nx), x fastest."""
    nz, ny, nx = shape
    dx, dy, dz = d1(nx), d1(ny), d1(nz)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return [np.kron(Iz, np.kron(Iy, dx)), np.kron(Iz, np.kron(dy, Ix)), np.kron(dz, np.kron(Iy, Ix))]


def divergence_matrix(shape, d1):
    D = axis_ops(shape, d1)
    M = int(np.prod(shape))
    out = np.zeros((3 * M, 6 * M))
    for c, (i, j) in enumerate(O.VOIGT_PAIRS):
        # component c = S_ij = S_ji enters r_i through D_j and r_j through D_i
        out[i * M:(i + 1) * M, c * M:(c + 1) * M] += D[j]
        if i != j:
            out[j * M:(j + 1) * M, c * M:(c + 1) * M] += D[i]
    return out


def brute_force_argmin(S, d1):
    """argmin ||V - S||_F subject to div V = 0, as dense weighted least squares:
    V = S - W^-1 D^T lambda, (D W^-1 D^T) lambda = D S, W = diag(1,1,1,2,2,2)."""
    shape = S.shape[1:]
    D = divergence_matrix(shape, d1)
    w = np.repeat(W6, int(np.prod(shape)))
    v0 = S.ravel()
    DW = D / w[None, :]
    lam = np.linalg.lstsq(DW @ D.T, D @ v0, rcond=None)[0]
    return (v0 - (DW.T @ lam)).reshape(S.shape)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def frob_rel(a, b):
    return O.frobenius_norm(a - b) / O.frobenius_norm(b)


# ------------------------------------------------------------------ P1 -------

@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (5, 5, 5), (4, 6, 8)])
def test_direct_dft(shape):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape)
    F = direct_dft3(f)
    half = shape[2] // 2 + 1
    assert np.max(np.abs(O.dft3(f) - F[..., :half])) <= 1e-13 * np.abs(F).max()
    back = O.idft3(F[..., :half], shape)
    assert np.max(np.abs(back - f)) <= 1e-13 * np.abs(f).max()


# ------------------------------------------------------------------ P2 -------

@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (4, 6, 8)])
@pytest.mark.parametrize("h", [1.0, 0.37])
def test_argmin_ddo(shape, h):
    S = random_field(shape, seed=sum(shape), scale=50.0) + 20.0
    ref = brute_force_argmin(S, lambda n: central_difference_matrix(n, h))
    got, removed = O.project(S, "ddo", h)
    assert rel(got, ref) <= 1e-12
    assert np.max(np.abs(removed - (S - got))) == 0.0


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (4, 6, 8)])
def test_argmin_cdo(shape):
    h = 0.5
    S = random_field(shape, seed=7 + sum(shape), scale=50.0) - 5.0
    ref = brute_force_argmin(S, lambda n: cotangent_matrix(n, h))
    got, _ = O.project(S, "cdo", h)
    assert rel(got, ref) <= 1e-12


def test_argmin_keeps_harmonic_modes():
    """The checkerboard (-1)^(i+j+k) and the mean are divergence-free under both
    discrete operators, so the argmin keeps them exactly."""
    n = 6
    Z, Y, X = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    S = np.stack([(-1.0) ** (X + Y + Z) * (c + 1) + 3.0 * c for c in range(6)])
    for op in ("ddo", "cdo"):
        got, _ = O.project(S, op)
        assert np.max(np.abs(got - S)) <= 1e-12


# ------------------------------------------------------------------ P3 -------

def load_stencil():
    rows = []
    with open(os.path.join(GOLDEN, "biharmonic_stencil_25pt.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                ox, oy, oz, c = line.split()
                rows.append((int(ox), int(oy), int(oz), float(c)))
    return rows


def test_stencil_fixture_is_consistent():
    st = load_stencil()
    assert len(st) == 25
    assert sum(c for *_, c in st) == 0.0               # annihilates constants


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 16)])
def test_stencil_symbol_equals_ddo_biharmonic(shape):
    nz, ny, nx = shape
    h = 0.8
    Q = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sym = np.zeros(shape)
    for ox, oy, oz, c in load_stencil():
        sym += c * np.cos(2 * math.pi * (Q[2] * ox / nx + Q[1] * oy / ny + Q[0] * oz / nz))
    sym /= 16.0 * h ** 4
    s2 = (O.ddo_symbol(nx, h)[Q[2]] ** 2 + O.ddo_symbol(ny, h)[Q[1]] ** 2
          + O.ddo_symbol(nz, h)[Q[0]] ** 2)
    assert np.max(np.abs(sym - s2 ** 2)) <= 1e-13 * 64 / h ** 4
    cosf = O.ddo_biharmonic_cosine(Q[2], Q[1], Q[0], nx, ny, nz, h)
    assert np.max(np.abs(cosf - s2 ** 2)) <= 1e-13 * 64 / h ** 4


def test_stencil_applied_in_real_space():
    """The stencil as a periodic convolution equals multiplication by (sum s^2)^2."""
    shape = (8, 10, 12)
    h = 1.0
    f = np.random.default_rng(5).standard_normal(shape)
    g = np.zeros(shape)
    for ox, oy, oz, c in load_stencil():
        g += c * np.roll(f, shift=(-oz, -oy, -ox), axis=(0, 1, 2))
    g /= 16.0 * h ** 4
    nz, ny, nx = shape
    sx = O.ddo_symbol(nx, h)[: nx // 2 + 1]
    sy = O.ddo_symbol(ny, h)
    sz = O.ddo_symbol(nz, h)
    s2 = sx[None, None, :] ** 2 + sy[None, :, None] ** 2 + sz[:, None, None] ** 2
    g2 = O.idft3(O.dft3(f) * s2 ** 2, shape)
    assert np.max(np.abs(g - g2)) <= 1e-12 * np.abs(g).max()


def test_literal_parenthesis_is_wrong():
    """Read with the parenthesis as printed, (42 - 24 (c_x + c_y) + c_z) + 2 sum c8 + 8 sum cc,
    the expansion is 25/(16 h^4) at q = 0 instead of 0, so it cannot be a biharmonic symbol;
    with -24 applied to all three cosines it vanishes there."""
    c4 = c8 = 1.0                     # every cosine at q = 0
    literal = (42 - 24 * (c4 + c4) + c4) + 2 * (3 * c8) + 8 * (3 * c4 * c4)
    corrected = 42 - 24 * (3 * c4) + 2 * (3 * c8) + 8 * (3 * c4 * c4)
    assert literal == 25 and corrected == 0
    assert O.ddo_biharmonic_cosine(0, 0, 0, 8, 8, 8, 1.0) == 0.0


# ------------------------------------------------------------------ P4 -------

@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("k", [(1, 0, 0), (1, 2, 3), (3, 4, 1), (4, 1, 2)])
def test_plane_wave(op, k):
    n = 8
    h = 1.3
    kx, ky, kz = k
    Z, Y, X = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    wave = np.cos(2 * math.pi * (kx * X + ky * Y + kz * Z) / n)
    rng = np.random.default_rng(sum(k))
    A = rng.standard_normal((3, 3))
    A = A + A.T
    S = np.stack([A[i, j] * wave for (i, j) in O.VOIGT_PAIRS])
    sym = O.axis_symbol(op, n, h)
    s = np.array([sym[kx], sym[ky], sym[kz]])
    if np.dot(s, s) == 0:
        expect = A
    else:
        nvec = s / np.linalg.norm(s)
        P = np.eye(3) - np.outer(nvec, nvec)
        expect = P @ A @ P
    got, _ = O.project(S, op, h)
    want = np.stack([expect[i, j] * wave for (i, j) in O.VOIGT_PAIRS])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.abs(A).max()


def test_plane_wave_nyquist_cdo_is_kept_along_nyquist_axis():
    """CDO: a wave with k_x = N/2 has xi_x = 0, so only the y-part of the symbol acts."""
    n = 8
    Z, Y, X = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    wave = np.cos(2 * math.pi * (4 * X + 1 * Y) / n)
    S = np.stack([wave * (c + 1) for c in range(6)])
    got, _ = O.project(S, "cdo")
    # P = I - e_y e_y^T: every component with a y index vanishes
    for c, (i, j) in enumerate(O.VOIGT_PAIRS):
        want = 0.0 if 1 in (i, j) else 1.0
        assert np.max(np.abs(got[c] - want * S[c])) <= 1e-13


# ------------------------------------------------- per-frequency routes -----

def test_literal_route_equals_pap():
    rng = np.random.default_rng(3)
    m = 500
    A = rng.standard_normal((3, 3, m)) + 1j * rng.standard_normal((3, 3, m))
    A = A + A.transpose(1, 0, 2)
    s = rng.standard_normal((3, m)) * rng.uniform(1e-3, 1e3, size=m)
    lit = O.project_spectrum_literal(A, s)
    pap = O.project_spectrum_pap(A, s)
    assert np.max(np.abs(lit - pap)) <= 1e-13 * np.abs(A).max()


def test_inc_inc_is_s4_pap():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((3, 3))
    A = A + A.T
    s = rng.standard_normal(3)
    nn = s / np.linalg.norm(s)
    P = np.eye(3) - np.outer(nn, nn)
    lhs = O.incompatibility(O.incompatibility(A, s), s)
    assert np.max(np.abs(lhs - np.dot(s, s) ** 2 * P @ A @ P)) <= 1e-12 * np.dot(s, s) ** 2 * 10


# ------------------------------------------------------------ invariants ----

def deriv_ddo(f, j, h):
    axis = {0: 2, 1: 1, 2: 0}[j]
    return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) / (2.0 * h)


def deriv_cdo(f, j, h):
    axis = {0: 2, 1: 1, 2: 0}[j]
    d = cotangent_matrix(f.shape[axis], h)
    return np.moveaxis(np.tensordot(d, np.moveaxis(f, axis, 0), axes=(1, 0)), 0, axis)


DERIV = {"ddo": deriv_ddo, "cdo": deriv_cdo}


@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 10), (16, 16, 16), (12, 12, 12)])
def test_invariants(op, shape):
    h = 0.7
    S = random_field(shape, seed=(17 if op == "ddo" else 29) + sum(shape), scale=100.0) + 40.0
    Seq, removed = O.project(S, op, h)
    c0 = S.mean(axis=(1, 2, 3))
    scale = O.frobenius_norm(S) * O.max_symbol_norm(op, shape, h)
    # I1 divergence-free in the same operator (two independent divergence routes for DDO)
    assert np.abs(O.divergence(Seq, op, h)).max() <= 1e-13 * scale
    if op == "ddo":
        assert np.abs(O.divergence_central_difference(Seq, h)).max() <= 1e-13 * scale
    # I2 idempotent
    again, _ = O.project(Seq, op, h)
    assert frob_rel(again, Seq) <= 1e-13
    # I5 orthogonality in the Frobenius inner product
    dev = Seq - c0[:, None, None, None]
    assert abs(O.frobenius_dot(removed, dev)) <= 1e-12 * O.frobenius_norm(removed) * O.frobenius_norm(dev)
    # I9 mean kept, and the removed part has zero mean
    assert np.max(np.abs(Seq.mean(axis=(1, 2, 3)) - c0)) <= 1e-12 * np.abs(S).max()
    # I7 linearity
    T = random_field(shape, seed=99, scale=30.0)
    a, b = 1.7, -0.4
    lin, _ = O.project(a * S + b * T, op, h)
    pt, _ = O.project(T, op, h)
    assert frob_rel(lin, a * Seq + b * pt) <= 1e-13
    # I8 the projection depends on the direction of the symbol only
    other, _ = O.project(S, op, 3.9 * h)
    assert frob_rel(other, Seq) <= 1e-13


@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_fixed_point_curl_curl(op):
    """I3: S = curl Phi curl of a symmetric trigonometric potential is returned unchanged."""
    shape = (8, 10, 12)
    h = 1.1
    rng = np.random.default_rng(21)
    Z, Y, X = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    Phi = np.zeros((3, 3) + shape)
    for _ in range(4):
        k = [rng.integers(-3, 4) for _ in range(3)]
        amp = rng.standard_normal((3, 3))
        amp = amp + amp.T
        ph = 2 * math.pi * (k[0] * X / shape[2] + k[1] * Y / shape[1] + k[2] * Z / shape[0])
        Phi += amp[:, :, None, None, None] * np.cos(ph + rng.uniform(0, 6.28))
    d = DERIV[op]
    eps = O.levi_civita()
    M = np.zeros((3, 3) + shape)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    for m in range(3):
                        for n in range(3):
                            e = eps[i, j, k] * eps[l, m, n]
                            if e != 0.0:
                                M[k, n] += e * d(d(Phi[j, m], i, h), l, h)
    S = O.matrix_to_voigt(M) + np.array([5.0, -3.0, 1.0, 2.0, 0.5, -1.0])[:, None, None, None]
    got, _ = O.project(S, op, h)
    assert frob_rel(got, S) <= 1e-12


@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_symmetric_gradient_maps_to_mean(op):
    """I4: S = c0 + sym grad a (same discrete gradient) projects to c0 exactly."""
    shape = (8, 8, 6)
    h = 0.9
    rng = np.random.default_rng(4)
    a = rng.standard_normal((3,) + shape) * 10
    d = DERIV[op]
    c0 = np.array([3.0, -1.0, 2.0, 0.3, 0.2, -0.7])
    S = np.stack([0.5 * (d(a[i], j, h) + d(a[j], i, h)) for (i, j) in O.VOIGT_PAIRS])
    S += c0[:, None, None, None]
    got, removed = O.project(S, op, h)
    assert np.max(np.abs(got - c0[:, None, None, None])) <= 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 4), (5, 7, 9)])
def test_parseval(shape):
    """I6: sum_x f^2 = (1/N^3) sum_q w_q |F_q|^2 over the Hermitian half (w = 2 off the
    self-conjugate x-planes)."""
    f = np.random.default_rng(2).standard_normal(shape)
    F = O.dft3(f)
    nx = shape[2]
    w = np.full(F.shape[2], 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    lhs = float(np.sum(f * f))
    rhs = float(np.sum(w * np.abs(F) ** 2)) / f.size
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_odd_grid_only_dc_is_harmonic():
    shape = (5, 7, 9)
    S = random_field(shape, seed=3, scale=10.0)
    for op in ("cdo", "ddo"):
        Seq, _ = O.project(S, op)
        assert np.abs(O.divergence(Seq, op)).max() <= 1e-12 * np.abs(S).max()


def test_residual_norms_definitions():
    shape = (8, 8, 8)
    S = random_field(shape, seed=12, scale=10.0)
    for op in ("cdo", "ddo"):
        l2, mx, rel_ = O.residual_norms(S, op, 1.0)
        r = O.divergence(S, op, 1.0)
        mag = np.sqrt(np.sum(r * r, axis=0))
        assert l2 == pytest.approx(float(np.sqrt(np.sum(mag ** 2))), rel=1e-12)
        assert mx == pytest.approx(float(mag.max()), rel=1e-12)
        assert 0.0 < rel_ < 1.0
        Seq, _ = O.project(S, op, 1.0)
        assert O.residual_norms(Seq, op, 1.0)[2] <= 1e-14


# ------------------------------------------- divergence and its scale ---
# Section 4.1 (eq:cdo) and Section 4.2 (eq:diff): the residual r_i = sum_j D_j S_ij of a
# field that is NOT equilibrated, against divergence operators built without the
# oracle's symbols: the dense cotangent (Fourier) differentiation matrix for CDO and
# periodic central differences (a dense matrix and np.roll) for DDO.

def _matrix_divergence(S, d1):
    shape = S.shape[1:]
    return (divergence_matrix(shape, d1) @ S.ravel()).reshape((3,) + shape)


def _divergence_pins_hold(shapes=((8, 6, 10), (4, 4, 4), (6, 8, 4)), h=0.7):
    """True when oracle.divergence and oracle.residual_norms agree with the matrix
    operators on random, non-equilibrated fields (both operators)."""
    for shape in shapes:
        S = random_field(shape, seed=41 + sum(shape), scale=30.0) + 7.0
        for op, d1 in (("cdo", lambda n: cotangent_matrix(n, h)), ("ddo", lambda n: central_difference_matrix(n, h))):
            ref = _matrix_divergence(S, d1)
            got = O.divergence(S, op, h)
            if not rel(got, ref) <= 1e-12:
                return False
            # the norms: l2, max over voxels of |r|, and rel with the brute-force symbol scale
            mag2 = np.sum(ref * ref, axis=0)
            c0 = S.mean(axis=(1, 2, 3))
            dev = S - c0[:, None, None, None]
            frob = math.sqrt(float(np.sum(W6[:, None, None, None] * dev * dev)))
            want = (math.sqrt(float(np.sum(mag2))), math.sqrt(float(mag2.max())),
                    math.sqrt(float(np.sum(mag2))) / (_brute_symbol_max(op, shape, h) * frob))
            norms = O.residual_norms(S, op, h)
            if not all(abs(g - w) <= 1e-12 * abs(w) for g, w in zip(norms, want)):
                return False
    return True


def _brute_symbol_max(op, shape, h):
    """max over every frequency q of the full grid of |s(q)|, where s(q) is measured by
    applying the operator's real-space derivative matrices (cotangent for CDO, central
    differences for DDO) to the plane wave exp(2 pi i q.x / N): D_j e = i s_j(q) e."""
    d1 = (lambda n: cotangent_matrix(n, h)) if op == "cdo" else (lambda n: central_difference_matrix(n, h))
    nz, ny, nx = shape
    best = 0.0
    per_axis = []
    for n in (nx, ny, nz):
        D = d1(n)
        x = np.arange(n)
        vals = []
        for q in range(n):
            e = np.exp(2j * math.pi * q * x / n)
            vals.append(((D @ e) / (1j * e)).real)          # D e = i s e, pointwise
        per_axis.append(np.array([v[0] for v in vals]))
    for qz in range(nz):
        for qy in range(ny):
            for qx in range(nx):
                s2 = per_axis[0][qx] ** 2 + per_axis[1][qy] ** 2 + per_axis[2][qz] ** 2
                best = max(best, s2)
    return math.sqrt(best)


def test_divergence_on_unequilibrated_fields():
    """oracle.divergence (both branches) and oracle.residual_norms against the matrix
    divergence operators on random fields that are far from equilibrium."""
    assert _divergence_pins_hold()


@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 10), (6, 8, 4), (12, 4, 6)])
@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("h", [1.0, 0.37])
def test_max_symbol_norm_is_the_grid_maximum(op, shape, h):
    """max_symbol_norm (the scale of the residual's rel) equals the maximum of |s(q)| over
    the whole grid, with s measured from the real-space operators on plane waves."""
    assert O.max_symbol_norm(op, shape, h) == pytest.approx(_brute_symbol_max(op, shape, h), rel=1e-12)


def test_ddo_divergence_routes_agree_with_roll():
    """The DDO branch's spectral divergence equals periodic central differences by np.roll
    on a non-equilibrated field (eq:diff is exactly the DDO symbol)."""
    S = random_field((6, 10, 8), seed=3, scale=25.0) - 2.0
    assert rel(O.divergence(S, "ddo", 0.45), O.divergence_central_difference(S, 0.45)) <= 1e-12


# ------------------------------------------- potential of the removed part ---
# Section 3.2: S_exp = S_equil + (grad y + grad y^T)/2.  The oracle's y is a least-squares
# solve per frequency; the pins check it against that definition in real space.

def _sym_grad_of(op, y, h):
    return O.sym_grad_central_difference(y, h) if op == "ddo" else O.sym_grad(y, op, h)


@pytest.mark.parametrize("op", ["cdo", "ddo"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 4), (8, 6, 12)])
def test_potential_symmetric_gradient_is_removed_part(op, shape):
    """sym grad y (DDO: real-space central differences, no transform) equals S - project(S);
    y has zero mean."""
    h = 0.7
    S = random_field(shape, seed=31, scale=40.0) + 10.0
    y = O.removed_potential(S, op, h)
    _, removed = O.project(S, op, h)
    assert rel(_sym_grad_of(op, y, h), removed) <= 1e-12
    assert np.abs(y.mean(axis=(1, 2, 3))).max() <= 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_potential_recovers_a_known_symmetric_gradient(op):
    """S = c0 + sym grad a + (an equilibrated field) gives y = a exactly, for a with zero
    mean and no zero-symbol modes (those are invisible to any symmetric gradient)."""
    shape = (8, 6, 10)
    h = 1.3
    rng = np.random.default_rng(9)
    A = O.dft3(rng.standard_normal((3,) + shape))
    s = np.stack(np.broadcast_arrays(*[O.axis_symbol(op, n, h)[sl] for n, sl in
                                       zip(shape[::-1], (np.s_[None, None, : shape[2] // 2 + 1],
                                                         np.s_[None, :, None], np.s_[:, None, None]))]))
    A = np.where(np.sum(s * s, axis=0) > 0, A, 0.0)
    a = O.idft3(A, shape)
    E, _ = O.project(random_field(shape, seed=10, scale=30.0), op, h)
    S = _sym_grad_of(op, a, h) + E + np.array([2.0, -1.0, 0.5, 0.3, 0.0, 1.0])[:, None, None, None]
    y = O.removed_potential(S, op, h)
    assert rel(y, a) <= 1e-12


# ------------------------------------------------------ zero-stress buffer ---

@pytest.mark.parametrize("op", ["cdo", "ddo"])
def test_buffered_box_is_equilibrated_and_sample_cropped(op):
    """The buffered box's projection is divergence-free over the whole box (the buffer
    included); the embedded result is its restriction to the sample; a sample that fills
    the box is the plain periodic projection."""
    h = 0.8
    S = random_field((8, 5, 7), seed=21, scale=30.0) + 5.0
    box, off = (12, 10), (3, 2)
    B = O.embed_in_buffer(S, box, off)
    assert np.all(B[:, :, :2] == 0) and np.all(B[:, :, :, 10:] == 0) and np.array_equal(B[:, :, 2:7, 3:10], S)
    Beq, _ = O.project(B, op, h)
    r = O.divergence_central_difference(Beq, h) if op == "ddo" else O.divergence(Beq, op, h)
    assert np.abs(r).max() <= 1e-12 * np.abs(B).max()
    got, rem = O.project_embedded(S, box, off, op, h)
    assert np.array_equal(got, Beq[:, :, 2:7, 3:10]) and np.allclose(rem, S - got, rtol=0, atol=1e-12)
    full = random_field((6, 8, 10), seed=22, scale=30.0)
    a, _ = O.project_embedded(full, (10, 8), (0, 0), op, h)
    b, _ = O.project(full, op, h)
    assert np.array_equal(a, b)


# ------------------------------------------------------- planted mistakes ---

def _potential_pin_fails(op="ddo", shape=(6, 8, 4)):
    S = random_field(shape, seed=12, scale=40.0)
    y = O.removed_potential(S, op, 0.8)
    _, removed = O.project(S, op, 0.8)
    return rel(_sym_grad_of(op, y, 0.8), removed) > 1e-6


def test_planted_potential_missing_rank_one_term_is_caught(monkeypatch):
    def mutant(R, s):
        rhs = -1j * np.einsum("ij...,j...->i...", R, s)
        ss = np.sum(s * s, axis=0)
        return np.where(ss > 0, 2.0 * rhs / np.where(ss > 0, ss, 1.0), 0.0)   # (1/2)|s|^2 I only

    monkeypatch.setattr(O.equilibrium, "potential_spectrum", mutant)
    assert _potential_pin_fails("ddo") and _potential_pin_fails("cdo")


def test_planted_potential_conjugate_is_caught(monkeypatch):
    orig = O.equilibrium.potential_spectrum
    monkeypatch.setattr(O.equilibrium, "potential_spectrum", lambda R, s: np.conj(orig(R, s)))
    assert _potential_pin_fails("ddo")


def _argmin_fails(monkeypatch_ctx, op, shape=(4, 6, 8)):
    S = random_field(shape, seed=5, scale=50.0) + 20.0
    d1 = (lambda n: central_difference_matrix(n, 1.0)) if op == "ddo" else (lambda n: cotangent_matrix(n, 1.0))
    ref = brute_force_argmin(S, d1)
    got, _ = O.project(S, op, 1.0)
    return rel(got, ref) > 1e-6


def test_planted_dropped_harmonic_modes_is_caught(monkeypatch):
    orig = O.equilibrium.project_spectrum_literal

    def mutant(A, s):
        out = orig(A, s)
        dead = np.sum(s * s, axis=0) == 0
        return np.where(dead, 0.0, out)

    monkeypatch.setattr(O.equilibrium, "project_spectrum_literal", mutant)
    assert _argmin_fails(monkeypatch, "ddo")


def test_planted_inexact_ddo_nyquist_is_caught(monkeypatch):
    def mutant(n, h):
        q = np.arange(n)
        return np.sin(2.0 * math.pi * q / n) / h

    monkeypatch.setattr(O.equilibrium, "ddo_symbol", mutant)
    assert _argmin_fails(monkeypatch, "ddo")


def test_planted_swapped_axes_is_caught(monkeypatch):
    orig = O.equilibrium._grid_symbols

    def mutant(op, shape, h, z0, z1):
        s = orig(op, shape, h, z0, z1)
        return s[[1, 0, 2]]

    monkeypatch.setattr(O.equilibrium, "_grid_symbols", mutant)
    assert _argmin_fails(monkeypatch, "cdo")


def test_planted_one_sided_offdiagonal_is_caught(monkeypatch):
    def mutant(V):
        M = np.zeros((3, 3) + V.shape[1:], dtype=V.dtype)
        for c, (i, j) in enumerate(O.VOIGT_PAIRS):
            M[i, j] = V[c]
        return M

    monkeypatch.setattr(O.equilibrium, "voigt_to_matrix", mutant)
    assert _argmin_fails(monkeypatch, "ddo")


def test_planted_sign_error_is_caught(monkeypatch):
    orig = O.equilibrium.incompatibility
    calls = {"n": 0}

    def mutant(A, s):
        calls["n"] += 1
        out = orig(A, s)
        return -out if calls["n"] % 2 == 0 else out

    monkeypatch.setattr(O.equilibrium, "incompatibility", mutant)
    assert _argmin_fails(monkeypatch, "ddo")


def test_planted_nyquist_second_derivative_is_caught(monkeypatch):
    """Giving the Nyquist index a nonzero CDO symbol (the even-derivative convention)
    disagrees with the argmin over the Fourier differentiation matrix."""
    def mutant(n):
        q = np.arange(n)
        return np.where(2 * q <= n, q, q - n).astype(np.float64)

    monkeypatch.setattr(O.equilibrium, "signed_wavenumber", mutant)
    assert _argmin_fails(monkeypatch, "cdo")


def _patch_divergence(monkeypatch, fn):
    """Replace the oracle's divergence where it is defined and where it is re-exported."""
    monkeypatch.setattr(O.equilibrium, "divergence", fn)
    monkeypatch.setattr(O, "divergence", fn)


def test_planted_doubled_cdo_divergence_is_caught(monkeypatch):
    orig = O.equilibrium.divergence
    _patch_divergence(monkeypatch, lambda S, op, h=1.0: 2.0 * orig(S, op, h) if op == "cdo" else orig(S, op, h))
    assert not _divergence_pins_hold()


def test_planted_divergence_without_i_is_caught(monkeypatch):
    """The derivative symbol applied without its factor i (a real multiplier)."""
    def mutant(S, op, h=1.0):
        S = np.asarray(S, dtype=np.float64)
        shape = S.shape[1:]
        F = O.dft3(S)
        s = O.equilibrium._grid_symbols(op, shape, h, 0, shape[0])
        M = O.voigt_to_matrix(F)
        R = np.stack([sum(s[j] * M[i, j] for j in range(3)) for i in range(3)])
        return O.idft3(R, shape)

    _patch_divergence(monkeypatch, mutant)
    assert not _divergence_pins_hold()


def test_planted_divergence_transposed_index_is_caught(monkeypatch):
    """r_i = sum_j D_i S_ij (derivative on the wrong index) instead of sum_j D_j S_ij."""
    def mutant(S, op, h=1.0):
        S = np.asarray(S, dtype=np.float64)
        shape = S.shape[1:]
        F = O.dft3(S)
        s = O.equilibrium._grid_symbols(op, shape, h, 0, shape[0])
        M = O.voigt_to_matrix(F)
        R = np.stack([sum(1j * s[i] * M[i, j] for j in range(3)) for i in range(3)])
        return O.idft3(R, shape)

    _patch_divergence(monkeypatch, mutant)
    assert not _divergence_pins_hold()


def test_planted_symbol_scale_is_caught(monkeypatch):
    """max_symbol_norm taken over one axis only (a dropped term) changes rel."""
    def mutant(op, shape, h):
        return float(np.max(np.abs(O.axis_symbol(op, shape[-1], h))))

    monkeypatch.setattr(O.equilibrium, "max_symbol_norm", mutant)
    monkeypatch.setattr(O, "max_symbol_norm", mutant)
    assert not _divergence_pins_hold()
