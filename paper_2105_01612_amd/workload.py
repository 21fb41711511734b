"""Seeded synthetic stress-field generator.

This module only produces inputs: periodic Voronoi polycrystals with a
piecewise-constant (optionally piecewise-linear) symmetric stress per grain
plus voxel noise, the kind of field the paper filters (Section 5.1: a periodic
Voronoi unit cell of Cu grains whose grain-averaged stress is piecewise
constant and discontinuous across grain boundaries; Section 5.2: a 256^3 field
of a measured polycrystal).  It contains none of the projection arithmetic, so
both the GPU library and the FP64 checker may consume its arrays.

Layout of every field: (6, nz, ny, nx), x fastest, components in Voigt order
(11, 22, 33, 23, 13, 12) with tensor index 1 = x, 2 = y, 3 = z.  Units: MPa.

Recipe (all "N(0, s)" are i.i.d. normal with standard deviation s):
  rng  = numpy Generator(PCG64(seed))
  draw order: grain seeds (G, 3) uniform in [0, 1)^3, grain stresses (G, 6),
  grain gradients (G, 6, 3) (only drawn when sigma_grad > 0), voxel noise
  (6, nz, ny, nx).
  grain(x) = nearest seed to the voxel centre ((i + 1/2) / n) under the
  periodic minimum-image metric of the unit cube (ties: lowest seed index).
  sigma_c(x) = stress_c[g] + grad_c[g] . d(x) + noise_c(x), where d(x) is the
  minimum-image displacement from the grain seed, in voxel units.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = ["FieldSpec", "voronoi_field", "CONFIG_SPECS", "config_field", "plane_shape", "grain_labels",
           "grain_average"]


@dataclasses.dataclass(frozen=True)
class FieldSpec:
    shape: Tuple[int, int, int]          # (nz, ny, nx)
    grains: int
    sigma_grain: float                   # MPa, per-grain constant stress
    sigma_noise: float                   # MPa, voxel noise
    sigma_grad: float = 0.0              # MPa per voxel, intragranular gradient
    seed: int = 0


def plane_shape(n: int) -> Tuple[int, int, int]:
    return (n, n, n)


def _grain_map(shape: Sequence[int], seeds: np.ndarray, chunk_planes: int):
    """Nearest-seed index and minimum-image displacement (voxel units) per voxel."""
    from scipy.spatial import cKDTree

    nz, ny, nx = shape
    # scipy's periodic tree wants coordinates in [0, boxsize); seeds are drawn in [0, 1).
    tree = cKDTree(seeds, boxsize=1.0)
    gx = (np.arange(nx) + 0.5) / nx
    gy = (np.arange(ny) + 0.5) / ny
    grain = np.empty((nz, ny, nx), dtype=np.int32)
    disp = np.empty((3, nz, ny, nx), dtype=np.float64)
    for z0 in range(0, nz, chunk_planes):
        z1 = min(nz, z0 + chunk_planes)
        gz = (np.arange(z0, z1) + 0.5) / nz
        Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        _, idx = tree.query(pts, k=1, workers=-1)
        idx = idx.astype(np.int32)
        grain[z0:z1] = idx.reshape(z1 - z0, ny, nx)
        d = pts - seeds[idx]
        d -= np.round(d)                         # minimum image in the unit cube
        d *= np.array([nx, ny, nz], dtype=np.float64)   # to voxel units per axis
        disp[:, z0:z1] = d.T.reshape(3, z1 - z0, ny, nx)
        del Z, Y, X, pts, d
    return grain, disp


def voronoi_field(spec: FieldSpec, dtype=np.float64, chunk_planes: Optional[int] = None) -> np.ndarray:
    """Generate one field of shape (6, nz, ny, nx) following the module recipe."""
    nz, ny, nx = spec.shape
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    seeds = rng.random((spec.grains, 3))
    stress = rng.normal(0.0, spec.sigma_grain, size=(spec.grains, 6))
    grads = rng.normal(0.0, spec.sigma_grad, size=(spec.grains, 6, 3)) if spec.sigma_grad > 0 else None
    if chunk_planes is None:
        chunk_planes = max(1, (1 << 22) // (ny * nx))
    need_disp = grads is not None
    grain, disp = _grain_map(spec.shape, seeds, chunk_planes)
    out = np.empty((6, nz, ny, nx), dtype=dtype)
    for c in range(6):
        f = stress[grain, c]
        if need_disp:
            g = grads[grain, c]                  # (nz, ny, nx, 3) gradient in (x, y, z)
            f = f + g[..., 0] * disp[0] + g[..., 1] * disp[1] + g[..., 2] * disp[2]
        out[c] = f
    del grain, disp
    if spec.sigma_noise > 0:
        for c in range(6):
            out[c] += rng.normal(0.0, spec.sigma_noise, size=(nz, ny, nx)).astype(dtype, copy=False)
    return out


def grain_labels(spec: FieldSpec, chunk_planes: Optional[int] = None) -> np.ndarray:
    """Grain index per voxel (nz, ny, nx) of the field ``voronoi_field(spec)`` (same seeds)."""
    nz, ny, nx = spec.shape
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    seeds = rng.random((spec.grains, 3))
    if chunk_planes is None:
        chunk_planes = max(1, (1 << 22) // (ny * nx))
    grain, _ = _grain_map(spec.shape, seeds, chunk_planes)
    return grain


def grain_average(S: np.ndarray, labels: np.ndarray, grains: int) -> np.ndarray:
    """Replace every voxel of each component by the mean of its grain (Section 5.1: the
    grain-averaged field the filter is applied to).  S: (6, nz, ny, nx)."""
    lab = labels.ravel()
    count = np.bincount(lab, minlength=grains).astype(np.float64)
    out = np.empty_like(S)
    for c in range(6):
        mean = np.bincount(lab, weights=S[c].ravel().astype(np.float64), minlength=grains) / np.maximum(count, 1.0)
        out[c] = mean[labels].astype(S.dtype, copy=False)
    return out


# Workloads: sizes, grain counts and distributions of the paper's two examples
# (a 64^3 / 100-grain periodic Voronoi cell, a 256^3 measured cell) scaled to the
# benchmark cases.  Seeds are fixed so every run sees identical inputs.
CONFIG_SPECS = {
    # 32^3, 20 grains, N(0,100) + N(0,5) noise: the FP64 parity case.
    "small": FieldSpec((32, 32, 32), grains=20, sigma_grain=100.0, sigma_noise=5.0, seed=1),
    # 256^3, 1000 grains, N(0,200) + gradient N(0,2)/voxel + N(0,10) noise: the headline case.
    "headline": FieldSpec((256, 256, 256), grains=1000, sigma_grain=200.0, sigma_noise=10.0,
                          sigma_grad=2.0, seed=2),
    # 512^3, 8000 grains, N(0,300) + N(0,15) noise: the largest single field.
    "largest": FieldSpec((512, 512, 512), grains=8000, sigma_grain=300.0, sigma_noise=15.0, seed=5),
    # 160^3, 2000 grains: grain-boundary-heavy case.
    "gb_heavy": FieldSpec((160, 160, 160), grains=2000, sigma_grain=300.0, sigma_noise=15.0, seed=50),
}


def batched_specs(n: int = 128, fields: int = 64, grains: int = 300, first_seed: int = 300):
    """Independent same-size fields: N(0,100) grains + N(0,5) noise, one seed each."""
    return [FieldSpec((n, n, n), grains=grains, sigma_grain=100.0, sigma_noise=5.0,
                      seed=first_seed + i) for i in range(fields)]


SERVING_SIZES = (64, 96, 128, 192, 256, 384)


def serving_spec(n: int, j: int) -> FieldSpec:
    """Pool field j of size class n: one grain per 16^3 voxels."""
    cls = SERVING_SIZES.index(n)
    grains = max(1, (n * n * n) // (16 ** 3))
    return FieldSpec((n, n, n), grains=grains, sigma_grain=100.0, sigma_noise=5.0,
                     seed=4100 + 100 * cls + j)


def config_field(name: str, dtype=np.float64) -> np.ndarray:
    return voronoi_field(CONFIG_SPECS[name], dtype=dtype)


def random_field(shape, seed: int, scale: float = 1.0, dtype=np.float64) -> np.ndarray:
    """Plain i.i.d. normal field (6, *shape) for small parity cases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (scale * rng.standard_normal((6,) + tuple(shape))).astype(dtype)


def poisson_arrivals(count: int, rate: float, seed: int = 4000) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of `count` requests at `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def request_sizes(count: int, seed: int = 4000, sizes=SERVING_SIZES) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.asarray(sizes)[rng.integers(0, len(sizes), size=count)]


def field_bytes(shape, itemsize: int) -> int:
    return 6 * int(math.prod(shape)) * itemsize
