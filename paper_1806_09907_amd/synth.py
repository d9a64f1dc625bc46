"""Seeded synthetic inputs for the registration workloads.

This module draws random numbers and paints synthetic volumes. It holds none
of the registration method's arithmetic: no B-spline expansion, no warping,
no similarity and no regulariser. Where a workload needs a moving image made
by warping the fixed one, the caller passes the warp in (the CPU oracle in the
tests, the GPU library in the benchmark), so both sides of a parity check see
identical inputs.

Workload recipes (all FP64 painted, rounded to FP32):

* 2D 64x64 blobs: 12 Gaussian blobs, centres U[0, n-1], sigma U(3, 10) px,
  amplitude U(0, 1); moving image warped by a cubic B-spline field with
  spacing 8 and control displacements N(0, 2 px).
* 3D 128^3 blobs: 40 blobs (same ranges) plus N(0, 0.01) iid noise; control
  displacements N(0, 3 voxels), spacing 8.
* 3D 256^3 CT-like: background -1000 HU, 16 random ellipsoids painted in
  order (semi-axes U(8, 80) voxels, random rotation, intensity
  U(-1000, 1000)), Gaussian smoothing sigma 1.5 voxels; the moving image is
  warped by a coarse cubic B-spline field (spacing 32) whose controls are
  rescaled so that max |control| = 6 voxels; by the convex-hull property of
  the non-negative, partition-of-unity basis the field never exceeds that.
* uneven batches: side lengths per axis drawn from {96, 112, 128, 144, 160}.

Control displacements are drawn in voxel units and converted to the
normalised [-1, 1] convention by the factor 2 / (n_a - 1) per axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 1806_09907

# config index -> seed offset block (seed = BASE_SEED + 1000 * k + pair)
def seed_for(config_index: int, pair: int = 0) -> int:
    return BASE_SEED + 1000 * config_index + pair


def heldout_seed(pair: int) -> int:
    return BASE_SEED + 1_000_000 + pair


def training_seed(pair: int) -> int:
    return BASE_SEED + 2_000_000 + pair


def n_control(n: int, spacing: int) -> int:
    """Number of cubic B-spline controls along an axis of n voxels.

    Controls sit at voxel (j - 1) * spacing for j = 0 .. n_c - 1, so that
    every voxel has its four supporting controls inside the grid.
    """
    return (n - 1) // spacing + 4


def blobs(shape_zyx: Sequence[int], nblobs: int, rng: np.random.Generator,
          sigma=(3.0, 10.0), amplitude=(0.0, 1.0)) -> np.ndarray:
    """Sum of isotropic Gaussian blobs, painted separably in FP64."""
    shape = tuple(int(s) for s in shape_zyx)
    d = len(shape)
    out = np.zeros(shape, dtype=np.float64)
    # centres are drawn x-first to be independent of the array axis order
    for _ in range(nblobs):
        c = [rng.uniform(0.0, shape[d - 1 - a] - 1) for a in range(d)]  # x, y, (z)
        s = rng.uniform(*sigma)
        amp = rng.uniform(*amplitude)
        prof = [np.exp(-0.5 * ((np.arange(shape[d - 1 - a]) - c[a]) / s) ** 2)
                for a in range(d)]
        if d == 2:
            out += amp * np.outer(prof[1], prof[0])
        else:
            out += amp * (prof[2][:, None, None] * prof[1][None, :, None]
                          * prof[0][None, None, :])
    return out


def control_field(n_xyz: Sequence[int], spacing: Sequence[int], std_vox: float,
                  rng: np.random.Generator) -> np.ndarray:
    """Random control displacements, N(0, std_vox) voxels, in normalised units.

    Returns an array [d][nc_z][nc_y][nc_x] (2D: [2][nc_y][nc_x]) with
    component order (x, y, z).
    """
    d = len(n_xyz)
    nc = [n_control(n_xyz[a], spacing[a]) for a in range(d)]
    shape = (d,) + tuple(reversed(nc))
    theta = rng.normal(0.0, std_vox, size=shape)
    for a in range(d):
        theta[a] *= 2.0 / (n_xyz[a] - 1)
    return theta


def ellipsoid_volume(n: int, rng: np.random.Generator, count: int = 16,
                     semi=(8.0, 80.0), intensity=(-1000.0, 1000.0),
                     background=-1000.0, smooth_sigma=1.5) -> np.ndarray:
    """CT-like piecewise-constant ellipsoids, smoothed by a Gaussian.

    Each ellipsoid (centre, semi-axes, rotation from a random unit quaternion,
    intensity) is painted over the voxels with Rt (x - c) inside the axes,
    in drawing order; only its bounding box is visited (half extent
    sqrt(sum_j R_ij^2 a_j^2) along world axis i)."""
    from scipy.ndimage import gaussian_filter

    vol = np.full((n, n, n), background, dtype=np.float64)
    for _ in range(count):
        centre = rng.uniform(0.0, n - 1, size=3)
        axes = rng.uniform(*semi, size=3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        rot = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
        value = rng.uniform(*intensity)
        ext = np.sqrt((rot ** 2) @ (axes ** 2))
        lo = np.clip(np.floor(centre - ext).astype(int) - 1, 0, n)
        hi = np.clip(np.ceil(centre + ext).astype(int) + 2, 0, n)
        if np.any(hi <= lo):
            continue
        dz = (np.arange(lo[2], hi[2], dtype=np.float64) - centre[2])[:, None, None]
        dy = (np.arange(lo[1], hi[1], dtype=np.float64) - centre[1])[None, :, None]
        dx = (np.arange(lo[0], hi[0], dtype=np.float64) - centre[0])[None, None, :]
        r = 0.0
        for j in range(3):
            lj = dx * rot[0, j] + dy * rot[1, j] + dz * rot[2, j]
            r = r + (lj / axes[j]) ** 2
        box = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        box[r <= 1.0] = value
    return gaussian_filter(vol, sigma=smooth_sigma, mode="nearest", truncate=4.0)


WarpFn = Callable[[Tuple[int, ...], Tuple[int, ...], np.ndarray, np.ndarray], np.ndarray]
"""warp(n_xyz, spacing_xyz, moving_fp32, theta_fp32) -> warped FP32 array.

theta is a cubic B-spline control grid in normalised units with the given
spacing; the function returns the moving image sampled at x + u(x) with the
library's conventions (trilinear, zero padding)."""


@dataclass
class Pair:
    fixed: np.ndarray        # FP32, [nz][ny][nx] (2D: [ny][nx])
    moving: np.ndarray       # FP32, same shape
    theta_gen: np.ndarray    # FP32 generating control grid (normalised units)
    n_xyz: Tuple[int, ...]
    spacing: Tuple[int, ...]
    seed: int


def blob_pair(n_xyz: Sequence[int], seed: int, warp: WarpFn, nblobs: int,
              disp_std_vox: float, noise_std: float = 0.0,
              spacing: int = 8) -> Pair:
    """Fixed = blobs (+ noise); moving = warp(fixed, random B-spline field)."""
    rng = np.random.default_rng(seed)
    n_xyz = tuple(int(v) for v in n_xyz)
    shape_zyx = tuple(reversed(n_xyz))
    fixed = blobs(shape_zyx, nblobs, rng)
    if noise_std > 0:
        fixed = fixed + rng.normal(0.0, noise_std, size=fixed.shape)
    fixed32 = fixed.astype(np.float32)
    sp = tuple([spacing] * len(n_xyz))
    theta = control_field(n_xyz, sp, disp_std_vox, rng).astype(np.float32)
    moving = np.ascontiguousarray(warp(n_xyz, sp, fixed32, theta), dtype=np.float32)
    return Pair(fixed32, moving, theta, n_xyz, sp, seed)


def pair_2d(seed: Optional[int] = None, warp: WarpFn = None, n: int = 64) -> Pair:
    """2D blobs: 12 blobs, displacement N(0, 2 px), spacing 8."""
    return blob_pair((n, n), seed_for(0) if seed is None else seed, warp,
                     nblobs=12, disp_std_vox=2.0)


def pair_3d(seed: Optional[int] = None, warp: WarpFn = None,
            n_xyz=(128, 128, 128)) -> Pair:
    """3D blobs: 40 blobs + N(0, 0.01) noise, displacement N(0, 3 vox)."""
    return blob_pair(n_xyz, seed_for(1) if seed is None else seed, warp,
                     nblobs=40, disp_std_vox=3.0, noise_std=0.01)


BATCH_SIDES = (96, 112, 128, 144, 160)


def uneven_sizes(npairs: int = 48, seed: Optional[int] = None) -> list:
    """Per-pair (nx, ny, nz), each side i.i.d. uniform over BATCH_SIDES."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    return [tuple(int(v) for v in rng.choice(BATCH_SIDES, size=3)) for _ in range(npairs)]


def ct_pair(n: int, seed: Optional[int], warp: WarpFn,
            max_disp_vox: float = 6.0, coarse_spacing: int = 32) -> Pair:
    """CT-like fixed volume; moving = warp by a smooth coarse B-spline field."""
    seed = seed_for(2) if seed is None else seed
    rng = np.random.default_rng(seed)
    fixed = ellipsoid_volume(n, rng).astype(np.float32)
    nc = n_control(n, coarse_spacing)
    raw = rng.normal(0.0, 1.0, size=(3, nc, nc, nc))
    raw *= max_disp_vox / np.max(np.abs(raw))
    raw *= 2.0 / (n - 1)
    theta = raw.astype(np.float32)
    sp = (coarse_spacing,) * 3
    moving = np.ascontiguousarray(warp((n, n, n), sp, fixed, theta), dtype=np.float32)
    return Pair(fixed, moving, theta, (n, n, n), sp, seed)


def random_theta(n_xyz: Sequence[int], spacing: Sequence[int], std_vox: float,
                 seed: int) -> np.ndarray:
    """A random evaluation point (control grid), N(0, std_vox) voxels."""
    rng = np.random.default_rng(seed)
    return control_field(tuple(n_xyz), tuple(spacing), std_vox, rng).astype(np.float32)


def random_controls(n_xyz: Sequence[int], nc_xyz: Sequence[int], std_vox: float,
                    seed: int) -> np.ndarray:
    """Random control values on a grid of nc_xyz controls (given by the
    caller), N(0, std_vox) voxels in normalised units, [d][nc_z][nc_y][nc_x]."""
    rng = np.random.default_rng(seed)
    d = len(n_xyz)
    theta = rng.normal(0.0, std_vox, size=(d,) + tuple(reversed(tuple(nc_xyz))))
    for a in range(d):
        theta[a] *= 2.0 / (n_xyz[a] - 1)
    return theta.astype(np.float32)


def random_dense(n_xyz: Sequence[int], std_vox: float, seed: int) -> np.ndarray:
    """A random dense displacement [d][nz][ny][nx] in normalised units."""
    rng = np.random.default_rng(seed)
    d = len(n_xyz)
    u = rng.normal(0.0, std_vox, size=(d,) + tuple(reversed(n_xyz)))
    for a in range(d):
        u[a] *= 2.0 / (n_xyz[a] - 1)
    return u.astype(np.float32)


def smooth_dense(n_xyz: Sequence[int], std_vox: float, seed: int,
                 sigma: float = 4.0) -> np.ndarray:
    """A smooth random dense displacement (Gaussian-filtered noise)."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    d = len(n_xyz)
    shape = tuple(reversed(n_xyz))
    u = np.empty((d,) + shape, dtype=np.float64)
    for a in range(d):
        f = gaussian_filter(rng.normal(size=shape), sigma=sigma, mode="wrap")
        f *= std_vox / max(np.std(f), 1e-30)
        u[a] = f * 2.0 / (n_xyz[a] - 1)
    return u.astype(np.float32)
