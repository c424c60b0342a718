"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *draws* inputs: magnetisation fields, vortex start states and
ensemble geometries.  It holds none of the method's arithmetic (no kernels, no
fields, no integrators); both the HIP library and the FP64 oracle receive the
arrays it returns and apply their own disk mask.

Conventions shared by both sides of the parity tests (the paper's geometry,
Sec. II.A): a disk of radius R on a square grid of cell edge a is boxed in a
D x D array, D = 2R/a, stored component-major as ``[3][D][D]`` (x, y, z;
row index = y cell, column index = x cell).  Cell (iy, ix) has its centre at
x = ix - (D-1)/2, y = iy - (D-1)/2 in units of a, so the disk centre is the
origin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Permalloy as used throughout the paper (Sec. II.A, Sec. III.A): exchange
# stiffness A, saturation magnetisation Ms, electron gyromagnetic ratio gamma.
PERMALLOY = dict(A=13e-12, Ms=860e3, gamma=1.76e11)
CELL_NM = 2.0  # cell edge a = 2 nm (Sec. III.A)


def box_size(R_nm: float, a_nm: float = CELL_NM) -> int:
    """Number of cells across the disk, D = 2R/a (must be an integer)."""
    d = 2.0 * R_nm / a_nm
    D = int(round(d))
    if abs(d - D) > 1e-9 or D < 1:
        raise ValueError(f"2R/a = {d} is not a positive integer")
    return D


def cell_centres(D: int):
    """Cell-centre coordinates (x, y) in units of a, each of shape [D, D]."""
    c = np.arange(D, dtype=np.float64) - (D - 1) / 2.0
    y, x = np.meshgrid(c, c, indexing="ij")
    return x, y


def random_unit_field(D: int, seed: int) -> np.ndarray:
    """Isotropically random unit vectors, float64 [3, D, D]."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, D, D))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v


def smooth_random_field(D: int, seed: int, tilt: float = 0.3) -> np.ndarray:
    """A vortex-like curling field with a random smooth perturbation.

    Used where a physically smooth state is wanted (exchange-dominated
    dynamics stay well resolved); float64 [3, D, D] of unit vectors.
    """
    rng = np.random.default_rng(seed)
    x, y = cell_centres(D)
    k = rng.uniform(0.05, 0.25, size=(3, 2))
    ph = rng.uniform(0, 2 * np.pi, size=3)
    v = np.stack([-y, x, np.zeros_like(x)]) / (np.hypot(x, y) + 1.0)
    for c in range(3):
        v[c] += tilt * np.sin(k[c, 0] * x + k[c, 1] * y + ph[c])
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v


def vortex_ansatz(D: int, x0: float, y0: float, *, q: int = 1, chirality: int = 1,
                  polarity: int = 1, core_width: float = 2.5) -> np.ndarray:
    """Vortex start state centred at (x0, y0) (units of a), float64 [3, D, D].

    In-plane angle phi = q*atan2(y-y0, x-x0) + chirality*pi/2 (a curling
    vortex of vorticity q; Sec. IV, start-state equation, read so that q=+1
    winds once counter-clockwise), with a Gaussian out-of-plane core
    m_z = polarity*exp(-rho^2/(2 w^2)) of width w = core_width cells and the
    in-plane part scaled to keep |m| = 1.
    """
    x, y = cell_centres(D)
    dx, dy = x - x0, y - y0
    phi = q * np.arctan2(dy, dx) + chirality * np.pi / 2.0
    mz = polarity * np.exp(-(dx * dx + dy * dy) / (2.0 * core_width ** 2))
    s = np.sqrt(np.clip(1.0 - mz * mz, 0.0, 1.0))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mz])


@dataclass
class EnsembleDisk:
    R_nm: float
    L_nm: float
    x0_nm: float
    y0_nm: float


def ragged_ensemble(n: int = 256, seed: int = 12072192, a_nm: float = CELL_NM):
    """Ragged ensemble of disks: R uniform on {30, 40, ..., 120} nm, L/R uniform
    in [0.05, 0.3], vortex offset radius uniform in [2, 15] nm at a uniform
    random angle.  Thickness is rounded to 0.01 nm."""
    rng = np.random.default_rng(seed)
    radii = rng.choice(np.arange(30, 121, 10), size=n).astype(np.float64)
    lor = rng.uniform(0.05, 0.3, size=n)
    off = rng.uniform(2.0, 15.0, size=n)
    ang = rng.uniform(0.0, 2 * np.pi, size=n)
    out = []
    for R, f, r, t in zip(radii, lor, off, ang):
        out.append(EnsembleDisk(float(R), float(round(R * f, 2)),
                                float(r * math.cos(t)), float(r * math.sin(t))))
    return out
