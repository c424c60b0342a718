"""Disk geometry on the square grid (paper Sec. II.A and the FFT padding of Sec. II.B).

Reading used here: D = 2R/a cells across the disk; cell (iy, ix) has its centre
at (ix-(D-1)/2, iy-(D-1)/2) in units of a and belongs to the disk when that
centre lies inside or on the circle of radius D/2.  The padded FFT size is the
smallest power of two P >= 2D, which is at least 2D-1 and so makes the
circular convolution equal to the linear one (no interaction with images).
"""
from __future__ import annotations

import math

import torch


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


class Disk:
    """A disk of radius R and thickness L on cells of edge a (all in nm)."""

    def __init__(self, R_nm: float, L_nm: float, a_nm: float = 2.0, P: int | None = None):
        d = 2.0 * R_nm / a_nm
        D = int(round(d))
        if abs(d - D) > 1e-9 or D < 1:
            raise ValueError(f"2R/a = {d} must be a positive integer")
        if L_nm <= 0 or a_nm <= 0:
            raise ValueError("L and a must be positive")
        self.R_nm, self.L_nm, self.a_nm = float(R_nm), float(L_nm), float(a_nm)
        self.D = D
        self.ell = L_nm / a_nm                      # thickness in units of a
        self.P = next_pow2(2 * D) if P is None else int(P)
        if self.P < 2 * D - 1:
            raise ValueError(f"P = {self.P} < 2D-1 = {2 * D - 1}: convolution would wrap")
        c = torch.arange(D, dtype=torch.float64) - (D - 1) / 2.0
        self.y, self.x = torch.meshgrid(c, c, indexing="ij")   # [D, D] each
        self.mask = (self.x ** 2 + self.y ** 2) <= (D / 2.0) ** 2
        self.n_cells = int(self.mask.sum())

    def apply_mask(self, m: torch.Tensor) -> torch.Tensor:
        """Zero every component outside the disk (last two dims are [D, D])."""
        return m * self.mask.to(m.dtype)

    def __repr__(self):
        return f"Disk(R={self.R_nm} nm, L={self.L_nm} nm, a={self.a_nm} nm, D={self.D}, P={self.P}, N={self.n_cells})"
