"""Thin-film Green's kernels (paper Sec. II.B).

With lengths in units of the cell edge a, the cell sum that replaces the
integral over d^2r' carries no extra factor, and the field of cell j at cell i
is H_alpha(i) = sum_beta K_alpha,beta(r_i - r_j) m_beta(j), where for a
displacement (u, v) != 0 with r = |(u, v)|, s = sqrt(r^2 + l^2), l = L/a:

  K_zz = (1/(2 pi l)) (1/s - 1/r)                 (z-summed source, z-averaged observer)
  K_xx = (l/(2 pi r^4)) (u^2/s - v^2/(s + r))
  K_yy = K_xx with u and v swapped
  K_xy = K_yx = (l/(2 pi r^4)) ((2s + r)/(s + r)) (u v / s)
  K_xz = K_yz = 0

and at zero displacement the self terms of a cylinder of radius r_o = 1/sqrt(pi)
(the circle of the cell's area):

  K_zz(0) = -N_z = -(l + r_o - sqrt(l^2 + r_o^2))/l
  K_xx(0) = K_yy(0) = -N_x,  N_x = (sqrt(l^2 + r_o^2) - r_o)/(2 l),  K_xy(0) = 0.

Reading: the printed transverse self term carries a positive sign, which
contradicts N_x + N_y + N_z = 1 stated right after it and the limit N_x -> 1/2
for long cells; the negative sign is used.  K_zz is evaluated in the
algebraically equal cancellation-free form -l/(2 pi r s (s + r)).
"""
from __future__ import annotations

import math

import torch


def self_factors(ell: float):
    """(N_x, N_z) of the cell cylinder of radius 1/sqrt(pi) and length ell."""
    ro = 1.0 / math.sqrt(math.pi)
    so = math.sqrt(ell * ell + ro * ro)
    Nz = (ell + ro - so) / ell
    Nx = (so - ro) / (2.0 * ell)
    return Nx, Nz


def kernels(u: torch.Tensor, v: torch.Tensor, ell: float):
    """Kernel values (Kxx, Kyy, Kxy, Kzz) at integer displacements (u, v).

    u, v: float64 tensors of equal shape; entries with u = v = 0 get the self
    terms.
    """
    u = u.to(torch.float64)
    v = v.to(torch.float64)
    r2 = u * u + v * v
    zero = r2 == 0
    r2s = torch.where(zero, torch.ones_like(r2), r2)     # avoid 0/0 at the origin
    r = torch.sqrt(r2s)
    s = torch.sqrt(r2s + ell * ell)
    pre = ell / (2.0 * math.pi * r2s * r2s)
    Kxx = pre * (u * u / s - v * v / (s + r))
    Kyy = pre * (v * v / s - u * u / (s + r))
    Kxy = pre * ((2.0 * s + r) / (s + r)) * (u * v / s)
    Kzz = -ell / (2.0 * math.pi * r * s * (s + r))
    Nx, Nz = self_factors(ell)
    Kxx = torch.where(zero, torch.full_like(Kxx, -Nx), Kxx)
    Kyy = torch.where(zero, torch.full_like(Kyy, -Nx), Kyy)
    Kxy = torch.where(zero, torch.zeros_like(Kxy), Kxy)
    Kzz = torch.where(zero, torch.full_like(Kzz, -Nz), Kzz)
    return Kxx, Kyy, Kxy, Kzz


def kzz_unsimplified(u: torch.Tensor, v: torch.Tensor, ell: float) -> torch.Tensor:
    """K_zz as printed, (1/(2 pi l))(1/s - 1/r), for r > 0 only (test helper)."""
    r = torch.sqrt(u.double() ** 2 + v.double() ** 2)
    s = torch.sqrt(r * r + ell * ell)
    return (1.0 / (2.0 * math.pi * ell)) * (1.0 / s - 1.0 / r)
