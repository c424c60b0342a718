"""Collective-coordinate relations of the vortex (paper Sec. IV, Sec. IV.B, Sec. V.C, Sec. VI).

* Gyrovector G = 2 pi Q m0/gamma with m0 = L Ms and Q = q p (Sec. IV).
* Thiele frequency omega_G = -k_F/G (eq. wG) and its dimensionless form
  Omega_G = omega_G t0 = -k_F a^2/(4 pi L A Q) (eq. OG).
* Harmonic potential U(X) = U(0) + k_F X^2/2 (eq. Ux).  In simulation units,
  with energies in J = 2AL and lengths in a, U/J = U0/J + (kt/2) (X/a)^2 with
  kt = k_F a^2/(2 A L); then Omega_G = -Q kt/(2 pi).
* Equipartition <r^2> = 2 kT/k_F (eq. r2); radial density p(r) =
  beta k_F r exp(-beta k_F r^2/2) (eq. pr) with peak at r_max = sqrt(kT/k_F)
  and p(r_max) = exp(-1/2)/r_max; speed density
  f(V) = beta m_G V exp(-beta m_G V^2/2) with m_G = G^2/k_F (Sec. VI).
* Linear law k_F ~ (1/4)(L^2/R)(A/a^2) (eq. kFlinear).

All functions are SI unless the name says otherwise.
"""
from __future__ import annotations

import math

from .units import MU0, Material


def gyrovector(mat: Material, L_m: float, Q: int = 1) -> float:
    """G = 2 pi Q L Ms / gamma (kg/s)."""
    return 2.0 * math.pi * Q * L_m * mat.Ms / mat.gamma


def omega_thiele(kF: float, mat: Material, L_m: float, Q: int = 1) -> float:
    """omega_G = -k_F/G (rad/s)."""
    return -kF / gyrovector(mat, L_m, Q)


def Omega_dimensionless(kF: float, mat: Material, a_m: float, L_m: float, Q: int = 1) -> float:
    """Omega_G = -k_F a^2/(4 pi L A Q)."""
    return -kF * a_m * a_m / (4.0 * math.pi * L_m * mat.A * Q)


def kt_from_kF(kF: float, mat: Material, a_m: float, L_m: float) -> float:
    """Curvature of U/J against (X/a)^2: kt = k_F a^2/(2 A L)."""
    return kF * a_m * a_m / (2.0 * mat.A * L_m)


def Omega_from_kt(kt: float, Q: int = 1) -> float:
    """Omega_G = -Q kt/(2 pi) in simulation units."""
    return -Q * kt / (2.0 * math.pi)


def kF_linear(mat: Material, a_m: float, L_m: float, R_m: float) -> float:
    """k_F ~ (1/4)(L^2/R)(A/a^2) (N/m)."""
    return 0.25 * L_m * L_m / R_m * mat.A / (a_m * a_m)


def r_rms(kT: float, kF: float) -> float:
    """sqrt(<r^2>) = sqrt(2 kT/k_F)."""
    return math.sqrt(2.0 * kT / kF)


def p_radial(r, kT: float, kF: float):
    """Boltzmann radial density beta k_F r exp(-beta k_F r^2/2)."""
    beta = 1.0 / kT
    return beta * kF * r * math.e ** (-0.5 * beta * kF * r * r)


def gyro_mass(mat: Material, L_m: float, kF: float, Q: int = 1) -> float:
    """m_G = G^2/k_F (kg)."""
    G = gyrovector(mat, L_m, Q)
    return G * G / kF


def gyro_mass_linear(mat: Material, R_m: float, a_m: float) -> float:
    """m_G with the linear k_F law: (2 pi)^2 R/(coef mu0 gamma^2), coef = lambda_ex^2/(8 a^2)."""
    lam2 = 2.0 * mat.A / (MU0 * mat.Ms ** 2)
    coef = lam2 / (8.0 * a_m * a_m)
    return (2.0 * math.pi) ** 2 / coef * R_m / (MU0 * mat.gamma ** 2)
