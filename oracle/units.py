"""Unit system of the simulation (paper Sec. II.A and Sec. III.A-B).

Energies are in units of J = 2AL (exchange energy between two cells, eq. for
H_ex), fields in units of Ms, the induction in units of B0 = 2A/(a^2 Ms), time
in units of t0 = 1/(gamma B0) and temperature as the scaled temperature
T_s = kT/J (Sec. III.B).  The coupling of demagnetisation and external fields
to the cell moments carries the factor c = a^2/lambda_ex^2 with the exchange
length lambda_ex = sqrt(2A/(mu0 Ms^2)) (eq. Hmm, eq. Bi).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

MU0 = 4e-7 * math.pi          # vacuum permeability (T m / A)
KB = 1.380649e-23             # Boltzmann constant (J / K)


@dataclass(frozen=True)
class Material:
    A: float = 13e-12          # exchange stiffness, J/m
    Ms: float = 860e3          # saturation magnetisation, A/m
    gamma: float = 1.76e11     # gyromagnetic ratio, 1/(T s)


@dataclass
class Params:
    """Dimensionless integration parameters.

    alpha     Gilbert damping.
    c         a^2/lambda_ex^2, multiplies the demag and external fields in b.
    hext      external field over Ms (3 numbers).
    temp      scaled temperature kT/(2AL).
    dtau      time step in units of t0.
    renorm    renormalise |m| = 1 after every full step.
    fd_factor divide the noise variance by (1 + alpha^2) (off = the paper's
              sigma^2 = 2 alpha T dtau).

    Time-dependent external field (the h_ext of eq. Hmm and eq. Bi as a function
    of time, a reading: the paper keeps it constant):
      h_ext(tau) = hext + hac sin(2 pi freq tau + phase)
                        + hpulse exp(-(tau - tpulse)^2 / (2 wpulse^2)),
    tau0 = the time at the first step of an integration call.
    """
    alpha: float = 0.0
    c: float = 0.0
    hext: tuple = (0.0, 0.0, 0.0)
    temp: float = 0.0
    dtau: float = 0.04
    renorm: bool = False
    fd_factor: bool = False
    hac: tuple = (0.0, 0.0, 0.0)
    freq: float = 0.0
    phase: float = 0.0
    hpulse: tuple = (0.0, 0.0, 0.0)
    tpulse: float = 0.0
    wpulse: float = 1.0
    tau0: float = 0.0

    def field_at(self, tau: float) -> tuple:
        """h_ext at time tau (3 floats)."""
        osc = math.sin(2.0 * math.pi * self.freq * tau + self.phase)
        pulse = math.exp(-((tau - self.tpulse) ** 2) / (2.0 * self.wpulse ** 2)) if any(self.hpulse) else 0.0
        return tuple(float(self.hext[i]) + float(self.hac[i]) * osc + float(self.hpulse[i]) * pulse
                     for i in range(3))

    def sigma(self) -> float:
        """Standard deviation of one noise component per step,
        sigma_s = sqrt(2 alpha T dtau) (Sec. III.C), optionally over (1+alpha^2)."""
        var = 2.0 * self.alpha * self.temp * self.dtau
        if self.fd_factor:
            var = var / (1.0 + self.alpha ** 2)
        # a tensor alpha keeps the autograd graph (gradients through the noise amplitude)
        return var.sqrt() if hasattr(var, "sqrt") else math.sqrt(var)


def exchange_length(mat: Material) -> float:
    """lambda_ex = sqrt(2A/(mu0 Ms^2)) in metres (Sec. II.A)."""
    return math.sqrt(2.0 * mat.A / (MU0 * mat.Ms ** 2))


def dimensionless(mat: Material, a_nm: float, L_nm: float, *, dt_ps: float | None = None,
                  T_K: float = 0.0) -> dict:
    """All derived quantities for cell edge a and thickness L.

    Returns lambda_ex (nm), c = a^2/lambda_ex^2, B0 (T), t0 (ps), f0 = gamma B0
    (1/s), J (J), the scaled temperature kT/J and, if dt_ps is given,
    dtau = dt/t0.
    """
    a = a_nm * 1e-9
    L = L_nm * 1e-9
    lam = exchange_length(mat)
    B0 = 2.0 * mat.A / (a * a * mat.Ms)
    t0 = 1.0 / (mat.gamma * B0)
    J = 2.0 * mat.A * L
    out = dict(lambda_ex_nm=lam * 1e9, c=(a / lam) ** 2, B0=B0, t0_ps=t0 * 1e12,
               f0=mat.gamma * B0, J=J, temp=KB * T_K / J, mu0Ms=MU0 * mat.Ms)
    if dt_ps is not None:
        out["dtau"] = dt_ps / (t0 * 1e12)
    return out
