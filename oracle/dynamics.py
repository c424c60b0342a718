"""Effective induction, LLG right-hand side and the two integrators.

* Induction (eq. Bi): b_i = sum of the unit vectors of the nearest-neighbour
  cells of i that belong to the disk, plus c (h_ext + H^M_i), c = a^2/lambda_ex^2.
  Cells outside the disk are absent, which gives the free boundary.
* Damped torque equation in dimensionless time (Sec. III.A):
  dm/dtau = m x b - alpha m x (m x b).
* RK4 (Sec. III.A): classical fourth-order Runge-Kutta with the full
  demagnetisation field evaluated at all four stages; stages are not
  normalised.
* Heun / H2 (Sec. III.C): with g = b dtau + sigma_s w and
  Delta(m) = m x [g - alpha (m x g)], the predictor is m~ = m + Delta(m) and the
  corrector m' = m + (Delta(m) + Delta~(m~))/2, where Delta~ uses b(m~) and the
  same noise vector w.
* A time-dependent external field enters b at each stage's own time: RK4 at
  tau_n, tau_n + dtau/2 (twice) and tau_n + dtau, Heun at tau_n (predictor)
  and tau_n + dtau (corrector), with tau_n = tau0 + n dtau.

Reading for the renormalisation, on which the paper is silent: when
``Params.renorm`` is set, |m| is reset to 1 after every full step (never at
intermediate stages).

Arrays are float64 tensors [..., 3, D, D]; outputs are zero outside the disk.
"""
from __future__ import annotations

import numpy as np
import torch

from .demag import demag_fft
from .geometry import Disk
from .philox import gaussian_field
from .units import Params


def exchange_field(m: torch.Tensor, disk: Disk) -> torch.Tensor:
    """Sum of nearest-neighbour unit vectors inside the disk."""
    mm = disk.apply_mask(m)
    b = torch.zeros_like(mm)
    b[..., 1:, :] += mm[..., :-1, :]
    b[..., :-1, :] += mm[..., 1:, :]
    b[..., :, 1:] += mm[..., :, :-1]
    b[..., :, :-1] += mm[..., :, 1:]
    return disk.apply_mask(b)


def _hext(prm: Params, like: torch.Tensor, tau: float | None) -> torch.Tensor:
    h = torch.tensor(prm.field_at(prm.tau0 if tau is None else tau), dtype=like.dtype)
    return h.view(3, 1, 1)


def effective_field(m: torch.Tensor, disk: Disk, prm: Params, H: torch.Tensor | None = None,
                    tau: float | None = None) -> torch.Tensor:
    """b = b_ex + c (h_ext(tau) + H^M) (eq. Bi); tau = None means prm.tau0."""
    if H is None:
        H = demag_fft(m, disk)
    b = exchange_field(m, disk) + prm.c * (_hext(prm, m, tau) + H)
    return disk.apply_mask(b)


def torque(m: torch.Tensor, b: torch.Tensor, alpha: float) -> torch.Tensor:
    """m x b - alpha m x (m x b), the right-hand side for a given induction."""
    mxb = torch.linalg.cross(m, b, dim=-3)
    return mxb - alpha * torch.linalg.cross(m, mxb, dim=-3)


def llg_rhs(m: torch.Tensor, disk: Disk, prm: Params, tau: float | None = None) -> torch.Tensor:
    """dm/dtau at state m and time tau (None: prm.tau0)."""
    mm = disk.apply_mask(m)
    return disk.apply_mask(torque(mm, effective_field(mm, disk, prm, tau=tau), prm.alpha))


def normalise(m: torch.Tensor, disk: Disk) -> torch.Tensor:
    n = torch.linalg.vector_norm(m, dim=-3, keepdim=True)
    n = torch.where(n > 0, n, torch.ones_like(n))
    return disk.apply_mask(m / n)


def rk4_step(m: torch.Tensor, disk: Disk, prm: Params, nsteps: int = 1) -> torch.Tensor:
    y = disk.apply_mask(m.to(torch.float64))
    h = prm.dtau
    for n in range(nsteps):
        t = prm.tau0 + n * float(h)          # the field is taken at each stage's own time
        k1 = llg_rhs(y, disk, prm, t)
        k2 = llg_rhs(y + 0.5 * h * k1, disk, prm, t + 0.5 * float(h))
        k3 = llg_rhs(y + 0.5 * h * k2, disk, prm, t + 0.5 * float(h))
        k4 = llg_rhs(y + h * k3, disk, prm, t + float(h))
        y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if prm.renorm:
            y = normalise(y, disk)
    return y


def heun_update(m: torch.Tensor, disk: Disk, prm: Params, w: torch.Tensor, tau: float | None = None) -> torch.Tensor:
    """One H2 step from m at time tau (None: prm.tau0) with the noise vector w
    (same shape as m); the predictor's field is taken at tau, the corrector's at
    tau + dtau."""
    sig = prm.sigma()
    t0 = prm.tau0 if tau is None else tau

    def delta(x, t):
        g = effective_field(x, disk, prm, tau=t) * prm.dtau + sig * w
        return disk.apply_mask(torque(x, g, prm.alpha))

    d1 = delta(m, t0)
    mt = m + d1
    d2 = delta(mt, t0 + float(prm.dtau))
    out = m + 0.5 * (d1 + d2)
    return normalise(out, disk) if prm.renorm else disk.apply_mask(out)


def heun_step(m: torch.Tensor, disk: Disk, prm: Params, *, seed: int, step0: int,
              replica: int = 0, nsteps: int = 1) -> torch.Tensor:
    """nsteps H2 steps; step n uses the Philox noise of time step step0 + n."""
    y = disk.apply_mask(m.to(torch.float64))
    for n in range(nsteps):
        w = torch.from_numpy(gaussian_field(seed, step0 + n, replica, disk.D))
        y = heun_update(y, disk, prm, w, prm.tau0 + n * float(prm.dtau))
    return y


def heun_step_replicas(m: torch.Tensor, disk: Disk, prm: Params, *, seed: int, step0: int,
                       replicas, nsteps: int = 1) -> torch.Tensor:
    """H2 steps for a batch of replicas m[r] (shape [B, 3, D, D])."""
    y = disk.apply_mask(m.to(torch.float64))
    reps = list(replicas)
    for n in range(nsteps):
        w = torch.from_numpy(gaussian_field(seed, step0 + n, np.asarray(reps), disk.D))
        y = heun_update(y, disk, prm, w, prm.tau0 + n * float(prm.dtau))
    return y
