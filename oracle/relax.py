"""Lagrange-constrained alignment relaxation, k_F fit and the Thiele frequency
(paper Sec. IV and Sec. IV.B).

Alignment relaxation (Sec. IV): every cell vector is aligned with its local
induction and the sweep is repeated until nothing changes; a fictitious field
that enters through a Lagrange multiplier holds the vortex at a chosen X.

Readings (the constraint form sits in a reference the paper does not restate):
* constraint  C(m) = sum_{|r_i - X| < r_cut} (m_z,i)^2 (r_i - X) = 0  (two
  equations: the m_z^2-weighted centroid of the cells within r_cut of X sits
  at X — the core-position definition of Sec. IV with its 4 lambda_ex cutoff
  centred on the target); r_cut = None takes the whole disk, which in large
  disks lets the constraint be met by out-of-plane tails far from the core
  instead of by moving the core;
* stationarity of E - lambda.C gives the fictitious field
  b^lam_i = 2 m_z,i (lambda . (r_i - X)) z-hat added to b_i (b = -dE/dm);
* sweep: all cells at once, m_i <- (b_i + b^lam_i + kappa m_i) / |...|; the
  kappa m_i term (kappa > 0) damps the checkerboard mode that simultaneous
  alignment would otherwise leave undamped and does not move the fixed point
  (m_i parallel to b_i + b^lam_i);
* after each sweep lambda takes one Newton step on C(m_new), with the
  Jacobian of the aligned state with respect to lambda at fixed induction,
  J = sum_i 4 m_z,i^2 (1 - m_z,i^2)/|t_i| (r_i - X)(r_i - X)^T;
* converged when max_i |m_i x (b_i + b^lam_i)| and |C| are both below tol.
U(X) is the energy of eq. Hmm of the relaxed state (the constraint field
does no work there).

k_F (eq. Ux, Sec. IV.B): least squares of U(r) - U(0) = kt r^2/2 + k4 r^4/4 over
relaxed states, with r the core position of each relaxed state in units of a
and energies in J; then the Thiele frequency (eqs. wG, OG) in simulation units
is Omega(r) = -Q U'(r)/(2 pi r) = -Q (kt + k4 r^2)/(2 pi).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .dynamics import effective_field, normalise
from .geometry import Disk
from .observables import vortex_core_position
from .units import Params


def constraint_terms(m: torch.Tensor, disk: Disk, X_nm, cutoff_nm=None):
    """(dx, dy) of every cell from X in units of a (zero outside the disk and
    outside the cutoff circle around X) and C(m)."""
    a = disk.a_nm
    dx = disk.x - X_nm[0] / a
    dy = disk.y - X_nm[1] / a
    M = disk.mask
    if cutoff_nm is not None:
        M = M & (dx * dx + dy * dy < (cutoff_nm / a) ** 2)
    M = M.to(torch.float64)
    dx = dx * M
    dy = dy * M
    w = m[2] ** 2
    return dx, dy, torch.stack([(w * dx).sum(), (w * dy).sum()])


def relax(m0: torch.Tensor, disk: Disk, prm: Params, X_nm, *, kappa: float = 2.0, tol: float = 1e-9,
          max_sweeps: int = 100000, cutoff_nm=None):
    """Constrained alignment relaxation from m0.  Returns (m, lambda, sweeps, residual, C)."""
    m = normalise(disk.apply_mask(m0.to(torch.float64)), disk)
    dx, dy, _ = constraint_terms(m, disk, X_nm, cutoff_nm)
    lam = torch.zeros(2, dtype=torch.float64)
    res, C = float("inf"), None
    for it in range(max_sweeps):
        b = effective_field(m, disk, prm)
        bl = torch.zeros_like(m)
        bl[2] = 2.0 * m[2] * (lam[0] * dx + lam[1] * dy)
        tot = b + bl
        res = float(torch.linalg.vector_norm(torch.linalg.cross(m, tot, dim=0), dim=0).max())
        _, _, C = constraint_terms(m, disk, X_nm, cutoff_nm)
        if res < tol and float(C.abs().max()) < tol:
            return m, lam, it, res, C
        t = tot + kappa * m
        tn = torch.linalg.vector_norm(t, dim=0)
        tn = torch.where(tn > 0, tn, torch.ones_like(tn))
        mn = disk.apply_mask(t / tn)
        _, _, Cn = constraint_terms(mn, disk, X_nm, cutoff_nm)
        g = 4.0 * mn[2] ** 2 * (1.0 - mn[2] ** 2) / tn
        J = torch.stack([torch.stack([(g * dx * dx).sum(), (g * dx * dy).sum()]),
                         torch.stack([(g * dx * dy).sum(), (g * dy * dy).sum()])])
        if float(torch.linalg.det(J).abs()) > 0:
            lam = lam - torch.linalg.solve(J, Cn)
        m = mn
    return m, lam, max_sweeps, res, C


def fit_kF(r_cells, dU):
    """(kt, k4) from U(r) - U(0) = kt r^2/2 + k4 r^4/4 (least squares); r in a, U in J."""
    r = np.asarray(r_cells, dtype=np.float64)
    A = np.stack([0.5 * r ** 2, 0.25 * r ** 4], axis=1)
    kt, k4 = np.linalg.lstsq(A, np.asarray(dU, dtype=np.float64), rcond=None)[0]
    return float(kt), float(k4)


def thiele_omega(kt: float, k4: float, r_cells: float, Q: int = 1) -> float:
    """Omega(r) = -Q U'(r)/(2 pi r) in units of 1/t0."""
    return -Q * (kt + k4 * r_cells ** 2) / (2.0 * math.pi)


def static_potential(disk: Disk, prm: Params, X_list_nm, make_start, lambda_ex_nm: float, **kw):
    """Relax at each X (nm, along x; constraint cutoff 4 lambda_ex unless given)
    and return (r_c in a, U in J, states)."""
    from .observables import energy
    kw.setdefault("cutoff_nm", 4.0 * lambda_ex_nm)
    rs, Us, states = [], [], []
    for X in X_list_nm:
        m, lam, it, res, C = relax(make_start(X), disk, prm, (X, 0.0), **kw)
        xc, yc, *_ = vortex_core_position(m, disk, lambda_ex_nm)
        rs.append(math.hypot(xc, yc) / disk.a_nm)
        Us.append(energy(m, disk, prm)[0])
        states.append(m)
    return np.array(rs), np.array(Us), states
