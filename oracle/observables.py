"""Observables: energy (eq. Hmm), spatial average <m> and the vortex core position (Sec. IV).

Energy in units of J = 2AL (eq. Hmm):
  E = -[ sum over nearest-neighbour pairs (i,j) of m_i.m_j
         + c sum_i (h_ext + H^M_i / 2).m_i ],
returned with its three parts (exchange, demagnetisation, external).

Core position (Sec. IV): the vorticity centre r_v is the shared corner of a
2 x 2 plaquette of disk cells around which the in-plane angle phi winds by
+2 pi; the core position is the m_z^2-weighted mean of the cell positions
within 4 lambda_ex of r_v:
  r_c = sum_{|r_i - r_v| < 4 lambda_ex} (m_z,i)^2 r_i / sum (m_z,i)^2.
Readings where the paper is silent: the plaquette winding is the sum of the
four counter-clockwise angle differences, each wrapped into [-pi, pi), over
2 pi and rounded; when several plaquettes wind by +1 the one nearest a given
hint (the previous core position) is taken, else the one whose four cells
carry the largest sum of m_z^2, ties going to the lowest (row, column); when
none winds by +1 the flag is 0, r_v is NaN and r_c is the m_z^2-weighted mean
over the whole disk.  The cutoff is strict.  Positions are in nm.
"""
from __future__ import annotations

import math

import torch

from .demag import demag_fft
from .dynamics import exchange_field
from .geometry import Disk
from .units import Params


def energy(m: torch.Tensor, disk: Disk, prm: Params):
    """(E, E_ex, E_demag, E_ext) in units of J for a single state [3, D, D]."""
    mm = disk.apply_mask(m.to(torch.float64))
    mask = disk.mask
    # nearest-neighbour bonds with both cells in the disk, each counted once
    hb = (mask[:, :-1] & mask[:, 1:])
    vb = (mask[:-1, :] & mask[1:, :])
    dot_h = (mm[:, :, :-1] * mm[:, :, 1:]).sum(0)
    dot_v = (mm[:, :-1, :] * mm[:, 1:, :]).sum(0)
    e_ex = -(dot_h[hb].sum() + dot_v[vb].sum())
    H = demag_fft(mm, disk)
    e_dm = -0.5 * prm.c * (H * mm).sum()
    h = torch.tensor(prm.field_at(prm.tau0), dtype=torch.float64).view(3, 1, 1)
    e_ext = -prm.c * (h * mm).sum()
    e = e_ex + e_dm + e_ext
    return float(e), float(e_ex), float(e_dm), float(e_ext)


def energy_from_exchange_field(m: torch.Tensor, disk: Disk, prm: Params) -> float:
    """Same total energy written with b_ex: -(1/2) sum m.b_ex - c sum (h + H/2).m."""
    mm = disk.apply_mask(m.to(torch.float64))
    H = demag_fft(mm, disk)
    h = torch.tensor(prm.field_at(prm.tau0), dtype=torch.float64).view(3, 1, 1)
    return float(-0.5 * (mm * exchange_field(mm, disk)).sum() - prm.c * ((h + 0.5 * H) * mm).sum())


def mean_m(m: torch.Tensor, disk: Disk):
    mm = disk.apply_mask(m.to(torch.float64))
    return tuple(float(mm[c][disk.mask].mean()) for c in range(3))


def _wrap(d: torch.Tensor) -> torch.Tensor:
    return torch.remainder(d + math.pi, 2 * math.pi) - math.pi


def plaquette_windings(m: torch.Tensor, disk: Disk) -> torch.Tensor:
    """Winding number of every 2x2 plaquette [D-1, D-1]; 0 where a corner is outside the disk.

    Plaquette (j, i) has corners (j,i), (j,i+1), (j+1,i+1), (j+1,i) traversed
    counter-clockwise (x grows with the column, y with the row).
    """
    mm = m.to(torch.float64)
    phi = torch.atan2(mm[1], mm[0])
    a = phi[:-1, :-1]
    b = phi[:-1, 1:]
    c = phi[1:, 1:]
    d = phi[1:, :-1]
    s = _wrap(b - a) + _wrap(c - b) + _wrap(d - c) + _wrap(a - d)
    wnd = torch.round(s / (2 * math.pi)).to(torch.int64)
    M = disk.mask
    ok = M[:-1, :-1] & M[:-1, 1:] & M[1:, 1:] & M[1:, :-1]
    return torch.where(ok, wnd, torch.zeros_like(wnd))


def vortex_core_position(m: torch.Tensor, disk: Disk, lambda_ex_nm: float, hint_nm=None):
    """(x_c, y_c, x_v, y_v, n_plus) with positions in nm; n_plus = number of +1 plaquettes."""
    mm = disk.apply_mask(m.to(torch.float64))
    a = disk.a_nm
    wnd = plaquette_windings(mm, disk)
    jj, ii = torch.nonzero(wnd == 1, as_tuple=True)
    n_plus = int(jj.numel())
    x, y = disk.x, disk.y
    mz2 = mm[2] ** 2 * disk.mask.to(torch.float64)
    if n_plus == 0:
        wsum = mz2.sum()
        xc = float((mz2 * x).sum() / wsum) * a
        yc = float((mz2 * y).sum() / wsum) * a
        return xc, yc, float("nan"), float("nan"), 0
    cx = x[0, ii] + 0.5          # plaquette corner = mean of its four cell centres
    cy = y[jj, 0] + 0.5
    if hint_nm is not None:
        score = -((cx - hint_nm[0] / a) ** 2 + (cy - hint_nm[1] / a) ** 2)
    else:
        score = mz2[jj, ii] + mz2[jj, ii + 1] + mz2[jj + 1, ii + 1] + mz2[jj + 1, ii]
    best = score.max()
    k = int(torch.nonzero(score == best)[0])      # lowest (row, column) among ties
    xv, yv = float(cx[k]), float(cy[k])
    cutoff = 4.0 * lambda_ex_nm / a
    near = ((x - xv) ** 2 + (y - yv) ** 2 < cutoff * cutoff) & disk.mask
    w = mz2 * near.to(torch.float64)
    ws = w.sum()
    xc = float((w * x).sum() / ws) * a
    yc = float((w * y).sum() / ws) * a
    return xc, yc, xv * a, yv * a, n_plus


def core_centroid(m: torch.Tensor, disk: Disk, lambda_ex_nm: float, xv_nm: float, yv_nm: float,
                  found: bool = True) -> torch.Tensor:
    """r_c (nm) as a differentiable function of m with the plaquette r_v and the
    cutoff set held fixed (the smooth part of the core-position definition);
    used to differentiate trajectory losses."""
    a = disk.a_nm
    mz2 = disk.apply_mask(m)[2] ** 2
    if found:
        cutoff = 4.0 * lambda_ex_nm / a
        near = ((disk.x - xv_nm / a) ** 2 + (disk.y - yv_nm / a) ** 2 < cutoff * cutoff) & disk.mask
    else:
        near = disk.mask
    w = mz2 * near.to(m.dtype)
    ws = w.sum()
    return torch.stack([(w * disk.x).sum() / ws * a, (w * disk.y).sum() / ws * a])
